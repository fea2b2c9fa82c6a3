// project.hip -- per-surfel projection and culling, per-tile pair counts and emission.
//
// Projection (per surfel; a workgroup per CU over a range of surfels): activations
// (normalised q, s = exp(s~) per Sec. 3.3, alpha = sigmoid), world -> sensor transform, the
// 64-byte record of lgsr_internal.h, and a conservative ray rectangle of the hit disk
// u^2 + v^2 <= k^2 (bounds along the centre, elevation and azimuth directions; see
// project_one): an elevation interval (rows, by binary search of the monotone row table) and
// an azimuth interval (columns, uniform, wrapping at 360 degrees), or whole rows of azimuth
// when a pole may lie inside.
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

// Angular safety margin of the culling cone (radians): far above float32 rounding of
// the angles involved, far below one beam spacing.
constexpr float kAngMargin = 2e-4f;
// Relative inflation of the disk's extents: covers float32 rounding of the frame and scales.
constexpr float kExtSlack = 1e-4f;
constexpr float kTwoPi = 6.28318530717958648f;

// Tile-column segments [a0, a1] and [b0, b1] (b1 < b0: empty) covered by columns
// c0 .. c0 + cw - 1 modulo W.
__device__ __forceinline__ void col_segments(int c0, int cw, int W, int TW, int &a0, int &a1, int &b0, int &b1)
{
    b0 = 1;
    b1 = 0;
    if (cw >= W) {
        a0 = 0;
        a1 = TW - 1;
        return;
    }
    int end = c0 + cw - 1;
    if (end < W) {
        a0 = c0 / kTile;
        a1 = end / kTile;
        return;
    }
    a0 = c0 / kTile;
    a1 = TW - 1;
    int bh = (end - W) / kTile;
    if (bh >= a0) {
        a0 = 0;
        a1 = TW - 1;
    } else {
        b0 = 0;
        b1 = bh;
    }
}

// first k in [0, H) with rows_sin[k] <= x (rows strictly decreasing); H if none
__device__ __forceinline__ int first_row_le(const float *__restrict__ rows, int stride, int H, float x)
{
    int lo = 0, hi = H;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (rows[stride * mid] <= x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// first k in [0, H) with rows_sin[k] < x; H if none
__device__ __forceinline__ int first_row_lt(const float *__restrict__ rows, int stride, int H, float x)
{
    int lo = 0, hi = H;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (rows[stride * mid] < x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Tiles met by a ray rectangle (rows r0..r1, columns c0 .. c0 + cw - 1 modulo W): tile rows
// tr0 .. tr0 + rows - 1, and in each the tile columns a0 .. a0 + na - 1 followed by
// b0 .. b0 + nb - 1; n tiles in all.
struct TileSpan {
    int tr0, a0, na, b0, nb, n;
};

__device__ __forceinline__ TileSpan tile_span(uint2 rc, const Grid &g)
{
    TileSpan s{0, 0, 0, 0, 0, 0};
    const int r0 = (int)(rc.x & 0xFFFFu), r1 = (int)(rc.x >> 16);
    const int c0 = (int)(rc.y & 0xFFFFu), cw = (int)(rc.y >> 16);
    if (cw <= 0 || r1 < r0) return s;
    int a0, a1, b0, b1;
    col_segments(c0, cw, g.W, g.TW, a0, a1, b0, b1);
    s.tr0 = r0 / kTile;
    s.a0 = a0;
    s.na = a1 - a0 + 1;
    s.b0 = b0;
    s.nb = b1 >= b0 ? b1 - b0 + 1 : 0;
    s.n = (r1 / kTile - s.tr0 + 1) * (s.na + s.nb);
    return s;
}

__device__ __forceinline__ int span_tile(const TileSpan &s, int k, int TH)
{
    const int w = s.na + s.nb;
    const int row = k / w, j = k - row * w;
    return tile_id(s.tr0 + row, j < s.na ? s.a0 + j : s.b0 + (j - s.na), TH);
}

// A lane walks the tiles of its own rectangle when there are at most this many; the tiles
// of a larger rectangle are shared out over the wave's 64 lanes.
constexpr int kOwnTiles = 8;

// Calls f(tile, v) for every tile met by each lane's ray rectangle rc, v being the value
// the rectangle's lane passed.  Every lane of the wavefront must call it (lanes with
// nothing to enumerate pass an empty rectangle).  A rectangle around the sensor meets every
// tile of the grid; walked by its own lane alone it would hold the whole wave for hundreds
// of serial steps, so rectangles of more than kOwnTiles tiles are taken one at a time by
// the whole wave, a tile per lane.  Projection (counting) and emission (writing) both
// enumerate with it; the order of the calls is of no consequence to either.
template <class F>
__device__ __forceinline__ void for_each_tile(uint2 rc, uint32_t v, const Grid &g, F &&f)
{
    const TileSpan s = tile_span(rc, g);
    const bool wide = s.n > kOwnTiles;
    if (!wide && s.n > 0) {
        const int rows = s.n / (s.na + s.nb);
        for (int r = 0; r < rows; ++r) {
            for (int j = 0; j < s.na; ++j) f(tile_id(s.tr0 + r, s.a0 + j, g.TH), v);
            for (int j = 0; j < s.nb; ++j) f(tile_id(s.tr0 + r, s.b0 + j, g.TH), v);
        }
    }
    uint64_t wm = __ballot(wide);
    const int lane = (int)(threadIdx.x & 63u);
    while (wm) {
        const int src = __builtin_ctzll(wm);
        wm &= wm - 1ull;
        TileSpan w;
        w.tr0 = __builtin_amdgcn_readlane(s.tr0, src);
        w.a0 = __builtin_amdgcn_readlane(s.a0, src);
        w.na = __builtin_amdgcn_readlane(s.na, src);
        w.b0 = __builtin_amdgcn_readlane(s.b0, src);
        w.nb = __builtin_amdgcn_readlane(s.nb, src);
        w.n = __builtin_amdgcn_readlane(s.n, src);
        const uint32_t wv = (uint32_t)__builtin_amdgcn_readlane((int)v, src);
        for (int k = lane; k < w.n; k += 64) f(span_tile(w, k, g.TH), wv);
    }
}

// Grids with at most this many tiles count and reserve pairs in LDS per workgroup.
constexpr int kLdsBins = 4096;
constexpr int kLdsRows = 4096;  // row tables up to this many rows are searched in LDS

// Record, range key and ray rectangle of surfel i; (0, 0) when it cannot be hit.
__device__ __forceinline__ uint2 project_one(const SurfelPtrs &S, const Pose &P, const float *__restrict__ rows,
                                             int rstride, const Grid &g, const RasterParams &p,
                                             float *__restrict__ recs, uint32_t *__restrict__ keys, int64_t i)
{
    Geom gm = project_geom(S.means, S.quats, S.log_scales, S.logits, i, P, p.near);
    if (!gm.valid) {
        keys[i] = kCulledKey;
        return make_uint2(0u, 0u);
    }
    float rec[kRec];
    make_record(gm, rec);
    float4 *dst = reinterpret_cast<float4 *>(recs + (size_t)i * kRec);
    dst[0] = make_float4(rec[0], rec[1], rec[2], rec[3]);
    dst[1] = make_float4(rec[4], rec[5], rec[6], rec[7]);
    dst[2] = make_float4(rec[8], rec[9], rec[10], rec[11]);
    dst[3] = make_float4(rec[12], rec[13], rec[14], rec[15]);
    keys[i] = __float_as_uint(gm.r);

    // Conservative ray rectangle of the hit region: the disk u^2 + v^2 <= k^2, i.e. the
    // points p = mu' + delta, delta = x a' + y b' with (x / s0)^2 + (y / s1)^2 <= k^2.  Along
    // a unit vector e, |delta . e| <= ext(e) = k sqrt((s0 a'.e)^2 + (s1 b'.e)^2); the bound
    // is taken along the centre direction m and the elevation and azimuth directions
    // e_el, e_az there.  With p = (r + d_m) m + d_el e_el + d_az e_az:
    //   elevation of the vertical-plane part: phi_c + atan2(d_el, r + d_m), within
    //   +- A = atan(ext_el / (r - ext_m)); the horizontal offset d_az only moves the
    //   elevation toward the equator, by at most the factor c = 1/sqrt(1 + (ext_az / (r -
    //   ext_m))^2) on its sine;
    //   azimuth: atan2(d_az, h) with h >= (r - ext_m) cos phi_c - ext_el |sin phi_c|.
    // The rows are searched by the sines of their elevations, so the elevation bounds are kept
    // as sines: sin(phi_c +- A) from sin phi_c = m_z, cos phi_c = |m_xy| and cos A, sin A, with
    // a bound past +-90 degrees told by the sign of cos(phi_c +- A).  As |d sin| <= |d angle|,
    // the angular margin added to a sine keeps the bound conservative.
    // Tilted (foreshortened) and elongated surfels get a footprint much tighter than the
    // bounding cone of radius k max(s0, s1).
    const int H = g.H, W = g.W;
    int r0, r1, c0, cw;
    const float mx = rec[R_M + 0], my = rec[R_M + 1], mz = fminf(1.f, fmaxf(-1.f, rec[R_M + 2]));
    const float ch = sqrtf(mx * mx + my * my);
    const float ct = ch > 0.f ? mx / ch : 1.f, st = ch > 0.f ? my / ch : 0.f;
    const float eel[3] = {-mz * ct, -mz * st, ch};
    const float eaz[3] = {-st, ct, 0.f};
    const float mm[3] = {mx, my, mz};
    auto ext = [&](const float *e) {
        const float pa = gm.s0 * (gm.a[0] * e[0] + gm.a[1] * e[1] + gm.a[2] * e[2]);
        const float pb = gm.s1 * (gm.b[0] * e[0] + gm.b[1] * e[1] + gm.b[2] * e[2]);
        return p.cutoff * sqrtf(pa * pa + pb * pb) * (1.f + kExtSlack);
    };
    const float ext_m = ext(mm), ext_el = ext(eel), ext_az = ext(eaz);
    const float rmin = gm.r - ext_m;
    if (rmin <= 0.05f * gm.r) {  // the disk reaches around the sensor: every ray
        r0 = 0; r1 = H - 1; c0 = 0; cw = W;
    } else {
        const float rho = sqrtf(fmaf(rmin, rmin, ext_el * ext_el));
        const float cA = rmin / rho, sA = ext_el / rho;
        const float q = ext_az / rmin;
        const float c = 1.f / sqrtf(1.f + q * q);
        float s_hi = fmaf(mz, cA, ch * sA), s_lo = fmaf(mz, cA, -ch * sA);
        const bool over_hi = fmaf(ch, cA, -mz * sA) <= 0.f;  // phi_c + A reaches +90 degrees
        const bool over_lo = fmaf(ch, cA, mz * sA) <= 0.f;   // phi_c - A reaches -90 degrees
        if (s_hi < 0.f) s_hi *= c;
        if (s_lo > 0.f) s_lo *= c;
        s_hi += kAngMargin;
        s_lo -= kAngMargin;
        const bool top = over_hi || s_hi >= 1.f, bottom = over_lo || s_lo <= -1.f;
        const bool pole = top || bottom;
        if (top) s_hi = 2.f;
        if (bottom) s_lo = -2.f;
        r0 = first_row_le(rows, rstride, H, s_hi);
        r1 = first_row_lt(rows, rstride, H, s_lo) - 1;
        const float hmin = rmin * ch - ext_el * fabsf(mz);
        if (pole || hmin <= 0.f) {
            c0 = 0; cw = W;
        } else {
            const float thc = atan2f(my, mx);
            const float dth = atanf(ext_az / hmin) + kAngMargin;
            const float scale = (float)W / kTwoPi;
            const int jlo = (int)ceilf((thc - dth) * scale);
            const int jhi = (int)floorf((thc + dth) * scale);
            const int w = jhi - jlo + 1;
            if (w >= W) {
                c0 = 0; cw = W;
            } else if (w <= 0) {
                cw = 0; c0 = 0;
            } else {
                c0 = jlo % W;
                if (c0 < 0) c0 += W;
                cw = w;
            }
        }
    }
    if (r0 > r1 || cw <= 0) return make_uint2(0u, 0u);
    return make_uint2((uint32_t)r0 | ((uint32_t)r1 << 16), (uint32_t)c0 | ((uint32_t)cw << 16));
}

// Projection and emission run one 1024-thread workgroup per CU at most, each on a contiguous
// range of nearly equal length (a thread takes surfels lo + t, lo + t + 1024, ...).  The
// projection is bound by its VALU work per CU: with one surfel per thread a 300k-surfel map
// made 293 workgroups, and the 37 CUs that took two set the kernel's time.  Smaller
// workgroups do not fix that, as the dispatcher packs several onto one CU.  One count flush
// and one reservation per (workgroup, tile) cover the workgroup's range.
constexpr int kProjThreads = 1024;

int surfel_blocks(int64_t n, int n_cu)
{
    if (n <= 0) return 1;  // one workgroup still writes the pose
    const int64_t b = (n + kProjThreads - 1) / kProjThreads;
    return (int)(b < n_cu ? b : (n_cu > 0 ? n_cu : 1));
}

__device__ __forceinline__ int64_t range_lo(int64_t n, int b) { return n * b / (int64_t)gridDim.x; }

// Projection plus the per-tile pair counts, tile_cnt[t * kShards + b mod kShards] for the
// surfels of workgroup b (zero on entry).  Dynamic LDS: T words when T <= kLdsBins, else none
// (counts then go straight to tile_cnt).
__global__ __launch_bounds__(kProjThreads) void project_kernel(SurfelPtrs S, Pose pose_val, const float *__restrict__ pose_dev,
                                                      float *__restrict__ pose_out,
                                                      const float *__restrict__ rows, Grid g, RasterParams p,
                                                      float *__restrict__ recs, uint2 *__restrict__ rects,
                                                      uint32_t *__restrict__ keys, uint32_t *__restrict__ tile_cnt)
{
    extern __shared__ uint32_t bins[];
    const bool lds_bins = g.T <= kLdsBins;
    if (lds_bins)
        for (int b = threadIdx.x; b < g.T; b += kProjThreads) bins[b] = 0u;
    // the row sines, searched twice per surfel, from LDS rather than memory
    const bool lds_rows = g.H <= kLdsRows;
    float *rsin = reinterpret_cast<float *>(bins + (lds_bins ? g.T : 0));
    if (lds_rows)
        for (int k = threadIdx.x; k < g.H; k += kProjThreads) rsin[k] = rows[2 * k];
    Pose P = pose_val;
    if (pose_dev) {
        for (int c = 0; c < 9; ++c) P.r[c] = pose_dev[(c / 3) * 4 + (c % 3)];
        for (int c = 0; c < 3; ++c) P.t[c] = pose_dev[4 * c + 3];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // constant indices: the pose stays in registers
#pragma unroll
        for (int c = 0; c < 12; ++c) pose_out[c] = (c & 3) < 3 ? P.r[3 * (c >> 2) + (c & 3)] : P.t[c >> 2];
    }
    const int64_t lo = range_lo(S.n, blockIdx.x), hi = range_lo(S.n, blockIdx.x + 1);
    const int sh = (int)(blockIdx.x & (kShards - 1));
    if (lds_bins || lds_rows) __syncthreads();
    for (int64_t i0 = lo; i0 < hi; i0 += kProjThreads) {  // the same trip count for every thread
        const int64_t i = i0 + threadIdx.x;
        uint2 rc = make_uint2(0u, 0u);
        if (i < hi) {
            rc = project_one(S, P, lds_rows ? rsin : rows, lds_rows ? 1 : 2, g, p, recs, keys, i);
            rects[i] = rc;
        }
        // the whole wave enumerates (lanes past the end with an empty rectangle)
        if (lds_bins) for_each_tile(rc, 0u, g, [&](int t, uint32_t) { atomicAdd(&bins[t], 1u); });
        else for_each_tile(rc, 0u, g, [&](int t, uint32_t) { atomicAdd(&tile_cnt[t * kShards + sh], 1u); });
    }
    if (lds_bins) {
        __syncthreads();
        for (int b = threadIdx.x; b < g.T; b += kProjThreads) {
            const uint32_t c = bins[b];
            if (c) atomicAdd(&tile_cnt[b * kShards + sh], c);
        }
    }
}

// Writes surfel ids into their tiles' buckets: cursor[t * kShards + s] starts at the first
// slot of shard s of tile t.
// Per workgroup, pairs are counted per tile in LDS, one range per tile is reserved with a
// single atomic, and the workgroup's pairs fill it.  Positions at or beyond P are dropped
// (they cannot occur when the counts came from project_kernel over the same rectangles).
__global__ __launch_bounds__(kProjThreads) void emit_kernel(const uint2 *__restrict__ rects, int64_t n, Grid g,
                                                            uint32_t *__restrict__ cursor, uint32_t *__restrict__ pv,
                                                            int64_t P)
{
    extern __shared__ uint32_t bins[];  // count, then reserved base, per tile
    const int64_t lo = range_lo(n, blockIdx.x), hi = range_lo(n, blockIdx.x + 1);
    const int sh = (int)(blockIdx.x & (kShards - 1));
    auto rect_of = [&](int64_t i) { return i < hi ? rects[i] : make_uint2(0u, 0u); };
    if (g.T > kLdsBins) {
        for (int64_t i0 = lo; i0 < hi; i0 += kProjThreads) {
            const int64_t i = i0 + threadIdx.x;
            for_each_tile(rect_of(i), (uint32_t)i, g, [&](int t, uint32_t sid) {
                const uint32_t pos = atomicAdd(&cursor[t * kShards + sh], 1u);
                if ((int64_t)pos < P) pv[pos] = sid;
            });
        }
        return;
    }
    uint32_t *cnt = bins, *base = bins + g.T;
    for (int b = threadIdx.x; b < g.T; b += kProjThreads) cnt[b] = 0u;
    __syncthreads();
    for (int64_t i0 = lo; i0 < hi; i0 += kProjThreads)
        for_each_tile(rect_of(i0 + threadIdx.x), 0u, g, [&](int t, uint32_t) { atomicAdd(&cnt[t], 1u); });
    __syncthreads();
    for (int b = threadIdx.x; b < g.T; b += kProjThreads) {
        const uint32_t c = cnt[b];
        if (c) base[b] = atomicAdd(&cursor[b * kShards + sh], c);
        cnt[b] = 0u;
    }
    __syncthreads();
    for (int64_t i0 = lo; i0 < hi; i0 += kProjThreads) {
        const int64_t i = i0 + threadIdx.x;
        for_each_tile(rect_of(i), (uint32_t)i, g, [&](int t, uint32_t sid) {
            const uint32_t pos = base[t] + atomicAdd(&cnt[t], 1u);
            if ((int64_t)pos < P) pv[pos] = sid;
        });
    }
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *__restrict__ p, uint32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// out[0] += number of surfels whose ray rectangle is not empty (one atomic per workgroup)
__global__ __launch_bounds__(256) void count_visible_kernel(const uint2 *__restrict__ rects, int64_t n,
                                                            uint32_t *__restrict__ out)
{
    __shared__ uint32_t ws[4];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t m = __ballot(i < n && (rects[i].y >> 16) > 0);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c = ws[0] + ws[1] + ws[2] + ws[3];
        if (c) atomicAdd(out, c);
    }
}

__global__ __launch_bounds__(256) void max_range_kernel(const uint2 *__restrict__ ranges, int T,
                                                        uint32_t *__restrict__ out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < T) {
        uint2 r = ranges[i];
        atomicMax(out, r.y - r.x);
    }
}

// out[0] += ray-surfel tests of the raster (64 per pair and overlapping wave sub-tile).  The
// tile of pair i is the last tile whose list starts at or before i (lists are laid out in
// tile order, empty ones included).
__global__ __launch_bounds__(256) void work_tests_kernel(const uint2 *__restrict__ ranges,
                                                         const uint32_t *__restrict__ ids,
                                                         const uint2 *__restrict__ rects, int64_t P, Grid g,
                                                         unsigned long long *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c = 0;
    if (i < P) {
        int lo = 0, hi = g.T - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((int64_t)ranges[mid].x <= i) lo = mid;
            else hi = mid - 1;
        }
        int t = lo;
        int tc = t / g.TH, tr = t - tc * g.TH;
        uint2 rc = rects[ids[i]];
        for (int w = 0; w < 4; ++w) {
            int sr0 = tr * kTile + (w >> 1) * kSub, sc0 = tc * kTile + (w & 1) * kSub;
            if (sr0 < g.H && sc0 < g.W && sub_overlap(rc, sr0, sc0, g.W)) c += 64;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

// out[1] += composited hits, out[2] += rays with a hit (from the per-ray state)
__global__ __launch_bounds__(256) void work_hits_kernel(const float4 *__restrict__ st1, int64_t rays,
                                                        unsigned long long *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long k = 0, h = 0;
    if (i < rays) {
        int K = __float_as_int(st1[i].w);
        k = (unsigned long long)K;
        h = K > 0;
    }
    for (int o = 32; o >= 1; o >>= 1) {
        k += __shfl_xor(k, o, 64);
        h += __shfl_xor(h, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (k) atomicAdd(out + 1, k);
        if (h) atomicAdd(out + 2, h);
    }
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_work_counts(const uint2 *ranges, const uint32_t *ids, const uint2 *rects, int64_t P,
                              const float4 *st1, const Grid &g, unsigned long long *out, hipStream_t s)
{
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(out), 0u, 8, s);
    if (e != hipSuccess) return e;
    if (P > 0) work_tests_kernel<<<blocks_for(P, 256), 256, 0, s>>>(ranges, ids, rects, P, g, out);
    int64_t rays = (int64_t)g.H * g.W;
    work_hits_kernel<<<blocks_for(rays, 256), 256, 0, s>>>(st1, rays, out);
    return hipGetLastError();
}

hipError_t launch_project(const SurfelPtrs &S, const Pose &pose_val, const float *pose_dev, float *pose_out,
                          const float *rows, const Grid &g, const RasterParams &p, float *recs, uint2 *rects,
                          uint32_t *keys, uint32_t *tile_cnt, int blocks, hipStream_t s)
{
    const unsigned nb = (unsigned)(blocks > 0 ? blocks : 1);
    size_t lds = (g.T <= kLdsBins ? (size_t)g.T * sizeof(uint32_t) : 0) + (g.H <= kLdsRows ? (size_t)g.H * sizeof(float) : 0);
    project_kernel<<<nb, kProjThreads, lds, s>>>(S, pose_val, pose_dev, pose_out, rows, g, p, recs, rects, keys,
                                                 tile_cnt);
    return hipGetLastError();
}

hipError_t launch_emit(const uint2 *rects, int64_t n, const Grid &g, uint32_t *cursor, uint32_t *pv, int64_t P,
                       int blocks, hipStream_t s)
{
    if (n <= 0 || P <= 0) return hipSuccess;
    size_t lds = g.T <= kLdsBins ? 2 * (size_t)g.T * sizeof(uint32_t) : 0;
    emit_kernel<<<(unsigned)(blocks > 0 ? blocks : 1), kProjThreads, lds, s>>>(rects, n, g, cursor, pv, P);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    fill_u32_kernel<<<blocks_for(n, 256), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_count_visible(const uint2 *rects, int64_t n, uint32_t *out, hipStream_t s)
{
    hipError_t e = launch_fill_u32(out, 0u, 1, s);
    if (e != hipSuccess || n <= 0) return e;
    count_visible_kernel<<<blocks_for(n, 256), 256, 0, s>>>(rects, n, out);
    return hipGetLastError();
}

hipError_t launch_max_range(const uint2 *ranges, int T, uint32_t *out, hipStream_t s)
{
    hipError_t e = launch_fill_u32(out, 0u, 1, s);
    if (e != hipSuccess) return e;
    max_range_kernel<<<blocks_for(T, 256), 256, 0, s>>>(ranges, T, out);
    return hipGetLastError();
}

}  // namespace lgsr
