// raster.hip -- per-tile front-to-back compositing (forward) and its reverse-order backward.
//
// A workgroup renders one 16 x 16 tile; each of its four wavefronts owns an 8 x 8 sub-tile,
// one ray per lane, and walks the tile's range-sorted surfel list on its own (no barriers).
// A list entry is wave-uniform, so its surfel id, ray rectangle and 64-byte record are
// read with scalar loads into SGPRs; an entry whose rectangle misses the wave's sub-tile is
// skipped by a scalar branch before the record is touched.
//
// Forward per ray (Sec. 3.1 / 3.4 rendering, 2DGS surfel):
//   w = T alpha_hat, A += w, S_D += w t, S_N += w nt, T *= 1 - alpha_hat, stop once T < T_min;
//   depth = S_D / A, opacity = A, normal = S_N / A, drop = [A < drop_tau].
// It stores per ray (A, depth, T_final, last list position) and (normal, K).
//
// Backward per ray, list walked from the wave's last contributor down (lanes aligned on
// list position, each lane acting only on its own contributors), with
//   gD~ = gD / A, gN~ = gN / A, gA~ = gA - (gD depth + gN . normal) / A,
//   c_j = gD~ t_j + gN~ . nt_j + gA~,  B_j = sum_{i > j} w_i c_i,
//   dL/dalpha_hat_j = T_j c_j - B_j / (1 - alpha_hat_j),
// T_j recovered as T_{j+1} / (1 - alpha_hat_j) from the bit-identical recomputed
// alpha_hat_j.  The per-(ray, surfel) gradient w.r.t. the record quantities
// (nt, c, U, V, alpha) is summed over the wave by a butterfly and added with one vector
// atomic (11 lanes) per surfel and wave into the record-gradient buffer.
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

__global__ __launch_bounds__(256) void raster_fwd_kernel(
    const uint32_t *__restrict__ ids, const uint2 *__restrict__ ranges, const float *__restrict__ recs,
    const uint2 *__restrict__ rects, const float *__restrict__ rows, const float *__restrict__ cols, Grid g,
    RasterParams p, float *__restrict__ depth, float *__restrict__ opacity, float *__restrict__ normal,
    uint8_t *__restrict__ drop, float4 *__restrict__ st0, float4 *__restrict__ st1)
{
    const int tile = xcd_tile(blockIdx.x, g.T);
    const int tc = tile / g.TH, tr = tile - tc * g.TH;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int sr0 = tr * kTile + (wave >> 1) * kSub, sc0 = tc * kTile + (wave & 1) * kSub;
    const int k = sr0 + (lane >> 3), j = sc0 + (lane & 7);
    const bool valid = k < g.H && j < g.W;
    Ray ray = make_ray(rows, cols, valid ? k : 0, valid ? j : 0);

    float T = 1.f, A = 0.f, SD = 0.f, SN0 = 0.f, SN1 = 0.f, SN2 = 0.f;
    int K = 0, last = -1;
    bool done = !valid;
    const uint2 rg = ranges[tile];
    if (sr0 < g.H && sc0 < g.W) {
        for (uint32_t pos = rg.x; pos < rg.y; ++pos) {
            const uint32_t id = ids[pos];
            if (sub_overlap(rects[id], sr0, sc0, g.W)) {
                const Rec s = load_rec(recs, id);
                const Hit h = hit_test(s, ray, p);
                if (h.pass && !done) {
                    float w = T * h.ah;
                    A += w;
                    SD = fmaf(w, h.t, SD);
                    SN0 = fmaf(w, s.nt0, SN0);
                    SN1 = fmaf(w, s.nt1, SN1);
                    SN2 = fmaf(w, s.nt2, SN2);
                    T = T * (1.f - h.ah);
                    ++K;
                    last = (int)pos;
                    done = T < p.T_min;
                }
                if (__all(done)) break;
            }
        }
    }
    if (!valid) return;
    const int r = k * g.W + j;
    float D = 0.f, N0 = 0.f, N1 = 0.f, N2 = 0.f;
    if (K > 0) {
        D = SD / A;
        N0 = SN0 / A;
        N1 = SN1 / A;
        N2 = SN2 / A;
    }
    depth[r] = D;
    opacity[r] = A;
    normal[3 * r + 0] = N0;
    normal[3 * r + 1] = N1;
    normal[3 * r + 2] = N2;
    drop[r] = (K == 0 || A < p.drop_tau) ? 1 : 0;
    st0[r] = make_float4(A, D, T, __int_as_float(last));
    st1[r] = make_float4(N0, N1, N2, __int_as_float(K));
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ __launch_bounds__(256) void raster_bwd_kernel(
    const uint32_t *__restrict__ ids, const uint2 *__restrict__ ranges, const float *__restrict__ recs,
    const uint2 *__restrict__ rects, const float *__restrict__ rows, const float *__restrict__ cols, Grid g,
    RasterParams p, const float4 *__restrict__ st0, const float4 *__restrict__ st1, const float *__restrict__ gDp,
    const float *__restrict__ gAp, const float *__restrict__ gNp, float *__restrict__ recgrad)
{
    const int tile = xcd_tile(blockIdx.x, g.T);
    const int tc = tile / g.TH, tr = tile - tc * g.TH;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int sr0 = tr * kTile + (wave >> 1) * kSub, sc0 = tc * kTile + (wave & 1) * kSub;
    if (sr0 >= g.H || sc0 >= g.W) return;  // whole wave outside the image
    const int k = sr0 + (lane >> 3), j = sc0 + (lane & 7);
    const bool valid = k < g.H && j < g.W;
    Ray ray = make_ray(rows, cols, valid ? k : 0, valid ? j : 0);

    int last = -1;
    float T = 1.f, gbD = 0.f, gbN0 = 0.f, gbN1 = 0.f, gbN2 = 0.f, gbA = 0.f;
    if (valid) {
        const int r = k * g.W + j;
        float4 a = st0[r], b = st1[r];
        last = __float_as_int(a.w);
        if (last >= 0) {
            float A = a.x, D = a.y;
            T = a.z;
            float iA = 1.f / A;
            float gd = gDp[r], ga = gAp[r];
            float gn0 = gNp[3 * r], gn1 = gNp[3 * r + 1], gn2 = gNp[3 * r + 2];
            gbD = gd * iA;
            gbN0 = gn0 * iA;
            gbN1 = gn1 * iA;
            gbN2 = gn2 * iA;
            gbA = ga - (gd * D + gn0 * b.x + gn1 * b.y + gn2 * b.z) * iA;
        }
    }
    const int pmax = wave_max_i(last);
    const uint2 rg = ranges[tile];
    float B = 0.f;
    for (int pos = pmax; pos >= (int)rg.x; --pos) {
        const uint32_t id = ids[pos];
        if (!sub_overlap(rects[id], sr0, sc0, g.W)) continue;
        const Rec s = load_rec(recs, id);
        float gv[11];
#pragma unroll
        for (int c = 0; c < 11; ++c) gv[c] = 0.f;
        bool contrib = false;
        if (pos <= last) {
            Hit h = hit_test(s, ray, p);
            if (h.pass) {
                contrib = true;
                float one_m = 1.f - h.ah;
                float r1m = __builtin_amdgcn_rcpf(one_m);
                float Tj = T * r1m;
                float w = Tj * h.ah;
                float cj = fmaf(gbD, h.t, fmaf(gbN0, s.nt0, fmaf(gbN1, s.nt1, fmaf(gbN2, s.nt2, gbA))));
                float dah = fmaf(Tj, cj, -B * r1m);
                B = fmaf(w, cj, B);
                T = Tj;
                float dt = gbD * w;
                float dalpha = 0.f, dG = 0.f;
                if (h.aG < p.alpha_max) {
                    dalpha = dah * h.G;
                    dG = dah * s.alpha;
                }
                float dq2 = -0.5f * h.G * dG;
                float u = h.nu * h.inv, v = h.nv * h.inv;
                float du = 2.f * u * dq2, dv = 2.f * v * dq2;
                float dnu = du * h.inv, dnv = dv * h.inv;
                float dden = -fmaf(du, u, fmaf(dv, v, dt * h.t)) * h.inv;
                float dc = dt * h.inv;
                gv[G_NT + 0] = fmaf(gbN0, w, dden * ray.dh[0]);
                gv[G_NT + 1] = fmaf(gbN1, w, dden * ray.dh[1]);
                gv[G_NT + 2] = fmaf(gbN2, w, dden * ray.dh[2]);
                gv[G_C] = dc;
                gv[G_U + 0] = dnu * ray.dh[0];
                gv[G_U + 1] = dnu * ray.dh[1];
                gv[G_U + 2] = dnu * ray.dh[2];
                gv[G_V + 0] = dnv * ray.dh[0];
                gv[G_V + 1] = dnv * ray.dh[1];
                gv[G_V + 2] = dnv * ray.dh[2];
                gv[G_ALPHA] = dalpha;
            }
        }
        if (__any(contrib)) {
            float mine = 0.f;
#pragma unroll
            for (int c = 0; c < 11; ++c) {
                float sum = wave_sum(gv[c]);
                mine = (lane == c) ? sum : mine;
            }
            if (lane < 11) unsafeAtomicAdd(recgrad + (size_t)id * kGrad + lane, mine);
        }
    }
}

static inline unsigned grid_tiles(const Grid &g) { return (unsigned)g.T; }

hipError_t launch_raster_fwd(const uint32_t *ids, const uint2 *ranges, const float *recs, const uint2 *rects,
                             const float *rows, const float *cols, const Grid &g, const RasterParams &p,
                             float *depth, float *opacity, float *normal, uint8_t *drop, float4 *st0, float4 *st1,
                             hipStream_t s)
{
    if (g.T <= 0) return hipSuccess;
    raster_fwd_kernel<<<grid_tiles(g), 256, 0, s>>>(ids, ranges, recs, rects, rows, cols, g, p, depth, opacity,
                                                    normal, drop, st0, st1);
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const uint32_t *ids, const uint2 *ranges, const float *recs, const uint2 *rects,
                             const float *rows, const float *cols, const Grid &g, const RasterParams &p,
                             const float4 *st0, const float4 *st1, const float *gD, const float *gA,
                             const float *gN, float *recgrad, hipStream_t s)
{
    if (g.T <= 0) return hipSuccess;
    raster_bwd_kernel<<<grid_tiles(g), 256, 0, s>>>(ids, ranges, recs, rects, rows, cols, g, p, st0, st1, gD, gA,
                                                    gN, recgrad);
    return hipGetLastError();
}

}  // namespace lgsr
