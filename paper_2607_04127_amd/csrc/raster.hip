// raster.hip -- chunk-parallel front-to-back compositing and its reverse-order backward.
//
// Each tile (16 x 16 rays) owns a range-sorted list of surfels.  The lists are cut into
// chunks of `seg` entries.  A task is one (chunk, 8 x 8 sub-tile) pair and runs as a
// workgroup of one wavefront (one ray per lane): it stages, 64 list entries at a time, the
// ids and 64-byte records of the entries whose ray rectangle meets its sub-tile in LDS with
// coalesced vector loads, then walks them broadcasting each record from LDS.  Chunking
// spreads long lists over many workgroups (load balance); one-wave workgroups keep the
// SIMDs filled when sub-tiles of one chunk differ widely in cost.
//
// Compositing (Sec. 3.1 / 3.4 rendering with the 2DGS surfel), per ray and hit:
//   w = T alpha_hat, A += w, S_D += w t, S_N += w nt, T *= 1 - alpha_hat, stop once T < T_min.
// Segments compose associatively: with the transmittance T_pre in front of a chunk, its
// local sums (from T = 1) enter as (T_pre T_loc, A + T_pre A_loc, ...).  Every chunk stops
// locally at T_loc < T_min, which is exact for the first chunk of a tile (T_pre = 1).  The
// merge walks a ray's chunks in order; if T_pre T_loc drops below T_min inside a later
// chunk, the ray terminated there and that one chunk is re-walked sequentially from T_pre
// (fix-up) while later chunks are dropped.
//
// Backward, per ray and chunk (list walked from the wave's last contributor down, lanes
// aligned on list position, each lane acting only on its own contributors):
//   gD~ = gD / A, gN~ = gN / A, gA~ = gA - (gD depth + gN . normal) / A,
//   c_j = gD~ t_j + gN~ . nt_j + gA~,  B_j = sum_{i > j} w_i c_i (global weights),
//   dL/dalpha_hat_j = T_j c_j - B_j / (1 - alpha_hat_j).
// B at the end of a chunk is gD~ S_D + gN~ . S_N + gA~ S_A over the later chunks' sums: the
// merge leaves those suffix sums per (chunk, ray) (all but the sums of the chunk a fix-up
// re-walks, which the fix-up leaves per ray), so each backward task forms its B from the
// upstream gradient directly and no set-up pass runs between the loss and the backward.
// T_j is recovered as T_{j+1} / (1 - alpha_hat_j) from the bit-identical recomputed
// alpha_hat_j.  The per-(ray, surfel) gradient w.r.t.
// the record quantities (nt, c, cu, U, cv, V, alpha; U and V split along m as the record
// splits them; and the hit-distance terms along m) is summed over the wave and added with
// one vector atomic (15 lanes) per surfel and wave.
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

// Per (chunk, ray) slot fields; slot(item, f, rt) with rt = wave * 64 + lane.  The forward
// writes a slot only where the chunk has a contributor for the ray (its bit in the task's
// composite mask, kmask), and every reader looks at the mask first: F_TEND, F_LAST, F_K and
// the chunk's local sums F_SA .. F_SN2.  The merge turns F_TEND into the global transmittance and, where the
// chunk keeps a contributor (F_LAST >= 0), F_SA .. F_SN2 into the sums of all later chunks
// of the tile in global weights (the fix-up chunk's aside).
enum : int { F_TEND = 0, F_SA, F_SD, F_SN0, F_SN1, F_SN2, F_LAST, F_K, kSlotFields };

__device__ __forceinline__ size_t slot(uint32_t item, int f, int rt)
{
    return ((size_t)item * kSlotFields + f) * 256 + rt;
}

struct Lane {
    int wave, lane, rt, sr0, sc0, k, j;
    bool valid, wave_in;
};

// Ray t (0..255) of tile `tile`: wave t / 64 owns one 8 x 8 sub-tile.
__device__ __forceinline__ Lane lane_of(int tile, const Grid &g, int t = (int)threadIdx.x)
{
    Lane L;
    const int tc = tile / g.TH, tr = tile - tc * g.TH;
    L.wave = __builtin_amdgcn_readfirstlane(t >> 6);
    L.lane = t & 63;
    L.rt = t;
    L.sr0 = tr * kTile + (L.wave >> 1) * kSub;
    L.sc0 = tc * kTile + (L.wave & 1) * kSub;
    L.k = L.sr0 + (L.lane >> 3);
    L.j = L.sc0 + (L.lane & 7);
    L.valid = L.k < g.H && L.j < g.W;
    L.wave_in = L.sr0 < g.H && L.sc0 < g.W;
    return L;
}

// ---------------------------------------------------------------------------------------
// forward (the chunk list comes from the tile sort launch)
// ---------------------------------------------------------------------------------------

struct Acc {
    float T, A, SD, SN0, SN1, SN2;
    int K, last;
};

// A chunk's (tile, first, end) as scalar values (all lanes read the same entry).
__device__ __forceinline__ uint4 uniform_chunk(const uint4 *__restrict__ chunks, uint32_t item)
{
    const uint4 c = chunks[item];
    return make_uint4(__builtin_amdgcn_readfirstlane(c.x), __builtin_amdgcn_readfirstlane(c.y),
                      __builtin_amdgcn_readfirstlane(c.z), 0u);
}

// One wavefront per task (chunk item, sub-tile wave): a workgroup of one wave, so that a
// slot frees as soon as its sub-tile is done and sub-tiles of very different cost do not
// hold each other's LDS.  Blocks are dealt to the 8 XCDs round-robin; the task of block b
// keeps an item's four waves on one XCD (they read the same list entries) while consecutive
// items go to different XCDs (dense and sparse azimuth sectors are spread evenly).  The
// grid is a multiple of 32 blocks.
__device__ __forceinline__ uint32_t task_of(uint32_t b) { return (b >> 5) * 32u + (b & 7u) * 4u + ((b >> 3) & 3u); }

static_assert(kTileChunks <= 64, "the merge keeps a run's chunks as the bits of a 64-bit word");

constexpr int kTaskGroup = 32;
static unsigned task_blocks(int items) { return (unsigned)(((int64_t)4 * items + kTaskGroup - 1) / kTaskGroup * kTaskGroup); }

// Up to 64 list entries staged in LDS by one wave: of the entries whose ray rectangle meets
// the wave's sub-tile, in list order, the surfel ids, list positions and 64-byte records.
constexpr int kWStage = 64;
constexpr int kChunkMax = 256;  // longest chunk the automatic choice makes
struct WaveStage {
    float4 rec[kWStage][4];
    uint32_t id[kWStage];
    uint32_t pos[kWStage];
};

// Stages list entries [a, a + n), n <= 64; returns how many meet the sub-tile (uniform).
// Lane l loads entry l's ray rectangle and whole record together (two memory latencies in
// all: the id, then both), and the entries that meet the sub-tile are written compacted.
// Afterwards lane k holds staged slot k's list position and surfel id (slot_pos, slot_id),
// which the walk reads with readlane instead of LDS.
__device__ __forceinline__ uint32_t stage_wave(WaveStage &ws, const uint32_t *__restrict__ ids,
                                               const float *__restrict__ recs, const uint2 *__restrict__ rects,
                                               uint32_t a, uint32_t n, const Lane &L, int W, uint32_t &slot_pos,
                                               uint32_t &slot_id)
{
    const uint32_t l = (uint32_t)L.lane;
    const bool in = l < n;
    const uint32_t id = in ? ids[a + l] : 0u;
    const float4 *r4 = reinterpret_cast<const float4 *>(recs) + (size_t)id * 4;
    float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0, q2 = q0, q3 = q0;
    uint2 rc = make_uint2(0u, 0u);
    if (in) {
        rc = rects[id];
        q0 = r4[0];
        q1 = r4[1];
        q2 = r4[2];
        q3 = r4[3];
    }
    const bool meet = in && sub_overlap(rc, L.sr0, L.sc0, W);
    const uint64_t bal = __ballot(meet);
    const uint32_t m = __builtin_amdgcn_readfirstlane((uint32_t)__popcll(bal));
    const uint32_t k = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    if (meet) {
        ws.id[k] = id;
        ws.pos[k] = a + l;
        ws.rec[k][0] = q0;
        ws.rec[k][1] = q1;
        ws.rec[k][2] = q2;
        ws.rec[k][3] = q3;
    }
    __syncthreads();
    slot_pos = ws.pos[l];  // meaningful for l < m
    slot_id = ws.id[l];
    return m;
}

__device__ __forceinline__ Rec staged_rec(const WaveStage &ws, uint32_t i)
{
    const float4 x = ws.rec[i][0], y = ws.rec[i][1], z = ws.rec[i][2], w = ws.rec[i][3];
    return Rec{x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w, z.x, z.y, z.z, z.w, w.x, w.y, w.z, w.w};
}

// Composite list entries [a, b) for this wave's rays, starting from acc (transmittance
// acc.T); lanes with `active` false only follow along.  A lane stops once T < T_min; the
// wave stops, and stages nothing more, once all of its lanes have.
__device__ __forceinline__ void composite(WaveStage &ws, const uint32_t *__restrict__ ids,
                                          const float *__restrict__ recs, const uint2 *__restrict__ rects,
                                          uint32_t a, uint32_t b, const Lane &L, const Ray &ray,
                                          const RasterParams &p, int W, bool active, Acc &acc)
{
    bool done = !active || !L.wave_in;
    for (uint32_t base = a; base < b; base += kWStage) {
        if (__all(done)) return;
        uint32_t slot_pos, slot_id;
        const uint32_t m = stage_wave(ws, ids, recs, rects, base, min((uint32_t)kWStage, b - base), L, W, slot_pos,
                                      slot_id);
        // Entry i: the hit test, and the composite on lanes that pass; true once every lane
        // is done (only a composite can change that).
        auto step = [&](const Rec &s, uint32_t i) -> bool {
            Hit h;
            const float q2 = hit_geom(h, s, ray, p);
            if (!__any(h.pass && !done)) return false;  // no lane reaches the opacity test
            hit_opacity(h, q2, s, p);
            if (h.pass && !done) {
                float w = acc.T * h.ah;
                acc.A += w;
                acc.SD = fmaf(w, h.t, acc.SD);
                acc.SN0 = fmaf(w, s.nt0, acc.SN0);
                acc.SN1 = fmaf(w, s.nt1, acc.SN1);
                acc.SN2 = fmaf(w, s.nt2, acc.SN2);
                acc.T = acc.T * (1.f - h.ah);
                ++acc.K;
                acc.last = (int)__builtin_amdgcn_readlane((int)slot_pos, (int)i);
                done = acc.T < p.T_min;
            }
            return __all(done);
        };
        // Two record buffers in turn: the next entry's record is read from LDS while this one
        // is tested, with no register copies between them.
        Rec ra = staged_rec(ws, 0), rb;
        for (uint32_t i = 0; i < m; i += 2) {
            rb = staged_rec(ws, i + 1 < m ? i + 1 : i);
            if (step(ra, i) || i + 1 >= m) break;
            ra = staged_rec(ws, i + 2 < m ? i + 2 : i);
            if (step(rb, i + 1)) break;
        }
        __syncthreads();  // the stage is no longer read
    }
}

// Block b of a request's forward chunk launch (b = blockIdx.x for a single request).
__device__ __forceinline__ void fwd_chunk_task(
    const uint4 *__restrict__ chunks, const uint32_t *__restrict__ n_items, const uint32_t *__restrict__ ids,
    const float *__restrict__ recs, const uint2 *__restrict__ rects, const float *__restrict__ rows,
    const float *__restrict__ cols, const Grid &g, const RasterParams &p, float *__restrict__ slots,
    uint64_t *__restrict__ kmask, uint32_t b)
{
    __shared__ WaveStage ws;
    const uint32_t task = task_of(b), item = task >> 2;
    if (item >= *n_items) return;
    const uint4 ch = uniform_chunk(chunks, item);
    const Lane L = lane_of((int)ch.x, g, (int)((task & 3u) * 64u + threadIdx.x));
    if (!L.wave_in) {  // the sub-tile lies outside the image
        if (threadIdx.x == 0) kmask[task] = 0ull;
        return;
    }
    Ray ray = make_ray(rows, cols, L.valid ? L.k : 0, L.valid ? L.j : 0);
    Acc acc{1.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0, -1};
    composite(ws, ids, recs, rects, ch.y, ch.z, L, ray, p, g.W, L.valid, acc);
    const uint64_t km = __ballot(L.valid && acc.K > 0);
    if (threadIdx.x == 0) kmask[task] = km;
    // the slot of a ray without a composite here is read by no one: its mask bit is clear
    if (!L.valid || acc.K == 0) return;
    slots[slot(item, F_TEND, L.rt)] = acc.T;
    slots[slot(item, F_LAST, L.rt)] = __int_as_float(acc.last);
    slots[slot(item, F_K, L.rt)] = __int_as_float(acc.K);
    slots[slot(item, F_SA, L.rt)] = acc.A;
    slots[slot(item, F_SD, L.rt)] = acc.SD;
    slots[slot(item, F_SN0, L.rt)] = acc.SN0;
    slots[slot(item, F_SN1, L.rt)] = acc.SN1;
    slots[slot(item, F_SN2, L.rt)] = acc.SN2;
}

__global__ __launch_bounds__(64) void raster_fwd_chunk_kernel(
    const uint4 *__restrict__ chunks, const uint32_t *__restrict__ n_items, const uint32_t *__restrict__ ids,
    const float *__restrict__ recs, const uint2 *__restrict__ rects, const float *__restrict__ rows,
    const float *__restrict__ cols, Grid g, RasterParams p, float *__restrict__ slots, uint64_t *__restrict__ kmask)
{
    fwd_chunk_task(chunks, n_items, ids, recs, rects, rows, cols, g, p, slots, kmask, blockIdx.x);
}

__device__ __forceinline__ void write_ray(const Lane &L, const Grid &g, const RasterParams &p, float A, float SD,
                                          float SN0, float SN1, float SN2, float T, int K, float *__restrict__ depth,
                                          float *__restrict__ opacity, float *__restrict__ normal,
                                          uint8_t *__restrict__ drop, float4 *__restrict__ st0,
                                          float4 *__restrict__ st1)
{
    const int r = L.k * g.W + L.j;
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
    st0[r] = make_float4(A, D, T, 0.f);
    st1[r] = make_float4(N0, N1, N2, __int_as_float(K));
}

// One workgroup per tile: combine the chunks of every ray in list order (slots become
// global: end transmittance, and the sums of the later chunks in global weights), detect
// termination in a later chunk (-> fix-up record) and write the frame for rays that need
// no fix-up.  The tile's chunks are split into kMergeGroups runs handled side by side, 256
// threads (one per ray) each: first the product of each run's chunk transmittances (a
// chunk's transmittance is exactly 1 for a ray it does not touch), which gives every run
// its exact incoming transmittance; then each run walks its chunks from there; then each
// run walks its chunks back from the later runs' sums, leaving every contributing chunk the
// sums behind it, and one pass per ray joins the runs' sums in order up to the first run in
// which the ray terminates.
constexpr int kMergeGroups = 4;  // at most; the launch picks 1 or 4 (blockDim.x / 256)
constexpr int kMergeThreads = 256 * kMergeGroups;

// LDS floats per run: the product of its chunk transmittances, then its end T, A, SD, SN0,
// SN1, SN2, K and fix chunk, each for 256 rays.
constexpr int kMergeRunFloats = 9 * 256;

__device__ __forceinline__ void run_bounds(uint32_t c0, uint32_t c1, int grp, int ng, uint32_t &r0, uint32_t &r1)
{
    const uint32_t q = (c1 - c0 + ng - 1) / ng;
    r0 = min(c1, c0 + grp * q);
    r1 = min(c1, r0 + q);
}

// Runs per tile: enough workgroups to fill the machine first, then shorter chains.
int merge_groups(int T) { return T <= 512 ? 4 : 1; }

// Tile `tile` of a request's merge launch.
__device__ __forceinline__ void merge_tile(const uint32_t *__restrict__ chunk_base, const Grid &g,
                                           const RasterParams &p, float *__restrict__ slots,
                                           float *__restrict__ depth, float *__restrict__ opacity,
                                           float *__restrict__ normal, uint8_t *__restrict__ drop,
                                           float4 *__restrict__ st0, float4 *__restrict__ st1,
                                           float4 *__restrict__ fixA, float4 *__restrict__ fixB,
                                           uint32_t *__restrict__ fixflag, const uint64_t *__restrict__ kmask,
                                           int tile)
{
    extern __shared__ float msm[];  // ng runs x kMergeRunFloats
    const int ng = (int)(blockDim.x >> 8);
    // a run is four whole waves, so its index is uniform in a wave (chunk loops and mask loads
    // become scalar)
    const int t = (int)(threadIdx.x & 255u), grp = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 8));
    const Lane L = lane_of(tile, g, t);
    const uint32_t c0 = chunk_base[tile], c1 = chunk_base[tile + 1];
    uint32_t r0, r1;
    run_bounds(c0, c1, grp, ng, r0, r1);
    auto P_of = [&](int q) -> float & { return msm[q * kMergeRunFloats + t]; };
    auto S_of = [&](int q, int f) -> float & { return msm[q * kMergeRunFloats + (1 + f) * 256 + t]; };
    constexpr int kB = 8;  // chunks whose slots are loaded together (one memory latency per batch)
    // kmask[4 item + wave]: the lanes of this wave's sub-tile with a composite in chunk item
    // (the forward's); a slot of any other lane holds T_end = 1 and no sums, so only these
    // lanes load, and a batch of chunks in which no lane has a composite is skipped
    const int wv = L.wave;
    auto masks = [&](uint32_t it0, uint64_t (&mk)[kB]) -> uint64_t {
        uint64_t any = 0ull;
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            mk[q] = it0 + q < r1 ? kmask[(size_t)(it0 + q) * 4 + wv] : 0ull;
            any |= mk[q];
        }
        return any;
    };
    const int ln = L.lane;
    // 1. the run's transmittance product (read by the later runs only)
    if (grp + 1 < ng) {
        float P = 1.f;
        for (uint32_t it0 = r0; it0 < r1; it0 += kB) {
            uint64_t mk[kB];
            if (masks(it0, mk) == 0ull) continue;
            float v[kB];
#pragma unroll
            for (int q = 0; q < kB; ++q) v[q] = (mk[q] >> ln & 1ull) ? slots[slot(it0 + q, F_TEND, L.rt)] : 1.f;
#pragma unroll
            for (int q = 0; q < kB; ++q) P *= v[q];
        }
        P_of(grp) = P;
    }
    __syncthreads();
    // 2. the run from its incoming transmittance
    float T = 1.f, A = 0.f, SD = 0.f, SN0 = 0.f, SN1 = 0.f, SN2 = 0.f;
    int K = 0, fix = -1;
    for (int q = 0; q < grp; ++q) T *= P_of(q);
    // bit (it - r0) of `kept`: chunk it keeps a contributor for this lane's ray (a run has at
    // most kTileChunks <= 64 chunks); a run of at most kB chunks also keeps those chunks'
    // global sums in v for step 3
    const bool one_batch = r1 - r0 <= (uint32_t)kB;
    uint64_t kept = 0ull;
    float v[kB][7];
    for (uint32_t it0 = r0; it0 < r1; it0 += kB) {
        uint64_t mk[kB];
        if (masks(it0, mk) == 0ull) continue;
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            if (mk[q] >> ln & 1ull) {
                const uint32_t it = it0 + q;
                v[q][0] = slots[slot(it, F_K, L.rt)];
                v[q][1] = slots[slot(it, F_TEND, L.rt)];
                v[q][2] = slots[slot(it, F_SA, L.rt)];
                v[q][3] = slots[slot(it, F_SD, L.rt)];
                v[q][4] = slots[slot(it, F_SN0, L.rt)];
                v[q][5] = slots[slot(it, F_SN1, L.rt)];
                v[q][6] = slots[slot(it, F_SN2, L.rt)];
            }
        }
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            const uint32_t it = it0 + q;
            if (it >= r1) break;
            if (!(mk[q] >> ln & 1ull)) continue;  // no composite: F_LAST is -1, nothing to add
            if (fix >= 0 || T < p.T_min) {  // after termination: the chunk contributes nothing
                slots[slot(it, F_LAST, L.rt)] = __int_as_float(-1);
                continue;
            }
            const int Kl = __float_as_int(v[q][0]);
            const float Tn = T * v[q][1];
            if (it > c0 && Tn < p.T_min) {  // the ray terminates inside this chunk: re-walk it
                fix = (int)it;              // the run's end state is then the state before it
                slots[slot(it, F_LAST, L.rt)] = __int_as_float(-1);
                continue;
            }
            const float gA = T * v[q][2], gD = T * v[q][3], g0 = T * v[q][4], g1 = T * v[q][5], g2 = T * v[q][6];
            slots[slot(it, F_TEND, L.rt)] = Tn;
            kept |= 1ull << (it - r0);
            if (one_batch) {
                v[q][2] = gA;
                v[q][3] = gD;
                v[q][4] = g0;
                v[q][5] = g1;
                v[q][6] = g2;
            } else {
                slots[slot(it, F_SA, L.rt)] = gA;
                slots[slot(it, F_SD, L.rt)] = gD;
                slots[slot(it, F_SN0, L.rt)] = g0;
                slots[slot(it, F_SN1, L.rt)] = g1;
                slots[slot(it, F_SN2, L.rt)] = g2;
            }
            A += gA;
            SD += gD;
            SN0 += g0;
            SN1 += g1;
            SN2 += g2;
            K += Kl;
            T = Tn;
        }
    }
    S_of(grp, 0) = T;
    S_of(grp, 1) = A;
    S_of(grp, 2) = SD;
    S_of(grp, 3) = SN0;
    S_of(grp, 4) = SN1;
    S_of(grp, 5) = SN2;
    S_of(grp, 6) = __int_as_float(K);
    S_of(grp, 7) = __int_as_float(fix);
    __syncthreads();
    if (!L.valid) return;
    // 3. every contributing chunk of the run gets the sums of all later chunks: the later runs'
    // sums (zero past termination), then the run's own chunks walked backwards
    {
        float bA = 0.f, bD = 0.f, b0 = 0.f, b1 = 0.f, b2 = 0.f;
        for (int q = grp + 1; q < ng; ++q) {
            bA += S_of(q, 1);
            bD += S_of(q, 2);
            b0 += S_of(q, 3);
            b1 += S_of(q, 4);
            b2 += S_of(q, 5);
        }
        auto emit = [&](uint32_t it, const float (&c)[7]) {
            slots[slot(it, F_SA, L.rt)] = bA;
            slots[slot(it, F_SD, L.rt)] = bD;
            slots[slot(it, F_SN0, L.rt)] = b0;
            slots[slot(it, F_SN1, L.rt)] = b1;
            slots[slot(it, F_SN2, L.rt)] = b2;
            bA += c[2];
            bD += c[3];
            b0 += c[4];
            b1 += c[5];
            b2 += c[6];
        };
        if (one_batch) {
#pragma unroll
            for (int q = kB - 1; q >= 0; --q)
                if (kept >> q & 1ull) emit(r0 + q, v[q]);
        } else {
            for (uint32_t top = r1; top > r0;) {
                const uint32_t lo = top - r0 > (uint32_t)kB ? top - kB : r0;
                const uint64_t kb = (kept >> (lo - r0)) & ((1ull << (top - lo)) - 1ull);
                if (__any(kb != 0ull)) {
#pragma unroll
                    for (int q = 0; q < kB; ++q) {
                        const uint32_t it = top - 1 - q;
                        if (it >= lo && it < top && (kb >> (it - lo) & 1ull)) {
                            v[q][2] = slots[slot(it, F_SA, L.rt)];
                            v[q][3] = slots[slot(it, F_SD, L.rt)];
                            v[q][4] = slots[slot(it, F_SN0, L.rt)];
                            v[q][5] = slots[slot(it, F_SN1, L.rt)];
                            v[q][6] = slots[slot(it, F_SN2, L.rt)];
                        }
                    }
#pragma unroll
                    for (int q = 0; q < kB; ++q) {
                        const uint32_t it = top - 1 - q;
                        if (it < lo || it >= top) break;
                        if (kb >> (it - lo) & 1ull) emit(it, v[q]);
                    }
                }
                top = lo;
            }
        }
    }
    // 4. join the runs in order
    if (grp != 0) return;
    float aA = 0.f, aD = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f, Tf = 1.f;
    int aK = 0, fx = -1;
    for (int q = 0; q < ng; ++q) {
        aA += S_of(q, 1);
        aD += S_of(q, 2);
        a0 += S_of(q, 3);
        a1 += S_of(q, 4);
        a2 += S_of(q, 5);
        aK += __float_as_int(S_of(q, 6));
        Tf = S_of(q, 0);
        fx = __float_as_int(S_of(q, 7));
        if (fx >= 0 || Tf < p.T_min) break;  // later runs start below T_min: they add nothing
    }
    const int r = L.k * g.W + L.j;
    if (fx >= 0) {
        fixA[r] = make_float4(Tf, aA, aD, __int_as_float(aK));
        fixB[r] = make_float4(a0, a1, a2, __int_as_float(fx));
        fixflag[fx * 4 + L.wave] = 1u;  // the chunk has a ray of this sub-tile to re-walk
    } else {
        fixA[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        fixB[r] = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
        write_ray(L, g, p, aA, aD, a0, a1, a2, Tf, aK, depth, opacity, normal, drop, st0, st1);
    }
}

__global__ __launch_bounds__(kMergeThreads) void raster_merge_kernel(const uint32_t *__restrict__ chunk_base, Grid g,
                                                                     RasterParams p, float *__restrict__ slots,
                                                                     float *__restrict__ depth,
                                                                     float *__restrict__ opacity,
                                                                     float *__restrict__ normal,
                                                                     uint8_t *__restrict__ drop,
                                                                     float4 *__restrict__ st0, float4 *__restrict__ st1,
                                                                     float4 *__restrict__ fixA, float4 *__restrict__ fixB,
                                                                     uint32_t *__restrict__ fixflag,
                                                                     const uint64_t *__restrict__ kmask)
{
    merge_tile(chunk_base, g, p, slots, depth, opacity, normal, drop, st0, st1, fixA, fixB, fixflag, kmask,
               blockIdx.x);
}

// Re-walk the chunk in which a ray terminates, from its true transmittance, and finish it.
// One wave per (chunk, sub-tile) task, flagged by the merge.
__device__ __forceinline__ void fixup_task(
    const uint4 *__restrict__ chunks, const uint32_t *__restrict__ n_items, const uint32_t *__restrict__ ids,
    const float *__restrict__ recs, const uint2 *__restrict__ rects, const float *__restrict__ rows,
    const float *__restrict__ cols, const Grid &g, const RasterParams &p, float4 *__restrict__ fixA,
    float4 *__restrict__ fixB, float *__restrict__ slots, float *__restrict__ depth, float *__restrict__ opacity,
    float *__restrict__ normal, uint8_t *__restrict__ drop, float4 *__restrict__ st0, float4 *__restrict__ st1,
    uint32_t *__restrict__ fixflag, uint32_t b)
{
    __shared__ WaveStage ws;
    const uint32_t task = task_of(b), item = task >> 2;
    if (item >= *n_items) return;
    if (__builtin_amdgcn_readfirstlane(fixflag[task]) == 0u) return;  // no ray of this sub-tile re-walks here
    if (threadIdx.x == 0) fixflag[task] = 0u;                         // zero for the next forward
    const uint4 ch = uniform_chunk(chunks, item);
    const Lane L = lane_of((int)ch.x, g, (int)((task & 3u) * 64u + threadIdx.x));
    const int r = L.valid ? L.k * g.W + L.j : 0;
    float4 fa = make_float4(0.f, 0.f, 0.f, 0.f), fb = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
    if (L.valid) {
        fb = fixB[r];
        fa = fixA[r];
    }
    const bool pend = L.valid && __float_as_int(fb.w) == (int)item;
    if (!__any(pend)) return;
    Ray ray = make_ray(rows, cols, L.valid ? L.k : 0, L.valid ? L.j : 0);
    Acc acc{pend ? fa.x : 1.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0, -1};
    composite(ws, ids, recs, rects, ch.y, ch.z, L, ray, p, g.W, pend, acc);
    if (!pend) return;
    slots[slot(item, F_TEND, L.rt)] = acc.T;
    slots[slot(item, F_LAST, L.rt)] = __int_as_float(acc.last);
    slots[slot(item, F_K, L.rt)] = __int_as_float(acc.K);
    write_ray(L, g, p, fa.y + acc.A, fa.z + acc.SD, fb.x + acc.SN0, fb.y + acc.SN1, fb.z + acc.SN2, acc.T,
              __float_as_int(fa.w) + acc.K, depth, opacity, normal, drop, st0, st1);
    // the chunk's sums for the backward of the earlier chunks (nothing after it contributes);
    // the chunk index stays in fixB.w
    fixA[r] = make_float4(acc.A, acc.SD, acc.SN0, acc.SN1);
    fixB[r] = make_float4(acc.SN2, 0.f, 0.f, __int_as_float((int)item));
}

__global__ __launch_bounds__(64) void raster_fixup_kernel(
    const uint4 *__restrict__ chunks, const uint32_t *__restrict__ n_items, const uint32_t *__restrict__ ids,
    const float *__restrict__ recs, const uint2 *__restrict__ rects, const float *__restrict__ rows,
    const float *__restrict__ cols, Grid g, RasterParams p, float4 *__restrict__ fixA,
    float4 *__restrict__ fixB, float *__restrict__ slots, float *__restrict__ depth, float *__restrict__ opacity,
    float *__restrict__ normal, uint8_t *__restrict__ drop, float4 *__restrict__ st0, float4 *__restrict__ st1,
    uint32_t *__restrict__ fixflag)
{
    fixup_task(chunks, n_items, ids, recs, rects, rows, cols, g, p, fixA, fixB, slots, depth, opacity, normal, drop,
               st0, st1, fixflag, blockIdx.x);
}

// ---------------------------------------------------------------------------------------
// forward over a batch of requests: one launch per stage for all of them
// ---------------------------------------------------------------------------------------

// The job of block b (jobs sorted by first block; at most kMaxFwdJobs, a uniform scan).
__device__ __forceinline__ int job_of(const FwdJobs &J, uint32_t b, bool merge)
{
    int j = 0;
    for (int k = 1; k < J.n; ++k)
        if (b >= (merge ? J.j[k].tile0 : J.j[k].block0)) j = k;
    return j;
}

__global__ __launch_bounds__(64) void raster_fwd_chunk_multi(FwdJobs J, RasterParams p)
{
    const int j = job_of(J, blockIdx.x, false);
    const FwdJob &q = J.j[j];
    fwd_chunk_task(q.R.chunks, q.R.n_items, q.R.ids, q.R.recs, q.R.rects, q.R.rows, q.R.cols, q.g, p, q.R.slots,
                   q.R.kmask, blockIdx.x - q.block0);
}

__global__ __launch_bounds__(kMergeThreads) void raster_merge_multi(FwdJobs J, RasterParams p)
{
    const int j = job_of(J, blockIdx.x, true);
    const FwdJob &q = J.j[j];
    merge_tile(q.R.chunk_base, q.g, p, q.R.slots, q.depth, q.opacity, q.normal, q.drop, q.R.st0, q.R.st1, q.R.fixA,
               q.R.fixB, q.R.fixflag, q.R.kmask, (int)(blockIdx.x - q.tile0));
}

__global__ __launch_bounds__(64) void raster_fixup_multi(FwdJobs J, RasterParams p)
{
    const int j = job_of(J, blockIdx.x, false);
    const FwdJob &q = J.j[j];
    fixup_task(q.R.chunks, q.R.n_items, q.R.ids, q.R.recs, q.R.rects, q.R.rows, q.R.cols, q.g, p, q.R.fixA, q.R.fixB,
               q.R.slots, q.depth, q.opacity, q.normal, q.drop, q.R.st0, q.R.st1, q.R.fixflag, blockIdx.x - q.block0);
}

// ---------------------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------------------

// Wave-wide sums of 16 per-lane values by transposition: v_permlane32_swap folds lanes
// 32-63 onto 0-31 for eight pairs (i, i + 8), v_permlane16_swap folds odd rows onto even rows
// for four pairs, and four DPP steps (xor 1, xor 2, half-row mirror, row mirror) finish
// each 16-lane row.  Afterwards lane 16 r + k (k < 4) holds the total of value 4 r + k.
// Needs all 64 lanes active.
template <int CTRL>
__device__ __forceinline__ float dpp_add(float v)
{
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ float swap32_add(float x, float y)
{
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap16_add(float x, float y)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float wave_sum16(const float (&g)[16], int lane)
{
    float a[8], b[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = swap32_add(g[i], g[i + 8]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float v = swap16_add(a[i], a[i + 4]);
        v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]
        v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]
        v = dpp_add<0x141>(v);  // row_half_mirror
        v = dpp_add<0x140>(v);  // row_mirror
        b[i] = v;
    }
    const int k = lane & 15;
    float r = b[0];
    r = k == 1 ? b[1] : r;
    r = k == 2 ? b[2] : r;
    r = k == 3 ? b[3] : r;
    return r;
}

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ __launch_bounds__(64) void raster_bwd_chunk_kernel(
    const uint4 *__restrict__ chunks, const uint32_t *__restrict__ n_items, const uint32_t *__restrict__ ids,
    const float *__restrict__ recs, const uint2 *__restrict__ rects, const float *__restrict__ rows,
    const float *__restrict__ cols, Grid g, RasterParams p, const float *__restrict__ slots,
    const float4 *__restrict__ st0, const float4 *__restrict__ st1, const float *__restrict__ gDp,
    const float *__restrict__ gAp, const float *__restrict__ gNp, const float4 *__restrict__ fixA,
    const float4 *__restrict__ fixB, const uint64_t *__restrict__ kmask, float *__restrict__ recgrad)
{
    __shared__ WaveStage ws;
    const uint32_t task = task_of(blockIdx.x), item = task >> 2;
    if (item >= *n_items) return;
    // lanes without a composite in this chunk have nothing to propagate
    const uint64_t km = kmask[task];
    if (km == 0ull) return;
    const uint4 ch = uniform_chunk(chunks, item);
    const Lane L = lane_of((int)ch.x, g, (int)((task & 3u) * 64u + threadIdx.x));
    Ray ray = make_ray(rows, cols, L.valid ? L.k : 0, L.valid ? L.j : 0);
    int last = -1;
    float T = 1.f, B = 0.f, gbD = 0.f, gbN0 = 0.f, gbN1 = 0.f, gbN2 = 0.f, gbA = 0.f;
    if (km >> L.lane & 1ull) {
        last = __float_as_int(slots[slot(item, F_LAST, L.rt)]);
        if (last >= 0) {
            // effective upstream gradients of the ray, and B at the end of the chunk from the
            // sums of the later chunks: the merge's suffix, plus the sums of a later chunk that
            // a fix-up re-walked; the fix-up chunk itself is the ray's last (B = 0)
            const int r = L.k * g.W + L.j;
            T = slots[slot(item, F_TEND, L.rt)];
            float sA = slots[slot(item, F_SA, L.rt)], sD = slots[slot(item, F_SD, L.rt)];
            float s0 = slots[slot(item, F_SN0, L.rt)], s1 = slots[slot(item, F_SN1, L.rt)];
            float s2 = slots[slot(item, F_SN2, L.rt)];
            const float4 a = st0[r], b = st1[r], fa = fixA[r], fb = fixB[r];
            const float gd = gDp[r], ga = gAp[r];
            const float gn0 = gNp[3 * r], gn1 = gNp[3 * r + 1], gn2 = gNp[3 * r + 2];
            const float iA = 1.f / a.x;
            gbD = gd * iA;
            gbN0 = gn0 * iA;
            gbN1 = gn1 * iA;
            gbN2 = gn2 * iA;
            gbA = ga - (gd * a.y + gn0 * b.x + gn1 * b.y + gn2 * b.z) * iA;
            const int fx = __float_as_int(fb.w);
            if ((int)item < fx) {
                sA += fa.x;
                sD += fa.y;
                s0 += fa.z;
                s1 += fa.w;
                s2 += fb.x;
            }
            if ((int)item != fx)
                B = fmaf(gbD, sD, fmaf(gbN0, s0, fmaf(gbN1, s1, fmaf(gbN2, s2, gbA * sA))));
        }
    }
    const int wmax = wave_max_i(last);
    if (wmax < 0) return;  // nothing to propagate
    const uint32_t a = ch.y, b = ch.z;
    const uint32_t nstages = (b - a + kWStage - 1) / kWStage;
    for (uint32_t sidx = nstages; sidx-- > 0;) {
        const uint32_t base = a + sidx * kWStage;
        if (wmax < (int)base) continue;
        uint32_t slot_pos, slot_id;
        const uint32_t m = stage_wave(ws, ids, recs, rects, base, min((uint32_t)kWStage, b - base), L, g.W,
                                      slot_pos, slot_id);
        // staged slots up to the wave's last contributor (slots are in list order)
        const uint32_t top = (uint32_t)__popcll(__ballot((uint32_t)L.lane < m && (int)slot_pos <= wmax));
        for (uint32_t i = top; i-- > 0;) {
            const int pos = __builtin_amdgcn_readlane((int)slot_pos, (int)i);
            const Rec s = staged_rec(ws, i);
            // every lane tests; the wave goes on only if some lane composites this entry, and
            // then runs the composite arithmetic on full waves, keeping its results (the
            // recurrence of T and B, the 15 gradient values) on the contributing lanes only
            Hit h;
            const float q2 = hit_geom(h, s, ray, p);
            if (!__any(pos <= last && h.pass)) continue;  // no lane reaches the opacity test
            hit_opacity(h, q2, s, p);
            const bool contrib = pos <= last && h.pass;
            if (!__any(contrib)) continue;
            const float one_m = 1.f - h.ah;
            const float r1m = __builtin_amdgcn_rcpf(one_m);
            const float Tj = T * r1m;
            const float w = Tj * h.ah;
            const float cj = fmaf(gbD, h.t, fmaf(gbN0, s.nt0, fmaf(gbN1, s.nt1, fmaf(gbN2, s.nt2, gbA))));
            const float dah = fmaf(Tj, cj, -B * r1m);
            const float Bn = fmaf(w, cj, B);
            T = contrib ? Tj : T;
            B = contrib ? Bn : B;
            // Lanes that do not composite this entry get zero weight, dL/dalpha_hat, G and 1/den,
            // so every gradient value below is zero there (the other factors, the direction
            // residual e, nu, nv and the record, are finite on every lane), without masking
            // each of them.  A clamped alpha_hat passes no gradient to alpha and G.
            const float wc = contrib ? w : 0.f;
            const float dahc = contrib && h.aG < p.alpha_max ? dah : 0.f;
            const float inv = contrib ? h.inv : 0.f, G = contrib ? h.G : 0.f;
            const float dt = gbD * wc;
            const float dalpha = dahc * G, dG = dahc * s.alpha;
            const float dq2 = -0.5f * G * dG;
            const float u = h.nu * inv, v = h.nv * inv, t = s.c * inv;
            const float du = 2.f * u * dq2, dv = 2.f * v * dq2;
            const float dnu = du * inv, dnv = dv * inv;
            // dL/dden through u and v; the path through t goes along e and into G_CM
            const float dduv = -fmaf(du, u, dv * v) * inv;
            const float gc = dt * inv, gte = gc * t, gci = gc * inv;
            const float nte = fmaf(s.nt0, h.e[0], fmaf(s.nt1, h.e[1], s.nt2 * h.e[2]));
            float gv[16];
            gv[G_NT + 0] = fmaf(gbN0, wc, fmaf(dduv, ray.dh[0], -gte * h.e[0]));
            gv[G_NT + 1] = fmaf(gbN1, wc, fmaf(dduv, ray.dh[1], -gte * h.e[1]));
            gv[G_NT + 2] = fmaf(gbN2, wc, fmaf(dduv, ray.dh[2], -gte * h.e[2]));
            gv[G_C] = gc;
            gv[G_CM] = gci * nte;
            gv[G_CI] = gci;
            gv[G_CU] = dnu;
            gv[G_U + 0] = dnu * h.e[0];
            gv[G_U + 1] = dnu * h.e[1];
            gv[G_U + 2] = dnu * h.e[2];
            gv[G_CV] = dnv;
            gv[G_V + 0] = dnv * h.e[0];
            gv[G_V + 1] = dnv * h.e[1];
            gv[G_V + 2] = dnv * h.e[2];
            gv[G_ALPHA] = dalpha;
#pragma unroll
            for (int c = kGradUsed; c < 16; ++c) gv[c] = 0.f;
            const uint32_t sid = (uint32_t)__builtin_amdgcn_readlane((int)slot_id, (int)i);
            const uint64_t cm = __builtin_amdgcn_ballot_w64(contrib);
            if ((cm & (cm - 1ull)) == 0ull) {
                // one contributing lane: its values are the sums; lane c takes value c
                const int src = (int)__builtin_ctzll(cm);
                float mine = 0.f;
#pragma unroll
                for (int c = 0; c < kGradUsed; ++c) {
                    const float x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(gv[c]), src));
                    mine = L.lane == c ? x : mine;
                }
                if (L.lane < kGradUsed) unsafeAtomicAdd(recgrad + (size_t)sid * kGrad + L.lane, mine);
            } else {
                const float mine = wave_sum16(gv, L.lane);
                const int k = L.lane & 15, c = 4 * (L.lane >> 4) + k;
                if (k < 4 && c < kGradUsed) unsafeAtomicAdd(recgrad + (size_t)sid * kGrad + c, mine);
            }
        }
        __syncthreads();  // the stage is no longer read
    }
}

// ---------------------------------------------------------------------------------------
// work counter (query only)
// ---------------------------------------------------------------------------------------

// out += ray tests a front-to-back walk needs: per wave sub-tile, 64 per list entry that
// overlaps it, up to the last contributor of its slowest ray (the whole list when a ray
// never falls below T_min).  One workgroup per tile, after the forward.
__global__ __launch_bounds__(256) void work_needed_kernel(const uint32_t *__restrict__ chunk_base,
                                                          const uint32_t *__restrict__ ids,
                                                          const uint2 *__restrict__ rects,
                                                          const uint2 *__restrict__ ranges, Grid g, RasterParams p,
                                                          const float *__restrict__ slots,
                                                          const uint64_t *__restrict__ kmask,
                                                          const float4 *__restrict__ st0,
                                                          unsigned long long *__restrict__ out)
{
    const int tile = blockIdx.x;
    const Lane L = lane_of(tile, g);
    const uint2 rg = ranges[tile];
    int need = -1;
    if (L.valid) {
        const uint32_t c0 = chunk_base[tile], c1 = chunk_base[tile + 1];
        int last = -1;
        for (uint32_t it = c0; it < c1; ++it)
            if (kmask[(size_t)it * 4 + L.wave] >> L.lane & 1ull)
                last = max(last, __float_as_int(slots[slot(it, F_LAST, L.rt)]));
        const bool dead = st0[L.k * g.W + L.j].z < p.T_min;
        need = dead ? last : (int)rg.y - 1;
    }
    need = wave_max_i(need);
    unsigned long long c = 0;
    if (need >= 0) {
        const int r16 = L.sr0, c16 = L.sc0;
        const uint32_t end = min((uint32_t)need + 1u, rg.y);
        for (uint32_t pos = rg.x + (uint32_t)L.lane; pos < end; pos += 64u)
            c += sub_overlap(rects[ids[pos]], r16, c16, g.W) ? 64ull : 0ull;
    }
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    if (L.lane == 0 && c) atomicAdd(out, c);
}

// out[0] += per ray, the list entries that pass every per-hit test (cut-off, alpha_thr, near,
// den_eps) whether or not the ray has stopped compositing before them; out[1] += rays with at
// least one.  One workgroup per tile, one ray per thread, records read straight from memory
// (query only, not on the rendering path).
__global__ __launch_bounds__(256) void count_hits_kernel(const uint32_t *__restrict__ ids,
                                                         const float *__restrict__ recs,
                                                         const uint2 *__restrict__ rects,
                                                         const uint2 *__restrict__ ranges,
                                                         const float *__restrict__ rows,
                                                         const float *__restrict__ cols, Grid g, RasterParams p,
                                                         unsigned long long *__restrict__ out)
{
    const int tile = blockIdx.x;
    const Lane L = lane_of(tile, g);
    const uint2 rg = ranges[tile];
    unsigned long long c = 0;
    if (L.wave_in) {
        const Ray ray = make_ray(rows, cols, L.valid ? L.k : 0, L.valid ? L.j : 0);
        for (uint32_t pos = rg.x; pos < rg.y; ++pos) {
            const uint32_t id = ids[pos];
            if (!sub_overlap(rects[id], L.sr0, L.sc0, g.W)) continue;
            const Hit h = hit_test(load_rec(recs, id), ray, p);
            c += (L.valid && h.pass) ? 1ull : 0ull;
        }
    }
    unsigned long long hit = c > 0 ? 1ull : 0ull;
    for (int o = 32; o >= 1; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        hit += __shfl_xor(hit, o, 64);
    }
    if (L.lane == 0) {
        if (c) atomicAdd(out, c);
        if (hit) atomicAdd(out + 1, hit);
    }
}

// ---------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------

int chunk_size(int64_t P, int requested)
{
    if (requested > 0) return requested;
    // about 8192 chunks, 32768 one-wave tasks (several rounds of 8 resident waves on each of
    // 1024 SIMDs; short chunks also keep the re-walk of a terminating ray short), balanced
    // against the per-chunk cost of the merge; at most kChunkMax
    int64_t s = (P + 8191) / 8192;
    s = (s + 15) / 16 * 16;
    if (s < 32) s = 32;
    if (s > kChunkMax) s = kChunkMax;
    return (int)s;
}

int64_t chunk_items_max(int64_t P, int T, int seg) { return (int64_t)T + (P + seg - 1) / seg; }

size_t chunk_slot_floats(int64_t items_max) { return (size_t)items_max * kSlotFields * 256; }

hipError_t launch_raster_fwd(const RasterBufs &R, const Grid &g, const RasterParams &p, float *depth,
                             float *opacity, float *normal, uint8_t *drop, hipStream_t s)
{
    if (g.T <= 0) return hipSuccess;
    const int im = (int)R.items_max;
    if (im > 0)
        raster_fwd_chunk_kernel<<<task_blocks(im), 64, 0, s>>>(R.chunks, R.n_items, R.ids, R.recs, R.rects, R.rows,
                                                               R.cols, g, p, R.slots, R.kmask);
    const int ng = merge_groups(g.T);
    raster_merge_kernel<<<g.T, 256 * ng, (size_t)ng * kMergeRunFloats * sizeof(float), s>>>(
        R.chunk_base, g, p, R.slots, depth, opacity, normal, drop, R.st0, R.st1, R.fixA, R.fixB, R.fixflag, R.kmask);
    if (im > 0)
        raster_fixup_kernel<<<task_blocks(im), 64, 0, s>>>(R.chunks, R.n_items, R.ids, R.recs, R.rects, R.rows,
                                                           R.cols, g, p, R.fixA, R.fixB, R.slots, depth, opacity,
                                                           normal, drop, R.st0, R.st1, R.fixflag);
    return hipGetLastError();
}

hipError_t launch_raster_fwd_multi(FwdJobs &J, const RasterParams &p, hipStream_t s)
{
    if (J.n <= 0) return hipSuccess;
    uint32_t blocks = 0, tiles = 0;
    for (int k = 0; k < J.n; ++k) {
        J.j[k].block0 = blocks;
        J.j[k].tile0 = tiles;
        blocks += J.j[k].R.items_max > 0 && J.j[k].g.T > 0 ? task_blocks((int)J.j[k].R.items_max) : 0u;
        tiles += (uint32_t)(J.j[k].g.T > 0 ? J.j[k].g.T : 0);
    }
    if (blocks > 0) raster_fwd_chunk_multi<<<blocks, 64, 0, s>>>(J, p);
    if (tiles > 0) {
        const int ng = kMergeGroups;
        raster_merge_multi<<<tiles, 256 * ng, (size_t)ng * kMergeRunFloats * sizeof(float), s>>>(J, p);
    }
    if (blocks > 0) raster_fixup_multi<<<blocks, 64, 0, s>>>(J, p);
    return hipGetLastError();
}

hipError_t launch_work_needed(const RasterBufs &R, const Grid &g, const RasterParams &p, unsigned long long *out,
                              hipStream_t s)
{
    work_needed_kernel<<<g.T, 256, 0, s>>>(R.chunk_base, R.ids, R.rects, R.ranges, g, p, R.slots, R.kmask, R.st0,
                                           out);
    return hipGetLastError();
}

hipError_t launch_count_hits(const RasterBufs &R, const Grid &g, const RasterParams &p, unsigned long long *out,
                             hipStream_t s)
{
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(out), 0u, 4, s);
    if (e != hipSuccess || g.T <= 0) return e;
    count_hits_kernel<<<g.T, 256, 0, s>>>(R.ids, R.recs, R.rects, R.ranges, R.rows, R.cols, g, p, out);
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const RasterBufs &R, const Grid &g, const RasterParams &p, const float *gD,
                             const float *gA, const float *gN, float *recgrad, hipStream_t s)
{
    const int im = (int)R.items_max;
    if (g.T <= 0 || im <= 0) return hipSuccess;
    raster_bwd_chunk_kernel<<<task_blocks(im), 64, 0, s>>>(R.chunks, R.n_items, R.ids, R.recs, R.rects, R.rows,
                                                           R.cols, g, p, R.slots, R.st0, R.st1, gD, gA, gN, R.fixA,
                                                           R.fixB, R.kmask, recgrad);
    return hipGetLastError();
}

}  // namespace lgsr
