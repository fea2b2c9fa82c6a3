// sort.hip -- tile offsets and the per-tile front-to-back order of the pair lists.
//
// Emission writes each tile's surfel ids into the tile's bucket in no particular order.
// The compositing order of Sec. 3.4 (ascending sensor range, ties by surfel index) is then
// established per tile by one workgroup: a least-significant-digit radix sort with 9-bit
// digits on (range bits - tile minimum), stable within the workgroup, kept in registers and
// LDS when the list fits (kTsCap entries) and streamed through the two spare pair buffers
// otherwise.  Equal range keys are put in index order by sorting on the index first and
// then again on the range (both passes stable), which happens only for tiles that hold
// exactly equal ranges.
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

constexpr int kTsThreads = 1024;
constexpr int kTsWaves = kTsThreads / 64;
constexpr int kTsItems = 8;
constexpr int kTsCap = kTsThreads * kTsItems;  // entries sorted without leaving the CU
constexpr int kDigitBits = 9;
constexpr int kDigits = 1 << kDigitBits;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Lanes of the wave (among `valid` ones) holding the same digit as this lane.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid)
{
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kDigitBits; ++b) {
        const uint64_t m = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? m : ~m;
    }
    return valid ? peers : 0ull;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(v, o, 64);
        if (l >= o) v += y;
    }
    return v;
}

struct TileSortSmem {
    uint32_t key[kTsCap + 1];  // the extra slot takes writes of lanes without an entry
    uint32_t val[kTsCap + 1];
    uint16_t wcnt[kTsWaves][kDigits];  // per wave digit counts, then their prefix over waves
    uint32_t dbase[kDigits];
    uint32_t wsum[kTsWaves];
    uint32_t red[kTsWaves][4];
};

__device__ __forceinline__ uint32_t digit_of(uint32_t x, uint32_t base, int shift)
{
    return ((x - base) >> shift) & (uint32_t)(kDigits - 1);
}

// Exclusive scan over the workgroup of one value per thread (threads >= kDigits pass 0).
// Ends with a barrier.
__device__ __forceinline__ uint32_t block_excl_scan(TileSortSmem &sm, uint32_t v)
{
    const int t = threadIdx.x, w = t >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (lane_id() == 63) sm.wsum[w] = inc;
    __syncthreads();
    uint32_t ws[kTsWaves];
#pragma unroll
    for (int k = 0; k < kTsWaves; ++k) ws[k] = sm.wsum[k];
    uint32_t off = 0;
#pragma unroll
    for (int k = 0; k < kTsWaves; ++k) off += k < w ? ws[k] : 0u;
    __syncthreads();
    return off + inc - v;
}

// Stable ranking of a chunk of m <= kTsCap entries held as element j = (w R + r) 64 + lane.
// On return off[r] is the entry's position among the entries of its wave with the same
// digit (in j order), sm.wcnt[w][d] holds the number of digit-d entries in waves before w,
// and thread t < kDigits returns the chunk's count of digit t.  Ends with a barrier.
__device__ __forceinline__ uint32_t rank_chunk(TileSortSmem &sm, const uint32_t *kx, const uint32_t *vx,
                                               uint32_t *off, int m, int R, bool by_val, uint32_t base, int shift)
{
    const int t = threadIdx.x, w = t >> 6;
    uint32_t *wc32 = reinterpret_cast<uint32_t *>(&sm.wcnt[0][0]);
    for (int i = t; i < kTsWaves * kDigits / 2; i += kTsThreads) wc32[i] = 0u;
    __syncthreads();
    const int j0 = w * R * 64 + lane_id();
#pragma unroll
    for (int r = 0; r < kTsItems; ++r) {
        if (r < R) {
            const bool valid = j0 + r * 64 < m;
            const uint32_t d = digit_of(by_val ? vx[r] : kx[r], base, shift);
            const uint64_t peers = match_digit(d, valid);
            const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
            // the wave's LDS accesses execute in order: every lane of the digit reads the
            // count before its first lane stores the new one
            const uint32_t before = sm.wcnt[w][d];
            if (valid && rank == 0) sm.wcnt[w][d] = (uint16_t)(before + (uint32_t)__popcll(peers));
            off[r] = before + rank;
        }
        // keep the rounds apart: hoisting every round's ballots together exhausts SGPRs
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    uint32_t total = 0;
    if (t < kDigits) {
        uint32_t c[kTsWaves];
#pragma unroll
        for (int v = 0; v < kTsWaves; ++v) c[v] = sm.wcnt[v][t];
#pragma unroll
        for (int v = 0; v < kTsWaves; ++v) {
            sm.wcnt[v][t] = (uint16_t)total;
            total += c[v];
        }
    }
    __syncthreads();
    return total;
}

__device__ __forceinline__ void block_minmax(TileSortSmem &sm, uint32_t &kmin, uint32_t &kmax, uint32_t &vmin,
                                             uint32_t &vmax)
{
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor(kmin, o, 64));
        kmax = max(kmax, (uint32_t)__shfl_xor(kmax, o, 64));
        vmin = min(vmin, (uint32_t)__shfl_xor(vmin, o, 64));
        vmax = max(vmax, (uint32_t)__shfl_xor(vmax, o, 64));
    }
    if (lane_id() == 0) {
        sm.red[w][0] = kmin;
        sm.red[w][1] = kmax;
        sm.red[w][2] = vmin;
        sm.red[w][3] = vmax;
    }
    __syncthreads();
    kmin = sm.red[0][0];
    kmax = sm.red[0][1];
    vmin = sm.red[0][2];
    vmax = sm.red[0][3];
    for (int k = 1; k < kTsWaves; ++k) {
        kmin = min(kmin, sm.red[k][0]);
        kmax = max(kmax, sm.red[k][1]);
        vmin = min(vmin, sm.red[k][2]);
        vmax = max(vmax, sm.red[k][3]);
    }
    __syncthreads();
}

__device__ __forceinline__ int passes_for(uint32_t lo, uint32_t hi)
{
    if (hi <= lo) return 0;
    const int bits = 32 - __clz((int)(hi - lo));
    return (bits + kDigitBits - 1) / kDigitBits;
}

// ---- resident path: the whole list in registers, exchanged through LDS ----

__device__ __forceinline__ void resident_pass(TileSortSmem &sm, uint32_t *kx, uint32_t *vx, int m, int R,
                                              bool by_val, uint32_t base, int shift)
{
    const int t = threadIdx.x, w = t >> 6;
    uint32_t off[kTsItems];
    const uint32_t total = rank_chunk(sm, kx, vx, off, m, R, by_val, base, shift);
    const uint32_t excl = block_excl_scan(sm, t < kDigits ? total : 0u);
    if (t < kDigits) sm.dbase[t] = excl;
    __syncthreads();
    const int j0 = w * R * 64 + lane_id();
#pragma unroll
    for (int r = 0; r < kTsItems; ++r) {
        if (r < R) {
            const uint32_t d = digit_of(by_val ? vx[r] : kx[r], base, shift);
            uint32_t dst = min(sm.dbase[d] + (uint32_t)sm.wcnt[w][d] + off[r], (uint32_t)(kTsCap - 1));
            dst = j0 + r * 64 < m ? dst : (uint32_t)kTsCap;
            sm.key[dst] = kx[r];
            sm.val[dst] = vx[r];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTsItems; ++r) {
        if (r < R) {
            const int j = min(j0 + r * 64, m - 1);
            kx[r] = sm.key[j];
            vx[r] = sm.val[j];
        }
    }
}

// true if two neighbouring entries of the (sorted) list share a range key
__device__ __forceinline__ bool resident_has_ties(TileSortSmem &sm, const uint32_t *kx, int m, int R)
{
    const int j0 = (threadIdx.x >> 6) * R * 64 + lane_id();
    bool tie = false;
#pragma unroll
    for (int r = 0; r < kTsItems; ++r) {
        if (r < R) {
            const int j = j0 + r * 64;
            const uint32_t prev = sm.key[min(max(j - 1, 0), m - 1)];
            tie |= j < m && j > 0 && prev == kx[r];
        }
    }
    return __syncthreads_or(tie) != 0;
}

__device__ void sort_resident(TileSortSmem &sm, const uint32_t *__restrict__ keys, int64_t n,
                              uint32_t *__restrict__ ids, int m)
{
    const int w = threadIdx.x >> 6;
    const int R = (m + kTsThreads - 1) / kTsThreads;
    const int j0 = w * R * 64 + lane_id();
    uint32_t kx[kTsItems], vx[kTsItems];
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u, vmin = 0xFFFFFFFFu, vmax = 0u;
    // all loads of a phase are issued before any result is used (no per-lane branches)
#pragma unroll
    for (int r = 0; r < kTsItems; ++r) vx[r] = r < R ? ids[min(j0 + r * 64, m - 1)] : 0u;
#pragma unroll
    for (int r = 0; r < kTsItems; ++r) kx[r] = r < R && (int64_t)vx[r] < n ? keys[vx[r]] : 0xFFFFFFFFu;
#pragma unroll
    for (int r = 0; r < kTsItems; ++r) {
        if (r < R) {
            const int j = j0 + r * 64;
            sm.key[j < m ? j : kTsCap] = kx[r];
            if (j < m) {
                kmin = min(kmin, kx[r]);
                kmax = max(kmax, kx[r]);
                vmin = min(vmin, vx[r]);
                vmax = max(vmax, vx[r]);
            }
        }
    }
    block_minmax(sm, kmin, kmax, vmin, vmax);  // its barriers also publish sm.key
    const int kp = passes_for(kmin, kmax);
    for (int q = 0; q < kp; ++q) resident_pass(sm, kx, vx, m, R, false, kmin, q * kDigitBits);
    if (resident_has_ties(sm, kx, m, R)) {
        const int vp = passes_for(vmin, vmax);
        for (int q = 0; q < vp; ++q) resident_pass(sm, kx, vx, m, R, true, vmin, q * kDigitBits);
        for (int q = 0; q < kp; ++q) resident_pass(sm, kx, vx, m, R, false, kmin, q * kDigitBits);
    }
#pragma unroll
    for (int r = 0; r < kTsItems; ++r) {
        const int j = j0 + r * 64;
        if (r < R && j < m) ids[j] = vx[r];
    }
}

// ---- streaming path: lists longer than kTsCap, one workgroup, chunks through LDS ----

// Global writes of one phase become visible to the workgroup's reads of the next.
__device__ __forceinline__ void phase_barrier()
{
    __threadfence();
    __syncthreads();
    __threadfence();
}

__device__ void stream_pass(TileSortSmem &sm, const uint32_t *sk, const uint32_t *sv, uint32_t *dk, uint32_t *dv,
                            int m, bool by_val, uint32_t base, int shift)
{
    const int t = threadIdx.x, w = t >> 6;
    for (int i = t; i < kDigits; i += kTsThreads) sm.dbase[i] = 0u;
    __syncthreads();
    for (int j = t; j < m; j += kTsThreads) atomicAdd(&sm.dbase[digit_of(by_val ? sv[j] : sk[j], base, shift)], 1u);
    __syncthreads();
    uint32_t run = t < kDigits ? sm.dbase[t] : 0u;
    run = block_excl_scan(sm, run);
    for (int c0 = 0; c0 < m; c0 += kTsCap) {
        const int mc = min(kTsCap, m - c0);
        const int R = (mc + kTsThreads - 1) / kTsThreads;
        const int j0 = w * R * 64 + lane_id();
        uint32_t kx[kTsItems], vx[kTsItems], off[kTsItems];
#pragma unroll
        for (int r = 0; r < kTsItems; ++r) {
            const int j = j0 + r * 64;
            const bool ok = r < R && j < mc;
            kx[r] = ok ? sk[c0 + j] : 0u;
            vx[r] = ok ? sv[c0 + j] : 0u;
        }
        const uint32_t total = rank_chunk(sm, kx, vx, off, mc, R, by_val, base, shift);
        if (t < kDigits) sm.dbase[t] = run;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kTsItems; ++r) {
            if (r < R && j0 + r * 64 < mc) {
                const uint32_t d = digit_of(by_val ? vx[r] : kx[r], base, shift);
                const uint32_t dst = min(sm.dbase[d] + (uint32_t)sm.wcnt[w][d] + off[r], (uint32_t)(m - 1));
                dk[dst] = kx[r];
                dv[dst] = vx[r];
            }
        }
        if (t < kDigits) run += total;
        __syncthreads();
    }
    phase_barrier();
}

__device__ void sort_streaming(TileSortSmem &sm, const uint32_t *__restrict__ keys, int64_t n, uint32_t *ids,
                               uint32_t *k0, uint32_t *k1, uint32_t *v1, int m)
{
    const int t = threadIdx.x;
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u, vmin = 0xFFFFFFFFu, vmax = 0u;
    for (int j = t; j < m; j += kTsThreads) {
        const uint32_t v = ids[j], k = (int64_t)v < n ? keys[v] : 0xFFFFFFFFu;
        k0[j] = k;
        kmin = min(kmin, k);
        kmax = max(kmax, k);
        vmin = min(vmin, v);
        vmax = max(vmax, v);
    }
    block_minmax(sm, kmin, kmax, vmin, vmax);
    phase_barrier();
    // (k0, ids) and (k1, v1) alternate as source and destination
    uint32_t *sk = k0, *sv = ids, *dk = k1, *dv = v1;
    auto pass = [&](bool by_val, uint32_t base, int shift) {
        stream_pass(sm, sk, sv, dk, dv, m, by_val, base, shift);
        uint32_t *a = sk, *b = sv;
        sk = dk;
        sv = dv;
        dk = a;
        dv = b;
    };
    const int kp = passes_for(kmin, kmax);
    for (int q = 0; q < kp; ++q) pass(false, kmin, q * kDigitBits);
    bool tie = false;
    for (int j = t + 1; j < m; j += kTsThreads) tie |= sk[j - 1] == sk[j];
    if (__syncthreads_or(tie)) {
        const int vp = passes_for(vmin, vmax);
        for (int q = 0; q < vp; ++q) pass(true, vmin, q * kDigitBits);
        for (int q = 0; q < kp; ++q) pass(false, kmin, q * kDigitBits);
    }
    if (sv != ids) {
        for (int j = t; j < m; j += kTsThreads) ids[j] = sv[j];
    }
}

// One workgroup per tile; lists longer than kTsCap are left to tile_sort_stream_kernel.
__global__ __launch_bounds__(kTsThreads) void tile_sort_kernel(const uint2 *__restrict__ ranges, int T,
                                                               const uint32_t *__restrict__ keys, int64_t n,
                                                               uint32_t *ids)
{
    __shared__ TileSortSmem sm;
    const int tile = blockIdx.x;
    if (tile >= T) return;
    const uint2 rg = ranges[tile];
    const int m = (int)(rg.y - rg.x);
    if (m <= 1 || m > kTsCap) return;
    sort_resident(sm, keys, n, ids + rg.x, m);
}

__global__ __launch_bounds__(kTsThreads) void tile_sort_stream_kernel(const uint2 *__restrict__ ranges, int T,
                                                                      const uint32_t *__restrict__ keys, int64_t n,
                                                                      uint32_t *ids, uint32_t *k0, uint32_t *k1,
                                                                      uint32_t *v1)
{
    __shared__ TileSortSmem sm;
    const int tile = blockIdx.x;
    if (tile >= T) return;
    const uint2 rg = ranges[tile];
    const int m = (int)(rg.y - rg.x);
    if (m <= kTsCap) return;
    sort_streaming(sm, keys, n, ids + rg.x, k0 + rg.x, k1 + rg.x, v1 + rg.x, m);
}

// ---- tile offsets ----

// One workgroup.  cnt holds kShards counts per tile; with o the exclusive prefix sum of all
// counts in (tile, shard) order: cursor[t kShards + s] = o at that entry, ranges[t] = (o at
// (t, 0), o at (t + 1, 0)); out[0..1] = total (64-bit), out[2] = largest tile count.
__global__ __launch_bounds__(1024) void tile_scan_kernel(const uint32_t *__restrict__ cnt, int T,
                                                         uint2 *__restrict__ ranges, uint32_t *__restrict__ cursor,
                                                         uint32_t *__restrict__ out)
{
    static_assert(kShards == 8, "two uint4 loads per tile");
    __shared__ uint64_t wsum[16];
    __shared__ uint32_t wmax[16];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    uint64_t carry = 0;
    uint32_t mx = 0;
    for (int first = 0; first < T; first += 1024) {
        const int tile = first + t;
        uint4 a = make_uint4(0u, 0u, 0u, 0u), b = a;
        if (tile < T) {
            const uint4 *p = reinterpret_cast<const uint4 *>(cnt + (size_t)tile * kShards);
            a = p[0];
            b = p[1];
        }
        const uint32_t x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        uint64_t s = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) s += x[k];
        mx = max(mx, (uint32_t)min(s, (uint64_t)0xFFFFFFFFu));
        uint64_t inc = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t y = __shfl_up(inc, o, 64);
            if (l >= o) inc += y;
        }
        if (l == 63) wsum[w] = inc;
        __syncthreads();
        uint64_t off = carry, tot = 0;
        for (int k = 0; k < 16; ++k) {
            const uint64_t v = wsum[k];
            off += k < w ? v : 0;
            tot += v;
        }
        __syncthreads();
        off += inc - s;
        if (tile < T) {
            const uint32_t o0 = (uint32_t)off;
            uint32_t c[8];
            uint32_t o = o0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                c[k] = o;
                o += x[k];
            }
            uint4 *q = reinterpret_cast<uint4 *>(cursor + (size_t)tile * kShards);
            q[0] = make_uint4(c[0], c[1], c[2], c[3]);
            q[1] = make_uint4(c[4], c[5], c[6], c[7]);
            ranges[tile] = make_uint2(o0, o);
        }
        carry += tot;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
    if (l == 0) wmax[w] = mx;
    __syncthreads();
    if (t == 0) {
        for (int k = 1; k < 16; ++k) mx = max(mx, wmax[k]);
        out[0] = (uint32_t)carry;
        out[1] = (uint32_t)(carry >> 32);
        out[2] = mx;
    }
}

// ---------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------

int tile_sort_capacity() { return kTsCap; }

hipError_t launch_tile_scan(const uint32_t *cnt, int T, uint2 *ranges, uint32_t *cursor, uint32_t *out,
                            hipStream_t s)
{
    tile_scan_kernel<<<1, 1024, 0, s>>>(cnt, T, ranges, cursor, out);
    return hipGetLastError();
}

hipError_t launch_tile_sort(const uint2 *ranges, int T, const uint32_t *keys, int64_t n, uint32_t *ids, uint32_t *k0,
                            uint32_t *k1, uint32_t *v1, hipStream_t s)
{
    if (T <= 0) return hipSuccess;
    tile_sort_kernel<<<T, kTsThreads, 0, s>>>(ranges, T, keys, n, ids);
    if (k0 && k1 && v1) tile_sort_stream_kernel<<<T, kTsThreads, 0, s>>>(ranges, T, keys, n, ids, k0, k1, v1);
    return hipGetLastError();
}

}  // namespace lgsr
