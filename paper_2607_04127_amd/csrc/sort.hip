// sort.hip -- tile offsets and the per-tile front-to-back order of the pair lists.
//
// Emission writes each tile's surfel ids into the tile's bucket in no particular order.
// The compositing order of Sec. 3.4 (ascending sensor range, ties by surfel index) is then
// established per tile by one workgroup: a least-significant-digit radix sort with 9-bit
// digits on (range bits - tile minimum), stable within the workgroup, kept in registers and
// LDS (up to kTsCap entries).  Equal range keys are put in index order by sorting on the
// index first and then again on the range (both passes stable), which happens only for tiles
// that hold exactly equal ranges.  A longer list is cut into kTsCap-entry chunks, each sorted
// the same way by a workgroup of its own into packed (range << 32 | index) keys; every entry
// then finds its place as its position in its chunk plus, for each other chunk, the number of
// keys below it there (a binary search).  Packed keys are unique within a tile, so the
// merged order is exactly (range, index).
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

constexpr int kTsThreads = 1024;
constexpr int kTsWaves = kTsThreads / 64;
constexpr int kTsItems = 8;
constexpr int kTsCap = kTsThreads * kTsItems;  // entries sorted without leaving the CU
constexpr int kDigitBits = 9;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kRunMax = 16;  // longest run of equal range keys ordered in place

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

// Sorts the m entries of ids (m <= kTsCap) and writes the sorted ids back into ids, or, with
// kPacked, the sorted (range << 32 | index) keys into packed instead.
template <bool kPacked>
__device__ void sort_resident(TileSortSmem &sm, const uint32_t *__restrict__ keys, int64_t n,
                              uint32_t *__restrict__ ids, int m, unsigned long long *__restrict__ packed)
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
        // Runs of equal keys are adjacent now (sm.key, sm.val hold the sorted list after a
        // pass).  Short runs are put in index order in place; a run longer than kRunMax (or a
        // list that needed no pass) takes two more sorts: by index, then again by key.
        bool long_run = kp == 0;
        for (int j = threadIdx.x; j < m && kp > 0; j += kTsThreads) {
            const uint32_t kj = sm.key[j];
            if ((j > 0 && sm.key[j - 1] == kj) || j + 1 >= m || sm.key[j + 1] != kj) continue;  // not a run start
            int len = 2;
            while (len <= kRunMax && j + len < m && sm.key[j + len] == kj) ++len;
            long_run |= len > kRunMax;
        }
        if (__syncthreads_or(long_run)) {
            const int vp = passes_for(vmin, vmax);
            for (int q = 0; q < vp; ++q) resident_pass(sm, kx, vx, m, R, true, vmin, q * kDigitBits);
            for (int q = 0; q < kp; ++q) resident_pass(sm, kx, vx, m, R, false, kmin, q * kDigitBits);
        } else {
            for (int j = threadIdx.x; j < m; j += kTsThreads) {
                const uint32_t kj = sm.key[j];
                if ((j > 0 && sm.key[j - 1] == kj) || j + 1 >= m || sm.key[j + 1] != kj) continue;
                int len = 2;
                while (j + len < m && sm.key[j + len] == kj) ++len;
                // insertion sort of the run's indices (distinct), len <= kRunMax
                for (int a = j + 1; a < j + len; ++a) {
                    const uint32_t v = sm.val[a];
                    int b = a - 1;
                    while (b >= j && sm.val[b] > v) {
                        sm.val[b + 1] = sm.val[b];
                        --b;
                    }
                    sm.val[b + 1] = v;
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kTsItems; ++r)
                if (r < R) vx[r] = sm.val[min(j0 + r * 64, m - 1)];
        }
    }
#pragma unroll
    for (int r = 0; r < kTsItems; ++r) {
        const int j = j0 + r * 64;
        if (r < R && j < m) {
            if constexpr (kPacked)
                packed[j] = ((unsigned long long)kx[r] << 32) | vx[r];
            else
                ids[j] = vx[r];
        }
    }
}

// The raster's work list (one workgroup): every tile's list cut into c = ceil(len / seg)
// chunks of nearly equal length, at most kTileChunks (a longer list gets longer chunks:
// the merge walks a tile's chunks in sequence, so its longest tile sets its time); chunk q
// of tile t = (t, first, end); chunk_base[t] = index of the tile's first chunk,
// chunk_base[T] = *n_items = the number of chunks.
// Chunks at or beyond cap_items are not written (the host sizes the buffer before it uses
// the list; a list built on too small a buffer is built again).
__device__ void build_chunks_block(const uint2 *__restrict__ ranges, int T, int seg, uint4 *__restrict__ chunks,
                                   uint32_t *__restrict__ chunk_base, uint32_t *__restrict__ n_items,
                                   int64_t cap_items)
{
    static_assert(kTsThreads == 1024, "16 waves");
    __shared__ uint32_t wsum[16];
    const int t0 = threadIdx.x, w = t0 >> 6, l = t0 & 63;
    uint32_t carry = 0;
    for (int base = 0; base < T; base += 1024) {
        const int t = base + t0;
        uint2 r = make_uint2(0u, 0u);
        uint32_t c = 0;
        if (t < T) {
            r = ranges[t];
            c = min((r.y - r.x + (uint32_t)seg - 1u) / (uint32_t)seg, (uint32_t)kTileChunks);
        }
        uint32_t inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(inc, o, 64);
            if (l >= o) inc += y;
        }
        if (l == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t off = 0, tot = 0;
        for (int q = 0; q < 16; ++q) {
            uint32_t v = wsum[q];
            if (q < w) off += v;
            tot += v;
        }
        const uint32_t first = carry + off + inc - c;
        if (t < T) {
            chunk_base[t] = first;
            const uint64_t len = r.y - r.x;
            for (uint32_t q = 0; q < c; ++q) {
                const uint32_t a = r.x + (uint32_t)(q * len / c), b = r.x + (uint32_t)((q + 1) * len / c);
                if ((int64_t)first + q < cap_items) chunks[first + q] = make_uint4((uint32_t)t, a, b, 0u);
            }
        }
        carry += tot;
        __syncthreads();
    }
    if (t0 == 0) {
        chunk_base[T] = carry;
        *n_items = carry;
    }
}

// One workgroup per tile, and one more that builds the raster's chunk list; lists longer than
// kTsCap are left to the chunk kernels below.  Lists reaching past cap_pairs (a buffer too
// small for this frame, sorted again once it has grown) are skipped; sort_lists = 0 builds
// the chunk list only.
__global__ __launch_bounds__(kTsThreads) void tile_sort_kernel(const uint2 *__restrict__ ranges, int T,
                                                               const uint32_t *__restrict__ keys, int64_t n,
                                                               uint32_t *ids, ChunkList cl, int64_t cap_pairs,
                                                               int sort_lists)
{
    __shared__ TileSortSmem sm;
    const int tile = blockIdx.x;
    if (tile == T) {
        build_chunks_block(ranges, T, cl.seg, cl.chunks, cl.chunk_base, cl.n_items, cl.cap_items);
        return;
    }
    if (tile > T || !sort_lists) return;
    const uint2 rg = ranges[tile];
    const int m = (int)(rg.y - rg.x);
    if (m <= 1 || m > kTsCap || (int64_t)rg.y > cap_pairs) return;
    sort_resident<false>(sm, keys, n, ids + rg.x, m, nullptr);
}

// ---- lists longer than kTsCap: chunk sorts, then a merge by rank ----

// Workgroup b sorts chunk b % nch of long tile b / nch (if the list has that many chunks)
// into packed keys at the chunk's own positions of tmp.
__global__ __launch_bounds__(kTsThreads) void tile_chunk_sort_kernel(const uint2 *__restrict__ ranges,
                                                                     const uint32_t *__restrict__ long_tiles, int nch,
                                                                     const uint32_t *__restrict__ keys, int64_t n,
                                                                     uint32_t *ids, unsigned long long *tmp)
{
    __shared__ TileSortSmem sm;
    const uint32_t tile = long_tiles[blockIdx.x / nch];
    const int c0 = (int)(blockIdx.x % nch) * kTsCap;
    const uint2 rg = ranges[tile];
    const int m = (int)(rg.y - rg.x);
    if (c0 >= m) return;
    sort_resident<true>(sm, keys, n, ids + rg.x + c0, min(kTsCap, m - c0), tmp + rg.x + c0);
}

// Number of the len sorted keys of a below x.
__device__ __forceinline__ int lower_bound_u64(const unsigned long long *__restrict__ a, int len,
                                               unsigned long long x)
{
    int lo = 0;
    for (int step = 1 << (31 - __clz(max(len, 1))); step > 0; step >>= 1)
        if (lo + step <= len && a[lo + step - 1] < x) lo += step;
    return lo;
}

// Workgroup b places the entries of chunk b % nch of long tile b / nch: final position =
// position in the chunk + keys below it in every other chunk.  kItems entries per thread
// search side by side.
__global__ __launch_bounds__(kTsThreads) void tile_chunk_merge_kernel(const uint2 *__restrict__ ranges,
                                                                      const uint32_t *__restrict__ long_tiles, int nch,
                                                                      const unsigned long long *__restrict__ tmp,
                                                                      uint32_t *__restrict__ ids)
{
    const uint32_t tile = long_tiles[blockIdx.x / nch];
    const int c = (int)(blockIdx.x % nch);
    const uint2 rg = ranges[tile];
    const int m = (int)(rg.y - rg.x);
    const int c0 = c * kTsCap;
    if (c0 >= m) return;
    const int mc = min(kTsCap, m - c0);
    const unsigned long long *list = tmp + rg.x;
    unsigned long long x[kTsItems];
    int pos[kTsItems];
#pragma unroll
    for (int r = 0; r < kTsItems; ++r) {
        const int j = (int)threadIdx.x + r * kTsThreads;
        x[r] = j < mc ? list[c0 + j] : 0ull;
        pos[r] = j;
    }
    const int chunks = (m + kTsCap - 1) / kTsCap;
    for (int o = 0; o < chunks; ++o) {
        if (o == c) continue;
        const int len = min(kTsCap, m - o * kTsCap);
#pragma unroll
        for (int r = 0; r < kTsItems; ++r) pos[r] += lower_bound_u64(list + o * kTsCap, len, x[r]);
    }
#pragma unroll
    for (int r = 0; r < kTsItems; ++r) {
        const int j = (int)threadIdx.x + r * kTsThreads;
        if (j < mc) ids[rg.x + pos[r]] = (uint32_t)x[r];
    }
}

// ---- tile offsets ----

// One workgroup.  cnt holds kShards counts per tile; with o the exclusive prefix sum of all
// counts in (tile, shard) order: cursor[t kShards + s] = o at that entry, ranges[t] = (o at
// (t, 0), o at (t + 1, 0)); the counts are left zero; out[0..1] = total (64-bit), out[2] =
// largest tile count, out[3] =
// number of tiles with more than kTsCap entries, listed (in no particular order) in
// long_tiles.
__global__ __launch_bounds__(1024) void tile_scan_kernel(uint32_t *__restrict__ cnt, int T,
                                                         uint2 *__restrict__ ranges, uint32_t *__restrict__ cursor,
                                                         uint32_t *__restrict__ out, uint32_t *__restrict__ long_tiles,
                                                         uint32_t *__restrict__ host_out)
{
    static_assert(kShards == 8, "two uint4 loads per tile");
    __shared__ uint64_t wsum[16];
    __shared__ uint32_t wmax[16];
    __shared__ uint32_t nlong;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    if (t == 0) nlong = 0u;
    __syncthreads();
    uint64_t carry = 0;
    uint32_t mx = 0;
    for (int first = 0; first < T; first += 1024) {
        const int tile = first + t;
        uint4 a = make_uint4(0u, 0u, 0u, 0u), b = a;
        if (tile < T) {
            uint4 *p = reinterpret_cast<uint4 *>(cnt + (size_t)tile * kShards);
            a = p[0];
            b = p[1];
            // leave the counts zero for the next projection
            p[0] = make_uint4(0u, 0u, 0u, 0u);
            p[1] = make_uint4(0u, 0u, 0u, 0u);
        }
        const uint32_t x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        uint64_t s = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) s += x[k];
        mx = max(mx, (uint32_t)min(s, (uint64_t)0xFFFFFFFFu));
        if (tile < T && s > (uint64_t)kTsCap) long_tiles[atomicAdd(&nlong, 1u)] = (uint32_t)tile;
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
        out[3] = nlong;
        if (host_out) {  // the same four words straight into host memory (no copy launch)
            host_out[0] = (uint32_t)carry;
            host_out[1] = (uint32_t)(carry >> 32);
            host_out[2] = mx;
            host_out[3] = nlong;
        }
    }
}

// Emission advances every cursor by its (tile, shard) count, so afterwards cursor[t, s]
// holds the first slot of shard s + 1; this puts the first slots back for another emission.
__global__ __launch_bounds__(256) void restore_cursors_kernel(const uint2 *__restrict__ ranges, int T,
                                                              uint32_t *__restrict__ cursor)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= T) return;
    uint4 *q = reinterpret_cast<uint4 *>(cursor + (size_t)t * kShards);
    const uint4 a = q[0], b = q[1];
    q[0] = make_uint4(ranges[t].x, a.x, a.y, a.z);
    q[1] = make_uint4(a.w, b.x, b.y, b.z);
}

// ---------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------

int tile_sort_capacity() { return kTsCap; }

hipError_t launch_tile_scan(uint32_t *cnt, int T, uint2 *ranges, uint32_t *cursor, uint32_t *out,
                            uint32_t *long_tiles, uint32_t *host_out, hipStream_t s)
{
    tile_scan_kernel<<<1, 1024, 0, s>>>(cnt, T, ranges, cursor, out, long_tiles, host_out);
    return hipGetLastError();
}

hipError_t launch_restore_cursors(const uint2 *ranges, int T, uint32_t *cursor, hipStream_t s)
{
    if (T > 0) restore_cursors_kernel<<<(T + 255) / 256, 256, 0, s>>>(ranges, T, cursor);
    return hipGetLastError();
}

int tile_sort_chunks(int64_t longest) { return (int)((longest + kTsCap - 1) / kTsCap); }

hipError_t launch_tile_sort(const uint2 *ranges, int T, const uint32_t *keys, int64_t n, uint32_t *ids,
                            int64_t cap_pairs, bool sort_lists, const ChunkList &cl, hipStream_t s)
{
    if (T <= 0) return hipSuccess;
    tile_sort_kernel<<<T + 1, kTsThreads, 0, s>>>(ranges, T, keys, n, ids, cl, cap_pairs, sort_lists ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_tile_sort_long(const uint2 *ranges, const uint32_t *keys, int64_t n, uint32_t *ids,
                                 const uint32_t *long_tiles, int n_long, int nch, unsigned long long *tmp,
                                 hipStream_t s)
{
    if (n_long > 0 && nch > 1) {
        const unsigned grid = (unsigned)((int64_t)n_long * nch);
        tile_chunk_sort_kernel<<<grid, kTsThreads, 0, s>>>(ranges, long_tiles, nch, keys, n, ids, tmp);
        tile_chunk_merge_kernel<<<grid, kTsThreads, 0, s>>>(ranges, long_tiles, nch, tmp, ids);
    }
    return hipGetLastError();
}

}  // namespace lgsr
