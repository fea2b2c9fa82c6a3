// sort.hip -- device scans and a stable LSD radix sort of (key, value) pairs for gfx950.
//
// Both sorts of the renderer use it: the surfels by (centre range, index) and the
// (surfel, tile) pairs by tile, which keeps each tile's list in range order because the
// pairs are emitted in range order and every pass is stable.
//
// Radix pass (8-bit digits, 4096 keys per workgroup of 256 threads):
//   upsweep   per-workgroup digit histogram, wave-aggregated LDS adds;
//   scan      exclusive scan of the digit-major histogram matrix;
//   downsweep stable scatter: within a wave, keys with equal digits are ranked with eight
//             ballots (match-any by bits); waves and rounds are ordered through LDS counters.
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys per workgroup
constexpr int kScanTile = 4096;                       // elements per scan workgroup

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Lanes of the wave (among `valid` ones) holding the same 8-bit digit as this lane.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid)
{
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        uint64_t m = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? m : ~m;
    }
    return valid ? peers : 0ull;
}

__global__ __launch_bounds__(kSortThreads) void radix_upsweep(const uint32_t *__restrict__ keys, int64_t n,
                                                              int shift, uint32_t *__restrict__ hist, int nb)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    const int64_t base = (int64_t)blockIdx.x * kSortTile + threadIdx.x;
    uint32_t x[kSortItems];
#pragma unroll
    for (int rd = 0; rd < kSortItems; ++rd) {
        const int64_t i = base + rd * kSortThreads;
        x[rd] = i < n ? keys[i] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int rd = 0; rd < kSortItems; ++rd) {
        const bool valid = base + rd * kSortThreads < n;
        const uint32_t d = (x[rd] >> shift) & 255u;
        const uint64_t peers = match_digit(d, valid);
        if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Exclusive offset of (digit t, this workgroup) straight from the digit-major histogram:
// sum of all counts of lower digits plus this digit's counts in lower workgroups.  Used
// when the matrix is small (nb <= kSelfOffsetBlocks), saving the separate scan.
constexpr int kSelfOffsetBlocks = 256;

__device__ __forceinline__ uint32_t self_offset(const uint32_t *__restrict__ hist, int nb)
{
    __shared__ uint32_t wsum[4];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const uint32_t *row = hist + (size_t)t * nb;
    uint32_t before = 0, total = 0;
    for (int b = 0; b < nb; ++b) {
        const uint32_t c = row[b];
        before += b < (int)blockIdx.x ? c : 0u;
        total += c;
    }
    uint32_t inc = total;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (l >= o) inc += y;
    }
    if (l == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < w; ++k) off += wsum[k];
    return off + inc - total + before;
}

__global__ __launch_bounds__(kSortThreads) void radix_downsweep(const uint32_t *__restrict__ keys_in,
                                                                const uint32_t *__restrict__ vals_in,
                                                                uint32_t *__restrict__ keys_out,
                                                                uint32_t *__restrict__ vals_out, int64_t n,
                                                                int shift, const uint32_t *__restrict__ offs,
                                                                int nb, int scanned)
{
    __shared__ uint32_t base_off[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[4][256];
    const int t = threadIdx.x, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * kSortTile + t;
    uint32_t kx[kSortItems], vx[kSortItems];
#pragma unroll
    for (int rd = 0; rd < kSortItems; ++rd) {
        const int64_t i = base + rd * kSortThreads;
        kx[rd] = i < n ? keys_in[i] : 0u;
        vx[rd] = i < n ? vals_in[i] : 0u;
    }
    base_off[t] = scanned ? offs[(size_t)t * nb + blockIdx.x] : self_offset(offs, nb);
    run[t] = 0;
#pragma unroll
    for (int rd = 0; rd < kSortItems; ++rd) {
        const bool valid = base + rd * kSortThreads < n;
        const uint32_t key = kx[rd], val = vx[rd];
        const uint32_t d = (key >> shift) & 255u;
        for (int c = 0; c < 4; ++c) wcnt[c][t] = 0;
        __syncthreads();
        const uint64_t peers = match_digit(d, valid);
        const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {   // thread t owns digit t: prefix over waves, advance the running count
            const uint32_t r = run[t];
            const uint32_t c0 = wcnt[0][t], c1 = wcnt[1][t], c2 = wcnt[2][t], c3 = wcnt[3][t];
            wcnt[0][t] = r;
            wcnt[1][t] = r + c0;
            wcnt[2][t] = r + c0 + c1;
            wcnt[3][t] = r + c0 + c1 + c2;
            run[t] = r + c0 + c1 + c2 + c3;
        }
        __syncthreads();
        if (valid) {
            const uint32_t dst = base_off[d] + wcnt[w][d] + rank;
            keys_out[dst] = key;
            vals_out[dst] = val;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// exclusive scan of uint32 (optionally of in[gather[i]]), three phases
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(v, o, 64);
        if (l >= o) v += y;
    }
    return v;
}

// Exclusive scan of one value per thread over the workgroup (256 threads); returns the
// exclusive prefix and writes the total to *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[4];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    uint32_t inc = wave_incl_scan(v);
    if (l == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int k = 0; k < 4; ++k) {
        uint32_t s = wsum[k];
        if (k < w) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__device__ __forceinline__ void load16(const uint32_t *__restrict__ in, const uint32_t *__restrict__ gather,
                                       int64_t n, int64_t first, uint32_t *x)
{
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        int64_t i = first + k;
        x[k] = i < n ? (gather ? in[gather[i]] : in[i]) : 0u;
    }
}

__global__ __launch_bounds__(256) void scan_reduce(const uint32_t *__restrict__ in,
                                                   const uint32_t *__restrict__ gather, int64_t n,
                                                   uint32_t *__restrict__ sums)
{
    uint32_t x[16];
    load16(in, gather, n, (int64_t)blockIdx.x * kScanTile + threadIdx.x * 16, x);
    uint32_t s = 0;
    for (int k = 0; k < 16; ++k) s += x[k];
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Scans `nb` block sums (nb <= 4096) in one workgroup; writes the grand total.
__global__ __launch_bounds__(256) void scan_top(uint32_t *__restrict__ sums, int nb, uint32_t *__restrict__ total)
{
    uint32_t x[16];
    load16(sums, nullptr, nb, threadIdx.x * 16, x);
    uint32_t s = 0;
    for (int k = 0; k < 16; ++k) s += x[k];
    uint32_t tot;
    uint32_t off = block_excl_scan(s, &tot);
    for (int k = 0; k < 16; ++k) {
        int i = threadIdx.x * 16 + k;
        if (i < nb) sums[i] = off;
        off += x[k];
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

__global__ __launch_bounds__(256) void scan_down(const uint32_t *__restrict__ in,
                                                 const uint32_t *__restrict__ gather, int64_t n,
                                                 const uint32_t *__restrict__ sums, uint32_t *__restrict__ out)
{
    uint32_t x[16];
    int64_t first = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 16;
    load16(in, gather, n, first, x);
    uint32_t s = 0;
    for (int k = 0; k < 16; ++k) s += x[k];
    uint32_t tot;
    uint32_t off = block_excl_scan(s, &tot) + sums[blockIdx.x];
    for (int k = 0; k < 16; ++k) {
        int64_t i = first + k;
        if (i < n) out[i] = off;
        off += x[k];
    }
}

// One workgroup scans n <= 16 * 4096 elements in rounds of 4096 with a running carry.
__global__ __launch_bounds__(256) void scan_single(const uint32_t *__restrict__ in,
                                                   const uint32_t *__restrict__ gather, int64_t n,
                                                   uint32_t *__restrict__ out, uint32_t *__restrict__ total)
{
    uint32_t carry = 0;
    for (int64_t first_tile = 0; first_tile < n; first_tile += kScanTile) {
        uint32_t x[16];
        const int64_t first = first_tile + threadIdx.x * 16;
        load16(in, gather, n, first, x);
        uint32_t s = 0;
        for (int k = 0; k < 16; ++k) s += x[k];
        uint32_t tot;
        uint32_t off = block_excl_scan(s, &tot) + carry;
        for (int k = 0; k < 16; ++k) {
            const int64_t i = first + k;
            if (i < n) out[i] = off;
            off += x[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// ---------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------

size_t scan_tmp_words(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

hipError_t scan_u32(const uint32_t *in, const uint32_t *gather, uint32_t *out, uint32_t *total, int64_t n,
                    uint32_t *tmp, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb > kScanTile) return hipErrorInvalidValue;
    if (nb <= 1) {  // one tile: one launch
        scan_single<<<1, 256, 0, s>>>(in, gather, n, out, total);
        return hipGetLastError();
    }
    scan_reduce<<<(unsigned)nb, 256, 0, s>>>(in, gather, n, tmp);
    scan_top<<<1, 256, 0, s>>>(tmp, (int)nb, total);
    scan_down<<<(unsigned)nb, 256, 0, s>>>(in, gather, n, tmp, out);
    return hipGetLastError();
}

size_t radix_hist_words(int64_t n) { return (size_t)256 * (size_t)((n + kSortTile - 1) / kSortTile); }

hipError_t radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt, int64_t n,
                            int bits, uint32_t *hist, uint32_t *scan_tmp, hipStream_t s, bool *in_alt)
{
    *in_alt = false;
    if (n <= 0 || bits <= 0) return hipSuccess;
    int nb = (int)((n + kSortTile - 1) / kSortTile);
    uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
    const int scanned = nb > kSelfOffsetBlocks;
    for (int shift = 0; shift < bits; shift += 8) {
        radix_upsweep<<<nb, kSortThreads, 0, s>>>(ki, n, shift, hist, nb);
        if (scanned) {
            hipError_t e = scan_u32(hist, nullptr, hist, nullptr, (int64_t)256 * nb, scan_tmp, s);
            if (e != hipSuccess) return e;
        }
        radix_downsweep<<<nb, kSortThreads, 0, s>>>(ki, vi, ko, vo, n, shift, hist, nb, scanned);
        uint32_t *tk = ki, *tv = vi;
        ki = ko;
        vi = vo;
        ko = tk;
        vo = tv;
        *in_alt = !*in_alt;
    }
    return hipGetLastError();
}

}  // namespace lgsr
