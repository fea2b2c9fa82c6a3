// probe.hip -- streaming kernels that measure the HBM bandwidth a kernel can reach on this
// device (the denominator of the path's HBM fraction) and flush the caches between timed
// steps.  Not part of the rendering path.
//
// copy:  dst[i] = src[i]            (8 bytes moved per float)
// triad: a[i] = b[i] + s c[i]       (12 bytes moved per float)
// Each lane moves four 16-byte vectors per iteration with independent loads in flight; the
// grid is a fixed multiple of the CU count and strides over the arrays, so the launch shape
// does not depend on the array size.
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 256;
constexpr int kProbeBlocks = 256 * 16;
constexpr int kProbeUnroll = 4;

__global__ __launch_bounds__(kProbeThreads) void copy_kernel(const v4f *__restrict__ src, v4f *__restrict__ dst,
                                                             int64_t n4)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    for (; i + (kProbeUnroll - 1) * stride < n4; i += kProbeUnroll * stride) {
        v4f v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n4; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(kProbeThreads) void triad_kernel(const v4f *__restrict__ b,
                                                              const v4f *__restrict__ c, v4f *__restrict__ a,
                                                              float s, int64_t n4)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    for (; i + (kProbeUnroll - 1) * stride < n4; i += kProbeUnroll * stride) {
        v4f x[kProbeUnroll], y[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            x[u] = __builtin_nontemporal_load(b + i + u * stride);
            y[u] = __builtin_nontemporal_load(c + i + u * stride);
        }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const v4f r = {fmaf(s, y[u].x, x[u].x), fmaf(s, y[u].y, x[u].y), fmaf(s, y[u].z, x[u].z),
                           fmaf(s, y[u].w, x[u].w)};
            __builtin_nontemporal_store(r, a + i + u * stride);
        }
    }
    for (; i < n4; i += stride) {
        const v4f x = b[i], y = c[i];
        const v4f r = {fmaf(s, y.x, x.x), fmaf(s, y.y, x.y), fmaf(s, y.z, x.z), fmaf(s, y.w, x.w)};
        a[i] = r;
    }
}

hipError_t launch_stream_copy(const float *src, float *dst, int64_t n, hipStream_t s)
{
    const int64_t n4 = n / 4;
    if (n4 <= 0) return hipSuccess;
    copy_kernel<<<kProbeBlocks, kProbeThreads, 0, s>>>(reinterpret_cast<const v4f *>(src),
                                                       reinterpret_cast<v4f *>(dst), n4);
    return hipGetLastError();
}

hipError_t launch_stream_triad(const float *b, const float *c, float *a, float scale, int64_t n, hipStream_t s)
{
    const int64_t n4 = n / 4;
    if (n4 <= 0) return hipSuccess;
    triad_kernel<<<kProbeBlocks, kProbeThreads, 0, s>>>(reinterpret_cast<const v4f *>(b),
                                                        reinterpret_cast<const v4f *>(c),
                                                        reinterpret_cast<v4f *>(a), scale, n4);
    return hipGetLastError();
}

}  // namespace lgsr
