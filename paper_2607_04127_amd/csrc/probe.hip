// probe.hip -- streaming kernels that measure the HBM bandwidth a kernel can reach on this
// device (the denominator of the path's HBM fraction) and flush the caches between timed
// steps.  Not part of the rendering path.
//
// copy:  dst[i] = src[i]            (8 bytes moved per float)
// triad: a[i] = b[i] + s c[i]       (12 bytes moved per float)
// Two forms of each: four 16-byte vectors per lane and iteration with non-temporal loads and
// stores, or one vector with plain ones; the grid (a given number of 256-lane workgroups)
// strides over the arrays.  A caller takes the best over forms and grid sizes.
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kProbeThreads = 256;

template <int U, bool NT>
__device__ __forceinline__ v4f ld(const v4f *p)
{
    return NT ? __builtin_nontemporal_load(p) : *p;
}

template <int U, bool NT>
__device__ __forceinline__ void st(v4f v, v4f *p)
{
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <int U, bool NT>
__global__ __launch_bounds__(kProbeThreads) void copy_kernel(const v4f *__restrict__ src, v4f *__restrict__ dst,
                                                             int64_t n4)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    for (; i + (U - 1) * stride < n4; i += U * stride) {
        v4f v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld<U, NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) st<U, NT>(v[u], dst + i + u * stride);
    }
    for (; i < n4; i += stride) dst[i] = src[i];
}

template <int U, bool NT>
__global__ __launch_bounds__(kProbeThreads) void triad_kernel(const v4f *__restrict__ b, const v4f *__restrict__ c,
                                                              v4f *__restrict__ a, float s, int64_t n4)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    for (; i + (U - 1) * stride < n4; i += U * stride) {
        v4f x[U], y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            x[u] = ld<U, NT>(b + i + u * stride);
            y[u] = ld<U, NT>(c + i + u * stride);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const v4f r = {fmaf(s, y[u].x, x[u].x), fmaf(s, y[u].y, x[u].y), fmaf(s, y[u].z, x[u].z),
                           fmaf(s, y[u].w, x[u].w)};
            st<U, NT>(r, a + i + u * stride);
        }
    }
    for (; i < n4; i += stride) {
        const v4f x = b[i], y = c[i];
        const v4f r = {fmaf(s, y.x, x.x), fmaf(s, y.y, x.y), fmaf(s, y.z, x.z), fmaf(s, y.w, x.w)};
        a[i] = r;
    }
}

hipError_t launch_stream_probe(int kind, const float *b, const float *c, float *a, int64_t n, int blocks,
                               hipStream_t s)
{
    const int64_t n4 = n / 4;
    if (n4 <= 0) return hipSuccess;
    if (blocks <= 0) blocks = 4096;
    const v4f *b4 = reinterpret_cast<const v4f *>(b), *c4 = reinterpret_cast<const v4f *>(c);
    v4f *a4 = reinterpret_cast<v4f *>(a);
    switch (kind) {
    case 0: copy_kernel<4, true><<<blocks, kProbeThreads, 0, s>>>(b4, a4, n4); break;
    case 1: triad_kernel<4, true><<<blocks, kProbeThreads, 0, s>>>(b4, c4, a4, 3.f, n4); break;
    case 2: copy_kernel<1, false><<<blocks, kProbeThreads, 0, s>>>(b4, a4, n4); break;
    default: triad_kernel<1, false><<<blocks, kProbeThreads, 0, s>>>(b4, c4, a4, 3.f, n4); break;
    }
    return hipGetLastError();
}

}  // namespace lgsr
