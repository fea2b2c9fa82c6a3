// scan.hip -- the step before the renderer and the tracker's view of the map
// (arXiv 2607.04127 Sec. 3.1, Sec. 3.2).
//
// Scan to range image: the spherical projection of a scan onto the grid the map is rendered
// on.  Rows are uniform in elevation from el_max (row 0) to el_min (row H-1), columns uniform
// over the full turn (column j at azimuth 2 pi j / W); a point takes the nearest row and
// column, is kept inside the rows and the range gates, and the nearest return wins each
// pixel (equal ranges: the lower point index).  One thread per point packs (range bits,
// index) into a 64-bit key -- a non-negative float orders like its bit pattern -- and takes
// the pixel's minimum with one 64-bit atomic; a second pass per pixel unpacks the winner and
// copies its normal, turned to face the sensor.  The per-pixel keys are scratch (8 B per
// pixel), cleared by a fill kernel.
//
// Target covariance: Sigma = R diag(s_x^2, s_y^2, eps^2) R^T per surfel, R = [a b n] from the
// normalised quaternion, written as (xx, xy, xz, yy, yz, zz); a zero quaternion gives zero.
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

constexpr int kScanThreads = 256;
constexpr unsigned long long kNoReturn = ~0ull;

__global__ __launch_bounds__(kScanThreads) void fill_u64_kernel(unsigned long long *__restrict__ p, int64_t n,
                                                                unsigned long long v)
{
    for (int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kScanThreads)
        p[i] = v;
}

__global__ __launch_bounds__(kScanThreads) void scan_bin_kernel(int64_t n, const float *__restrict__ pts,
                                                                ScanGridF g, unsigned long long *__restrict__ slots)
{
    const int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    if (i >= n) return;
    const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
    const float r = sqrtf(fmaf(x, x, fmaf(y, y, z * z)));
    if (!(r >= g.r_min && r <= g.r_max)) return;
    const float el = atan2f(z, sqrtf(fmaf(x, x, y * y)));
    const float az = atan2f(y, x);
    const float kf = floorf((g.el_max - el) * g.rows_per_rad + 0.5f);
    if (!(kf >= 0.f && kf <= (float)(g.H - 1))) return;
    int j = (int)floorf(az * g.cols_per_rad + 0.5f) % g.W;
    if (j < 0) j += g.W;
    const int64_t pix = (int64_t)kf * g.W + j;
    const unsigned long long key = ((unsigned long long)__float_as_uint(r) << 32) | (unsigned long long)(uint32_t)i;
    atomicMin(slots + pix, key);
}

__global__ __launch_bounds__(kScanThreads) void scan_write_kernel(int64_t P, const unsigned long long *__restrict__ slots,
                                                                  const float *__restrict__ pts,
                                                                  const float *__restrict__ nrm, float *__restrict__ depth,
                                                                  float *__restrict__ normal, int32_t *__restrict__ index)
{
    const int64_t q = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    if (q >= P) return;
    const unsigned long long key = slots[q];
    float d = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
    int32_t idx = -1;
    if (key != kNoReturn) {
        idx = (int32_t)(uint32_t)key;
        d = __uint_as_float((uint32_t)(key >> 32));
        if (nrm) {
            n0 = nrm[3 * (int64_t)idx];
            n1 = nrm[3 * (int64_t)idx + 1];
            n2 = nrm[3 * (int64_t)idx + 2];
            const float p0 = pts[3 * (int64_t)idx], p1 = pts[3 * (int64_t)idx + 1], p2 = pts[3 * (int64_t)idx + 2];
            if (fmaf(n0, p0, fmaf(n1, p1, n2 * p2)) > 0.f) {
                n0 = -n0;
                n1 = -n1;
                n2 = -n2;
            }
        }
    }
    depth[q] = d;
    if (index) index[q] = idx;
    if (normal) {
        normal[3 * q] = n0;
        normal[3 * q + 1] = n1;
        normal[3 * q + 2] = n2;
    }
}

static unsigned grid_for(int64_t n)
{
    int64_t b = (n + kScanThreads - 1) / kScanThreads;
    return (unsigned)(b < 1 ? 1 : b);
}

hipError_t launch_scan_to_range(int64_t n, const float *pts, const float *nrm, const ScanGridF &g,
                                unsigned long long *slots, float *depth, float *normal, int32_t *index, hipStream_t s)
{
    const int64_t P = (int64_t)g.H * g.W;
    int64_t fb = (P + kScanThreads - 1) / kScanThreads;
    if (fb > 4096) fb = 4096;
    fill_u64_kernel<<<(unsigned)(fb < 1 ? 1 : fb), kScanThreads, 0, s>>>(slots, P, kNoReturn);
    if (n > 0) scan_bin_kernel<<<grid_for(n), kScanThreads, 0, s>>>(n, pts, g, slots);
    scan_write_kernel<<<grid_for(P), kScanThreads, 0, s>>>(P, slots, pts, nrm, depth, normal, index);
    return hipGetLastError();
}

// ---- target covariance ----

__global__ __launch_bounds__(kScanThreads) void target_cov_kernel(int64_t n, const float4 *__restrict__ quats,
                                                                  const float2 *__restrict__ log_scales, float eps2,
                                                                  float *__restrict__ cov)
{
    const int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
    if (i >= n) return;
    const float4 q = quats[i];
    const float qq = fmaf(q.x, q.x, fmaf(q.y, q.y, fmaf(q.z, q.z, q.w * q.w)));
    float2 *o = reinterpret_cast<float2 *>(cov + 6 * i);
    if (!(qq > 0.f)) {
        o[0] = o[1] = o[2] = make_float2(0.f, 0.f);
        return;
    }
    const float inv = rsqrtf(qq);
    const float w = q.x * inv, x = q.y * inv, y = q.z * inv, z = q.w * inv;
    // rotation columns a, b, n
    const float a0 = 1.f - 2.f * (y * y + z * z), a1 = 2.f * (x * y + w * z), a2 = 2.f * (x * z - w * y);
    const float b0 = 2.f * (x * y - w * z), b1 = 1.f - 2.f * (x * x + z * z), b2 = 2.f * (y * z + w * x);
    const float c0 = 2.f * (x * z + w * y), c1 = 2.f * (y * z - w * x), c2 = 1.f - 2.f * (x * x + y * y);
    const float2 ls = log_scales[i];
    const float dx = expf(2.f * ls.x), dy = expf(2.f * ls.y);
    auto S = [&](float ar, float br, float cr, float ac, float bc, float cc) {
        return fmaf(ar * dx, ac, fmaf(br * dy, bc, cr * eps2 * cc));
    };
    o[0] = make_float2(S(a0, b0, c0, a0, b0, c0), S(a0, b0, c0, a1, b1, c1));
    o[1] = make_float2(S(a0, b0, c0, a2, b2, c2), S(a1, b1, c1, a1, b1, c1));
    o[2] = make_float2(S(a1, b1, c1, a2, b2, c2), S(a2, b2, c2, a2, b2, c2));
}

hipError_t launch_target_cov(int64_t n, const float *quats, const float *log_scales, float eps, float *cov,
                             hipStream_t s)
{
    if (n > 0)
        target_cov_kernel<<<grid_for(n), kScanThreads, 0, s>>>(n, reinterpret_cast<const float4 *>(quats),
                                                               reinterpret_cast<const float2 *>(log_scales), eps * eps,
                                                               cov);
    return hipGetLastError();
}

}  // namespace lgsr
