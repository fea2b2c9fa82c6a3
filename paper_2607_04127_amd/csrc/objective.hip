// objective.hip -- the full mapping objective over a rendered frame and the scale
// regulariser over the map (arXiv 2607.04127 Sec. 3.4, Eq. 10-13; weights of Sec. 4.1).
//
//   frame terms:
//     w_depth / |Omega_D| sum_{Omega_D} |D^ - D|
//     - lambda_alpha / |Omega_D| sum_{Omega_D} log(A^ + eps)
//     + lambda_n lambda_ng / |Omega_N| sum_{Omega_N} (1 - N^.N_gicp / |N^|)
//     + lambda_n lambda_ns / |Omega_D| sum_{Omega_D, N_surf defined} (1 - N^.N_surf / |N^|)
//   N_surf at pixel (k, j): v = (P(k, j+1) - P(k, j-1)) x (P(k+1, j) - P(k-1, j)) with
//     P = D^ d, columns wrapping over the full turn; defined for rows 1..H-2 when the four
//     neighbours rendered a range and v != 0; v / |v| turned to face the sensor.
//   scale regulariser: lambda_s sum_i max(0, max(s_x, s_y) - s_max), s = exp(log_scales).
//
// Frame terms: per-block partial sums, one block folding them in a fixed order, then one
// thread per ray writing dL/d(D^, A^, N^).  The surface-normal term reaches the depth of
// the four neighbours, so the gradient kernel gathers: for ray q it evaluates the N_surf
// stencils of the four pixels whose stencil contains q (reading a radius-2 diamond of
// depths, which the caches serve) and adds each one's derivative along q's direction --
// no scatter, no atomics, no scratch.
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

constexpr int kObjThreads = 256;
constexpr int kObjMaxBlocks = 1024;
constexpr int kObjSums = 8;  // per-block partials: 4 float sums, 3 counts, 1 pad

struct FrameIn {
    const float *depth, *opacity, *normal, *td, *tn, *rows, *cols;
    int H, W;
};

__device__ __forceinline__ float3 beam_dir(const FrameIn &f, int k, int j)
{
    float sp = f.rows[2 * k], cp = f.rows[2 * k + 1];
    float st = f.cols[2 * j], ct = f.cols[2 * j + 1];
    return make_float3(cp * ct, cp * st, sp);
}

__device__ __forceinline__ float3 f3_sub(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float f3_dot(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ float3 f3_cross(float3 a, float3 b)
{
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 f3_scale(float3 a, float s) { return make_float3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float3 load3(const float *p, int64_t i)
{
    return make_float3(p[3 * i], p[3 * i + 1], p[3 * i + 2]);
}

// The rendered-surface normal stencil of pixel (k, j).
struct Stencil {
    float3 a, b, v;  // P_r - P_l, P_u - P_d, a x b
    float vn, sgn;   // |v|, +1 / -1 (turn to face the sensor)
};

__device__ __forceinline__ bool surf_stencil(const FrameIn &f, int k, int j, Stencil &s)
{
    if (k < 1 || k > f.H - 2) return false;
    const int jr = j + 1 == f.W ? 0 : j + 1;
    const int jl = j == 0 ? f.W - 1 : j - 1;
    const float Dr = f.depth[(int64_t)k * f.W + jr], Dl = f.depth[(int64_t)k * f.W + jl];
    const float Du = f.depth[(int64_t)(k + 1) * f.W + j], Dd = f.depth[(int64_t)(k - 1) * f.W + j];
    if (!(Dr > 0.f) || !(Dl > 0.f) || !(Du > 0.f) || !(Dd > 0.f)) return false;
    s.a = f3_sub(f3_scale(beam_dir(f, k, jr), Dr), f3_scale(beam_dir(f, k, jl), Dl));
    s.b = f3_sub(f3_scale(beam_dir(f, k + 1, j), Du), f3_scale(beam_dir(f, k - 1, j), Dd));
    s.v = f3_cross(s.a, s.b);
    s.vn = sqrtf(f3_dot(s.v, s.v));
    if (!(s.vn > 0.f)) return false;
    s.sgn = f3_dot(s.v, beam_dir(f, k, j)) > 0.f ? -1.f : 1.f;
    return true;
}

struct ObjTerms {
    float l1, la, cg, cs;  // |D^ - D|, log(A^ + eps), G-ICP (1 - cos), surface (1 - cos)
    uint32_t mD, mN, mS;
};

__device__ __forceinline__ ObjTerms obj_terms(const FrameIn &f, int64_t r, float eps)
{
    ObjTerms o{0.f, 0.f, 0.f, 0.f, 0u, 0u, 0u};
    const float D = f.td[r];
    if (!(D > 0.f)) return o;
    o.mD = 1u;
    o.l1 = fabsf(f.depth[r] - D);
    o.la = logf(f.opacity[r] + eps);
    const float3 Nh = load3(f.normal, r);
    const float nn = sqrtf(f3_dot(Nh, Nh));
    const float3 Nt = load3(f.tn, r);
    if (f3_dot(Nt, Nt) > 0.f) {
        o.mN = 1u;
        o.cg = nn > 0.f ? 1.f - f3_dot(Nh, Nt) / nn : 1.f;
    }
    Stencil s;
    const int k = (int)(r / f.W), j = (int)(r - (int64_t)k * f.W);
    if (surf_stencil(f, k, j, s)) {
        o.mS = 1u;
        o.cs = nn > 0.f ? 1.f - s.sgn * f3_dot(Nh, s.v) / (s.vn * nn) : 1.f;
    }
    return o;
}

__global__ __launch_bounds__(kObjThreads) void objective_partials(FrameIn f, float eps, float *__restrict__ partials)
{
    const int64_t n = (int64_t)f.H * f.W;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    uint32_t c0 = 0, c1 = 0, c2 = 0;
    for (int64_t r = (int64_t)blockIdx.x * kObjThreads + threadIdx.x; r < n; r += (int64_t)gridDim.x * kObjThreads) {
        ObjTerms t = obj_terms(f, r, eps);
        s0 += t.l1;
        s1 += t.la;
        s2 += t.cg;
        s3 += t.cs;
        c0 += t.mD;
        c1 += t.mN;
        c2 += t.mS;
    }
    __shared__ float sf[4][kObjThreads];
    __shared__ uint32_t su[3][kObjThreads];
    const int t = threadIdx.x;
    sf[0][t] = s0;
    sf[1][t] = s1;
    sf[2][t] = s2;
    sf[3][t] = s3;
    su[0][t] = c0;
    su[1][t] = c1;
    su[2][t] = c2;
    __syncthreads();
    for (int o = kObjThreads / 2; o > 0; o >>= 1) {
        if (t < o) {
#pragma unroll
            for (int q = 0; q < 4; ++q) sf[q][t] += sf[q][t + o];
#pragma unroll
            for (int q = 0; q < 3; ++q) su[q][t] += su[q][t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        float *p = partials + kObjSums * blockIdx.x;
        for (int q = 0; q < 4; ++q) p[q] = sf[q][0];
        for (int q = 0; q < 3; ++q) p[4 + q] = __uint_as_float(su[q][0]);
        p[7] = 0.f;
    }
}

// One workgroup folds the partials in a fixed order (deterministic); counts are exact.
__global__ __launch_bounds__(kObjThreads) void objective_finalize(int nb, const float *__restrict__ partials,
                                                                  ObjectiveWeights w, float *__restrict__ loss_out)
{
    __shared__ float sf[4][kObjThreads];
    __shared__ uint32_t su[3][kObjThreads];
    const int t = threadIdx.x;
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    uint32_t c[3] = {0u, 0u, 0u};
    for (int b = t; b < nb; b += kObjThreads) {
        const float *p = partials + kObjSums * b;
        for (int q = 0; q < 4; ++q) s[q] += p[q];
        for (int q = 0; q < 3; ++q) c[q] += __float_as_uint(p[4 + q]);
    }
    for (int q = 0; q < 4; ++q) sf[q][t] = s[q];
    for (int q = 0; q < 3; ++q) su[q][t] = c[q];
    __syncthreads();
    for (int o = kObjThreads / 2; o > 0; o >>= 1) {
        if (t < o) {
#pragma unroll
            for (int q = 0; q < 4; ++q) sf[q][t] += sf[q][t + o];
#pragma unroll
            for (int q = 0; q < 3; ++q) su[q][t] += su[q][t + o];
        }
        __syncthreads();
    }
    if (t != 0) return;
    const uint32_t cD = su[0][0], cN = su[1][0], cS = su[2][0];
    const float tD = cD ? w.w_depth * sf[0][0] / (float)cD : 0.f;
    const float tA = cD ? -w.lambda_alpha * sf[1][0] / (float)cD : 0.f;
    const float tNg = cN ? w.lambda_n * w.lambda_ng * sf[2][0] / (float)cN : 0.f;
    const float tNs = cD ? w.lambda_n * w.lambda_ns * sf[3][0] / (float)cD : 0.f;
    loss_out[0] = tD + tA + tNg + tNs;
    loss_out[1] = tD;
    loss_out[2] = tA;
    loss_out[3] = tNg;
    loss_out[4] = tNs;
    loss_out[5] = (float)cD;
    loss_out[6] = (float)cN;
    loss_out[7] = (float)cS;
}

// dl/dv of the surface-normal term of pixel p (in Omega_D, |N^_p| > 0, stencil defined):
// dl/dN_surf = -c0 N^/|N^|, N_surf = sgn v/|v|  =>  dl/dv = sgn (g - (g.u) u) / |v|, u = v/|v|.
__device__ __forceinline__ bool surf_dv(const FrameIn &f, int k, int j, float c0, Stencil &s, float3 &gv)
{
    if (k < 1 || k > f.H - 2) return false;  // no stencil on the first and last rows
    const int64_t p = (int64_t)k * f.W + j;
    if (!(f.td[p] > 0.f)) return false;
    const float3 Nh = load3(f.normal, p);
    const float nn2 = f3_dot(Nh, Nh);
    if (!(nn2 > 0.f)) return false;
    if (!surf_stencil(f, k, j, s)) return false;
    const float inv_nn = 1.f / sqrtf(nn2), inv_vn = 1.f / s.vn;
    const float3 g = f3_scale(Nh, -c0 * inv_nn);
    const float3 u = f3_scale(s.v, inv_vn);
    const float gu = f3_dot(g, u);
    const float k1 = s.sgn * inv_vn;
    gv = make_float3(k1 * fmaf(-gu, u.x, g.x), k1 * fmaf(-gu, u.y, g.y), k1 * fmaf(-gu, u.z, g.z));
    return true;
}

__global__ __launch_bounds__(kObjThreads) void objective_grad(FrameIn f, ObjectiveWeights w,
                                                              const float *__restrict__ loss_out,
                                                              float *__restrict__ gD, float *__restrict__ gA,
                                                              float *__restrict__ gN)
{
    const int64_t n = (int64_t)f.H * f.W;
    const int64_t r = (int64_t)blockIdx.x * kObjThreads + threadIdx.x;
    if (r >= n) return;
    const float cD = loss_out[5], cN = loss_out[6];
    const int k = (int)(r / f.W), j = (int)(r - (int64_t)k * f.W);
    float gd = 0.f, ga = 0.f;
    float3 gn = make_float3(0.f, 0.f, 0.f);
    if (cD > 0.f) {
        const float c0 = w.lambda_n * w.lambda_ns / cD;
        const float D = f.td[r];
        if (D > 0.f) {
            const float diff = f.depth[r] - D;
            gd = w.w_depth * (diff > 0.f ? 1.f : (diff < 0.f ? -1.f : 0.f)) / cD;
            ga = -w.lambda_alpha / (cD * (f.opacity[r] + w.eps));
            const float3 Nh = load3(f.normal, r);
            const float nn2 = f3_dot(Nh, Nh);
            if (nn2 > 0.f) {
                const float nn = sqrtf(nn2);
                const float3 Nt = load3(f.tn, r);
                if (f3_dot(Nt, Nt) > 0.f) {
                    const float cosv = f3_dot(Nh, Nt) / nn;
                    const float fg = -w.lambda_n * w.lambda_ng / (cN * nn);
                    const float cn = cosv / nn;
                    gn = make_float3(fg * fmaf(-cn, Nh.x, Nt.x), fg * fmaf(-cn, Nh.y, Nt.y), fg * fmaf(-cn, Nh.z, Nt.z));
                }
                Stencil s;
                if (surf_stencil(f, k, j, s)) {
                    const float3 Ns = f3_scale(s.v, s.sgn / s.vn);
                    const float cn = f3_dot(Nh, Ns) / nn2;
                    const float fs = -c0 / nn;
                    gn.x += fs * fmaf(-cn, Nh.x, Ns.x);
                    gn.y += fs * fmaf(-cn, Nh.y, Ns.y);
                    gn.z += fs * fmaf(-cn, Nh.z, Ns.z);
                }
            }
        }
        // The surface-normal terms whose stencil holds this ray: as the right neighbour of
        // (k, j-1), the left one of (k, j+1), the upper one of (k-1, j), the lower of (k+1, j).
        if (w.lambda_ns != 0.f) {
            const float3 dq = beam_dir(f, k, j);
            float acc = 0.f;
            Stencil s;
            float3 gv;
            if (surf_dv(f, k, j == 0 ? f.W - 1 : j - 1, c0, s, gv)) acc += f3_dot(dq, f3_cross(s.b, gv));
            if (surf_dv(f, k, j + 1 == f.W ? 0 : j + 1, c0, s, gv)) acc -= f3_dot(dq, f3_cross(s.b, gv));
            if (surf_dv(f, k - 1, j, c0, s, gv)) acc += f3_dot(dq, f3_cross(gv, s.a));
            if (surf_dv(f, k + 1, j, c0, s, gv)) acc -= f3_dot(dq, f3_cross(gv, s.a));
            gd += acc;
        }
    }
    gD[r] = gd;
    gA[r] = ga;
    gN[3 * r] = gn.x;
    gN[3 * r + 1] = gn.y;
    gN[3 * r + 2] = gn.z;
}

int objective_blocks(int64_t n_rays)
{
    int64_t b = (n_rays + kObjThreads * 4 - 1) / (kObjThreads * 4);
    if (b < 1) b = 1;
    if (b > kObjMaxBlocks) b = kObjMaxBlocks;
    return (int)b;
}

int objective_partial_floats(int64_t n_rays) { return objective_blocks(n_rays) * kObjSums; }

hipError_t launch_objective(int H, int W, const float *rows, const float *cols, const float *depth,
                            const float *opacity, const float *normal, const float *td, const float *tn,
                            const ObjectiveWeights &w, float *partials, float *loss_out, float *gD, float *gA,
                            float *gN, hipStream_t s)
{
    const int64_t n = (int64_t)H * W;
    FrameIn f{depth, opacity, normal, td, tn, rows, cols, H, W};
    const int nb = objective_blocks(n);
    objective_partials<<<nb, kObjThreads, 0, s>>>(f, w.eps, partials);
    objective_finalize<<<1, kObjThreads, 0, s>>>(nb, partials, w, loss_out);
    if (n > 0 && gD)
        objective_grad<<<(unsigned)((n + kObjThreads - 1) / kObjThreads), kObjThreads, 0, s>>>(f, w, loss_out, gD, gA,
                                                                                                  gN);
    return hipGetLastError();
}

// ---- scale regulariser ----

__global__ __launch_bounds__(kObjThreads) void scale_reg_kernel(int64_t n, const float2 *__restrict__ log_scales,
                                                                float lambda_s, float s_max,
                                                                float *__restrict__ partials,
                                                                float2 *__restrict__ grad)
{
    float sum = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kObjThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kObjThreads) {
        const float2 ls = log_scales[i];
        // the larger scale (exp is increasing: compare the logs), the first on a tie
        const bool second = ls.y > ls.x;
        const float s = expf(second ? ls.y : ls.x);
        if (s > s_max) {
            sum += s - s_max;
            if (grad) {
                float2 g = grad[i];
                if (second)
                    g.y += lambda_s * s;
                else
                    g.x += lambda_s * s;
                grad[i] = g;
            }
        }
    }
    __shared__ float sh[kObjThreads];
    const int t = threadIdx.x;
    sh[t] = sum;
    __syncthreads();
    for (int o = kObjThreads / 2; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    if (t == 0) partials[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kObjThreads) void scale_reg_finalize(int nb, const float *__restrict__ partials,
                                                                  float lambda_s, float *__restrict__ loss_out)
{
    __shared__ float sh[kObjThreads];
    const int t = threadIdx.x;
    float s = 0.f;
    for (int b = t; b < nb; b += kObjThreads) s += partials[b];
    sh[t] = s;
    __syncthreads();
    for (int o = kObjThreads / 2; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    if (t == 0) loss_out[0] = lambda_s * sh[0];
}

int scale_reg_blocks(int64_t n) { return objective_blocks(n); }

hipError_t launch_scale_reg(int64_t n, const float *log_scales, float lambda_s, float s_max, float *partials,
                            float *loss_out, float *grad_log_scales, hipStream_t s)
{
    const int nb = scale_reg_blocks(n);
    scale_reg_kernel<<<nb, kObjThreads, 0, s>>>(n, reinterpret_cast<const float2 *>(log_scales), lambda_s, s_max,
                                                 partials, reinterpret_cast<float2 *>(grad_log_scales));
    scale_reg_finalize<<<1, kObjThreads, 0, s>>>(nb, partials, lambda_s, loss_out);
    return hipGetLastError();
}

}  // namespace lgsr
