// loss.hip -- masked depth L1 + G-ICP normal cosine loss and its per-ray gradient
// (arXiv 2607.04127 Sec. 3.4, Eq. 10 left and Eq. 11 first term; weights of Sec. 4.1).
//
//   L = w_depth / |Omega_D| sum M_D |D^ - D| + lambda_n lambda_ng / |Omega_N| sum M_N (1 - N^.N / |N^|)
//   M_D = [D > 0], M_N = M_D [|N| > 0]
//
// Two launches: per-block partial sums (two float sums, two integer counts), then the
// per-ray gradient, whose workgroups each fold the partials in a fixed order
// (deterministic) for the global counts, the first one also writing loss_out[5].
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

constexpr int kLossThreads = 256;
constexpr int kLossMaxBlocks = 1024;

struct RayTerms {
    float l1, cosc;  // |D^ - D| M_D, (1 - cos) M_N
    uint32_t mD, mN;
};

__device__ __forceinline__ RayTerms ray_terms(int64_t r, const float *__restrict__ depth,
                                              const float *__restrict__ normal, const float *__restrict__ td,
                                              const float *__restrict__ tn)
{
    RayTerms o{0.f, 0.f, 0u, 0u};
    float D = td[r];
    if (!(D > 0.f)) return o;
    o.mD = 1u;
    o.l1 = fabsf(depth[r] - D);
    float t0 = tn[3 * r], t1 = tn[3 * r + 1], t2 = tn[3 * r + 2];
    if (fmaf(t0, t0, fmaf(t1, t1, t2 * t2)) > 0.f) {
        o.mN = 1u;
        float n0 = normal[3 * r], n1 = normal[3 * r + 1], n2 = normal[3 * r + 2];
        float nn = sqrtf(fmaf(n0, n0, fmaf(n1, n1, n2 * n2)));
        o.cosc = nn > 0.f ? 1.f - fmaf(n0, t0, fmaf(n1, t1, n2 * t2)) / nn : 1.f;
    }
    return o;
}

__global__ __launch_bounds__(kLossThreads) void loss_partials(int64_t n, const float *__restrict__ depth,
                                                              const float *__restrict__ normal,
                                                              const float *__restrict__ td,
                                                              const float *__restrict__ tn,
                                                              float *__restrict__ partials)
{
    float l1 = 0.f, cs = 0.f;
    uint32_t cD = 0, cN = 0;
    for (int64_t r = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * kLossThreads) {
        RayTerms t = ray_terms(r, depth, normal, td, tn);
        l1 += t.l1;
        cs += t.cosc;
        cD += t.mD;
        cN += t.mN;
    }
    __shared__ float s_l1[kLossThreads], s_cs[kLossThreads];
    __shared__ uint32_t s_cD[kLossThreads], s_cN[kLossThreads];
    const int t = threadIdx.x;
    s_l1[t] = l1;
    s_cs[t] = cs;
    s_cD[t] = cD;
    s_cN[t] = cN;
    __syncthreads();
    for (int o = kLossThreads / 2; o > 0; o >>= 1) {
        if (t < o) {
            s_l1[t] += s_l1[t + o];
            s_cs[t] += s_cs[t + o];
            s_cD[t] += s_cD[t + o];
            s_cN[t] += s_cN[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        float *q = partials + 4 * blockIdx.x;
        q[0] = s_l1[0];
        q[1] = s_cs[0];
        q[2] = __uint_as_float(s_cD[0]);
        q[3] = __uint_as_float(s_cN[0]);
    }
}

// Per-ray gradient.  It needs the global counts: every workgroup first folds the partials
// (thread t adds partials t, t + 256, ... in order, then a fixed tree folds the 256 sums;
// counts are exact integers, the float sums come out the same in every workgroup), and
// workgroup 0 writes loss_out.  This saves a separate one-workgroup launch.
__global__ __launch_bounds__(kLossThreads) void loss_grad(int64_t n, const float *__restrict__ depth,
                                                          const float *__restrict__ normal,
                                                          const float *__restrict__ td,
                                                          const float *__restrict__ tn, float w_depth,
                                                          float lambda_n, float lambda_ng, int nb,
                                                          const float *__restrict__ partials,
                                                          float *__restrict__ loss_out, float *__restrict__ gD,
                                                          float *__restrict__ gA, float *__restrict__ gN)
{
    __shared__ float s1[kLossThreads], s2[kLossThreads];
    __shared__ uint32_t k1[kLossThreads], k2[kLossThreads];
    const int t = threadIdx.x;
    {
        float l1 = 0.f, cs = 0.f;
        uint32_t cD = 0, cN = 0;
        for (int b = t; b < nb; b += kLossThreads) {
            l1 += partials[4 * b];
            cs += partials[4 * b + 1];
            cD += __float_as_uint(partials[4 * b + 2]);
            cN += __float_as_uint(partials[4 * b + 3]);
        }
        s1[t] = l1;
        s2[t] = cs;
        k1[t] = cD;
        k2[t] = cN;
        __syncthreads();
        for (int o = kLossThreads / 2; o > 0; o >>= 1) {
            if (t < o) {
                s1[t] += s1[t + o];
                s2[t] += s2[t + o];
                k1[t] += k1[t + o];
                k2[t] += k2[t + o];
            }
            __syncthreads();
        }
    }
    const uint32_t nD = k1[0], nN = k2[0];
    if (blockIdx.x == 0 && t == 0) {
        const float td0 = nD ? w_depth * s1[0] / (float)nD : 0.f;
        const float tn0 = nN ? lambda_n * lambda_ng * s2[0] / (float)nN : 0.f;
        loss_out[0] = td0 + tn0;
        loss_out[1] = td0;
        loss_out[2] = tn0;
        loss_out[3] = (float)nD;
        loss_out[4] = (float)nN;
    }
    const int64_t r = (int64_t)blockIdx.x * kLossThreads + threadIdx.x;
    if (r >= n) return;
    const float cD = (float)nD, cN = (float)nN;
    float gd = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
    float D = td[r];
    if (D > 0.f) {
        float diff = depth[r] - D;
        float sgn = diff > 0.f ? 1.f : (diff < 0.f ? -1.f : 0.f);
        gd = w_depth * sgn / cD;
        float t0 = tn[3 * r], t1 = tn[3 * r + 1], t2 = tn[3 * r + 2];
        if (fmaf(t0, t0, fmaf(t1, t1, t2 * t2)) > 0.f) {
            float n0 = normal[3 * r], n1 = normal[3 * r + 1], n2 = normal[3 * r + 2];
            float nn2 = fmaf(n0, n0, fmaf(n1, n1, n2 * n2));
            if (nn2 > 0.f) {
                float nn = sqrtf(nn2);
                float cosv = fmaf(n0, t0, fmaf(n1, t1, n2 * t2)) / nn;
                float f = -lambda_n * lambda_ng / (cN * nn);
                float cn = cosv / nn;
                g0 = f * fmaf(-cn, n0, t0);
                g1 = f * fmaf(-cn, n1, t1);
                g2 = f * fmaf(-cn, n2, t2);
            }
        }
    }
    gD[r] = gd;
    gA[r] = 0.f;
    gN[3 * r] = g0;
    gN[3 * r + 1] = g1;
    gN[3 * r + 2] = g2;
}

int loss_blocks(int64_t n_rays)
{
    int64_t b = (n_rays + kLossThreads - 1) / kLossThreads;  // one ray per thread up to kLossMaxBlocks
    if (b < 1) b = 1;
    if (b > kLossMaxBlocks) b = kLossMaxBlocks;
    return (int)b;
}

hipError_t launch_loss(int64_t n_rays, const float *depth, const float *normal, const float *td, const float *tn,
                       float w_depth, float lambda_n, float lambda_ng, float *partials, float *loss_out,
                       float *gD, float *gA, float *gN, hipStream_t s)
{
    int nb = loss_blocks(n_rays);
    loss_partials<<<nb, kLossThreads, 0, s>>>(n_rays, depth, normal, td, tn, partials);
    const int64_t gb = n_rays > 0 ? (n_rays + kLossThreads - 1) / kLossThreads : 1;
    loss_grad<<<(unsigned)gb, kLossThreads, 0, s>>>(n_rays, depth, normal, td, tn, w_depth, lambda_n, lambda_ng, nb,
                                                     partials, loss_out, gD, gA, gN);
    return hipGetLastError();
}

}  // namespace lgsr
