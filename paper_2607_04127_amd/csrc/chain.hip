// chain.hip -- record-space gradients -> surfel parameters and the 6-DoF pose.
//
// The backward raster leaves, per surfel, dL/d(nt, c, cu, U, cv, V, alpha) summed over rays
// (the slots of surfels with a ray rectangle, the only ones the raster writes, are cleared
// here after they are read, so the next backward finds every slot zero),
// where the hit test evaluates u = (cu + U.(d - m)) / den with cu = U.m (likewise v).  With
//   nt = sigma n',  c = nt . mu',  U = sigma (na x mu') / s0,  V = sigma (mu' x bn) / s1,
//   na = n' x a',  bn = b' x n'
// (sigma piecewise constant) the total U gradient is gU + gcu m, and with w = mu' x m
//   dmu' = gc nt + (sigma/s0) (gU + gcu m) x na + (sigma/s1) bn x (gV + gcv m)
//   dbn  = (sigma/s1) (gV x mu' - gcv w),   dna = (sigma/s0) (mu' x gU + gcu w)
//   da'  = dna x n',   db' = n' x dbn,
//   dn'  = sigma (gnt + (r gcm - (nt.zeta) gci) m + gc zeta) + a' x dna + dbn x b',
//   zeta = mu' - r m
//   ds0  = -(gU.U + gcu cu) / s0,   ds1 = -(gV.V + gcv cv) / s1
// (U is nearly perpendicular to m, so these forms avoid the cancellation that products with
// the unsplit gradient would suffer; gnt already holds the part of the hit-distance
// derivative along d - m, and the terms in m and zeta the rest), then world frame (multiply by R), the rotation columns
// (a, b, n) of the normalised quaternion and its normalisation, s~ = log s (Sec. 3.3) and
// alpha = sigmoid(o).  Pose, right perturbation T Exp(xi): drho = -sum dmu', domega =
// -sum(mu' x dmu' + a' x da' + b' x db' + n' x dn'); per-block partials are folded by one
// block in a fixed order with compensated sums, so the pose gradient is deterministic given
// the record gradients.
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

namespace lgsr {

constexpr int kChainThreads = 256;

__device__ __forceinline__ void cross(const float *x, const float *y, float *o)
{
    o[0] = x[1] * y[2] - x[2] * y[1];
    o[1] = x[2] * y[0] - x[0] * y[2];
    o[2] = x[0] * y[1] - x[1] * y[0];
}

__device__ __forceinline__ Pose load_pose(const float *__restrict__ pd)
{
    Pose P;
    for (int c = 0; c < 9; ++c) P.r[c] = pd[(c / 3) * 4 + (c % 3)];
    for (int c = 0; c < 3; ++c) P.t[c] = pd[4 * c + 3];
    return P;
}

__global__ __launch_bounds__(kChainThreads) void chain_kernel(SurfelPtrs S, const float *__restrict__ pose_dev,
                                                              RasterParams p, const uint2 *__restrict__ rects,
                                                              float *__restrict__ recgrad,
                                                              float *__restrict__ dm, float *__restrict__ dq,
                                                              float *__restrict__ dls, float *__restrict__ dlog,
                                                              float *__restrict__ partials)
{
    const Pose P = load_pose(pose_dev);
    const int64_t i = (int64_t)blockIdx.x * kChainThreads + threadIdx.x;
    float pr[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < S.n) {
        Geom g = project_geom(S.means, S.quats, S.log_scales, S.logits, i, P, p.near);
        float out_m[3] = {0.f, 0.f, 0.f}, out_q[4] = {0.f, 0.f, 0.f, 0.f}, out_s[2] = {0.f, 0.f}, out_o = 0.f;
        // only surfels with a ray rectangle (from the forward) can have a written slot
        const bool listed = (rects[i].y >> 16) > 0u;
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f), y = x, z = x, zz = x;
        if (listed) {
            float4 *G4 = reinterpret_cast<float4 *>(recgrad + (size_t)i * kGrad);
            x = G4[0];
            y = G4[1];
            z = G4[2];
            zz = G4[3];
            // leave the slot zero for the next backward
            const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
            G4[0] = z4;
            G4[1] = z4;
            G4[2] = z4;
            G4[3] = z4;
        }
        if (g.valid && listed) {
            const RecParts q = record_parts(g);
            const float gnt[3] = {x.x, x.y, x.z}, gc = x.w;
            const float gcu = y.x, gU[3] = {y.y, y.z, y.w};
            const float gcv = z.x, gV[3] = {z.y, z.z, z.w};
            const float ga = zz.x, gcm = zz.y, gci = zz.z;
            float mu[3] = {g.mh[0] + g.ml[0], g.mh[1] + g.ml[1], g.mh[2] + g.ml[2]};
            const float k0 = g.sigma / g.s0, k1 = g.sigma / g.s1;
            float gUt[3], gVt[3];
            for (int c = 0; c < 3; ++c) {
                gUt[c] = fmaf(gcu, q.m[c], gU[c]);
                gVt[c] = fmaf(gcv, q.m[c], gV[c]);
            }
            float t1[3], t2[3];
            cross(gUt, q.na, t1);
            cross(q.bn, gVt, t2);
            float gmu[3], gna[3], gbn[3], gav[3], gbv[3], gnv[3];
            for (int c = 0; c < 3; ++c) gmu[c] = gc * q.nt[c] + k0 * t1[c] + k1 * t2[c];
            cross(gV, mu, t1);
            cross(mu, gU, t2);
            for (int c = 0; c < 3; ++c) {
                gbn[c] = k1 * fmaf(-gcv, q.w[c], t1[c]);
                gna[c] = k0 * fmaf(gcu, q.w[c], t2[c]);
            }
            // na = n' x a', bn = b' x n'
            float t3[3], t4[3];
            cross(gna, g.n, gav);
            cross(g.n, gbn, gbv);
            cross(g.a, gna, t3);
            cross(gbn, g.b, t4);
            // zeta = mu' - r m: mh - r m rounded once (it is of the order of r times the
            // roundoff of m), plus the low part of the centre
            float zeta[3];
            for (int c = 0; c < 3; ++c) zeta[c] = fmaf(-g.r, q.m[c], g.mh[c]) + g.ml[c];
            const float ntz = fmaf(q.nt[0], zeta[0], fmaf(q.nt[1], zeta[1], q.nt[2] * zeta[2]));
            const float cm = fmaf(gcm, g.r, -gci * ntz);
            for (int c = 0; c < 3; ++c)
                gnv[c] = g.sigma * fmaf(gc, zeta[c], fmaf(cm, q.m[c], gnt[c])) + t3[c] + t4[c];
            const float gs0 = -fmaf(gcu, q.cu, gU[0] * q.U[0] + gU[1] * q.U[1] + gU[2] * q.U[2]) / g.s0;
            const float gs1 = -fmaf(gcv, q.cv, gV[0] * q.V[0] + gV[1] * q.V[1] + gV[2] * q.V[2]) / g.s1;
            // world frame
            float Ga[3], Gb[3], Gn[3];
            rot(P, gmu, out_m);
            rot(P, gav, Ga);
            rot(P, gbv, Gb);
            rot(P, gnv, Gn);
            // columns of R(qhat): a = (1-2(y2+z2), 2(xy+wz), 2(xz-wy)), b = (2(xy-wz), 1-2(x2+z2),
            // 2(yz+wx)), n = (2(xz+wy), 2(yz-wx), 1-2(x2+y2))
            float w = g.qh[0], qx = g.qh[1], qy = g.qh[2], qz = g.qh[3];
            float dw = 2.f * (Ga[1] * qz - Ga[2] * qy - Gb[0] * qz + Gb[2] * qx + Gn[0] * qy - Gn[1] * qx);
            float dx = 2.f * (Ga[1] * qy + Ga[2] * qz + Gb[0] * qy + Gb[2] * w + Gn[0] * qz - Gn[1] * w)
                     - 4.f * (Gb[1] * qx + Gn[2] * qx);
            float dy = 2.f * (Ga[1] * qx - Ga[2] * w + Gb[0] * qx + Gb[2] * qz + Gn[0] * w + Gn[1] * qz)
                     - 4.f * (Ga[0] * qy + Gn[2] * qy);
            float dz = 2.f * (Ga[1] * w + Ga[2] * qx - Gb[0] * w + Gb[2] * qy + Gn[0] * qx + Gn[1] * qy)
                     - 4.f * (Ga[0] * qz + Gb[1] * qz);
            float radial = dw * w + dx * qx + dy * qy + dz * qz;
            float iq = 1.f / g.qn;
            out_q[0] = (dw - radial * w) * iq;
            out_q[1] = (dx - radial * qx) * iq;
            out_q[2] = (dy - radial * qy) * iq;
            out_q[3] = (dz - radial * qz) * iq;
            out_s[0] = g.s0 * gs0;
            out_s[1] = g.s1 * gs1;
            out_o = g.alpha * (1.f - g.alpha) * ga;
            float c1[3], c2[3], c3[3], c4[3];
            cross(mu, gmu, c1);
            cross(g.a, gav, c2);
            cross(g.b, gbv, c3);
            cross(g.n, gnv, c4);
            for (int c = 0; c < 3; ++c) {
                pr[c] = -gmu[c];
                pr[3 + c] = -(c1[c] + c2[c] + c3[c] + c4[c]);
            }
        }
        for (int c = 0; c < 3; ++c) dm[3 * i + c] = out_m[c];
        for (int c = 0; c < 4; ++c) dq[4 * i + c] = out_q[c];
        dls[2 * i] = out_s[0];
        dls[2 * i + 1] = out_s[1];
        dlog[i] = out_o;
    }
    // block reduction of the pose terms: wave butterfly, then the 4 wave sums in order
    __shared__ float ws[4][6];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        float v = pr[c];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) ws[wv][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        int c = threadIdx.x;
        partials[(size_t)blockIdx.x * 6 + c] = ((ws[0][c] + ws[1][c]) + ws[2][c]) + ws[3][c];
    }
}

// 6 x 256 threads: thread (c, t) sums partials t, t + 256, ... of component c with
// Neumaier compensation; the 256 (sum, compensation) pairs are then folded in a fixed tree.
__global__ __launch_bounds__(256) void pose_finalize(int nb, const float *__restrict__ partials,
                                                     float *__restrict__ grad_pose)
{
    __shared__ float ss[256], cc[256];
    const int c = blockIdx.x, t = threadIdx.x;
    float s = 0.f, comp = 0.f;
    for (int b = t; b < nb; b += 256) {
        const float x = partials[(size_t)b * 6 + c];
        const float y = s + x;
        comp += fabsf(s) >= fabsf(x) ? (s - y) + x : (x - y) + s;
        s = y;
    }
    ss[t] = s;
    cc[t] = comp;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            const float a = ss[t], x = ss[t + o];
            const float y = a + x;
            cc[t] += cc[t + o] + (fabsf(a) >= fabsf(x) ? (a - y) + x : (x - y) + a);
            ss[t] = y;
        }
        __syncthreads();
    }
    if (t == 0) grad_pose[c] = ss[0] + cc[0];
}

int chain_blocks(int64_t n) { return n > 0 ? (int)((n + kChainThreads - 1) / kChainThreads) : 1; }

hipError_t launch_chain(const SurfelPtrs &S, const float *pose_dev, const RasterParams &p, const uint2 *rects,
                        float *recgrad,
                        float *d_means, float *d_quats, float *d_log_scales, float *d_logits, float *pose_partials,
                        float *grad_pose, hipStream_t s)
{
    int nb = chain_blocks(S.n);
    chain_kernel<<<nb, kChainThreads, 0, s>>>(S, pose_dev, p, rects, recgrad, d_means, d_quats, d_log_scales,
                                             d_logits, pose_partials);
    pose_finalize<<<6, 256, 0, s>>>(nb, pose_partials, grad_pose);
    return hipGetLastError();
}

}  // namespace lgsr
