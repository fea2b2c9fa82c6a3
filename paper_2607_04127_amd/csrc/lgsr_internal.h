// lgsr_internal.h -- device-side building blocks of the gfx950 surfel renderer.
//
// Formulation used on the GPU (equal in exact arithmetic to the plain definition of
// arXiv 2607.04127 Sec. 3.1 / Sec. 3.4 with the 2DGS surfel of Sec. 1):
//   sensor frame: mu' = R^T (mu - t), a' = R^T a, b' = R^T b, n' = R^T n, r = |mu'|;
//   sigma = +1 if n'.mu' <= 0 else -1, nt = sigma n' (the normal facing the sensor);
//   ray d: den = nt.d, hit range t = c / den with c = nt.mu' (<= 0),
//          u = nu / den, v = nv / den  with nu = U.d, nv = V.d,
//          U = sigma ((n' x a') x mu') / s0,  V = sigma (mu' x (b' x n')) / s1
//   (homogeneous form of the ray/plane hit: by the vector triple product,
//   (t d - mu') . a' / s0 = U.d / den for any three vectors a', b', n'; for an exactly
//   orthonormal frame n' x a' = b' and b' x n' = a').  The frame itself is only as
//   orthonormal as float32 allows (the pose rotation is a float32 input), so the record is
//   built from n' x a' and b' x n' rather than from b' and a': u and v then follow the
//   definition for the frame the kernels hold.
// At grazing incidence den is small and t, u, v are sensitive to the plane normal in
// proportion to 1/den, so the frame is formed from the quaternion and the pose in float
// pairs and rounded once (sensor_frame below).
// U.d nearly cancels for rays near the surfel centre (|U| ~ r / s), so it is evaluated as
//   nu = cu + U . ((d_hi - m) + d_lo),   cu = U . m computed from an error-compensated mu',
// where m is the float32 unit direction of the centre and d = d_hi + d_lo the exact ray
// direction (cos phi cos th is a product of two float32 values, split exactly by an FMA).
// The float32 rounding of U then only multiplies the small vector d - m.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lgsr {

constexpr int kTile = 16;      // tile edge in rays: a tile is 16 x 16 rays with one surfel list
constexpr int kSub = 8;        // wave sub-tile edge: 8 x 8 rays, one wavefront of 64 lanes
constexpr int kRec = 16;       // floats per surfel record
// Per-tile pair counters are split into kShards by the projection workgroup of the surfel
// (workgroup index mod kShards) so that no single counter takes an atomic from every
// workgroup; a tile's list is the concatenation of its shards.
constexpr int kShards = 8;
constexpr int kGrad = 16;      // floats per surfel record-gradient slot (kGradUsed used)
constexpr int kGradUsed = 15;
constexpr uint32_t kCulledKey = 0x7FFFFFFFu;  // depth key of a surfel that renders nothing

// Record layout (float index).
enum : int {
    R_NT = 0,   // 0..2 sensor-facing normal nt
    R_C = 3,    // c = nt . mu'
    R_U = 4,    // 4..6 U
    R_CU = 7,   // cu = U . m (compensated)
    R_V = 8,    // 8..10 V
    R_CV = 11,  // cv = V . m (compensated)
    R_M = 12,   // 12..14 m = mu' / r
    R_ALPHA = 15
};

// Record-gradient layout (float index): dL/d(nt, c, U, V, alpha) summed over rays.
// Record gradients.  u = (cu + U.(d - m)) / den is differentiated in that split: G_CU
// accumulates dL/dnu and G_U the vector dL/dnu (d - m), so that the chain rule meets U only
// through products that do not cancel (U is nearly perpendicular to m, and the rays near m).
// Likewise the hit distance t = c / den: its derivative in nt is -g delta, g = dL/dc =
// (dL/dt) / den, delta = t d - mu'.  With the record's rounded m, zeta = mu' - r m (about r
// times the float32 unit roundoff) and e = d - m,
//   delta = t e + (t - r) m - zeta,   t - r = (nt.zeta - r nt.e) / den,
// so G_NT takes -g t e per hit, G_CM the sum of g (nt.e) / den and G_CI the sum of g / den,
// and the chain adds (r G_CM - (nt.zeta) G_CI) m + G_C zeta.  Forming -g t d per hit and
// adding G_C mu' once per surfel instead would cancel two terms of size r to one of size
// |delta|, and treating m as exactly mu' / r would leave an error of g |zeta|: both are
// r / |delta| times the roundoff, large for a far, small surfel hit near its centre.  G_C
// (dL/dc) also carries the centre gradient.
enum : int { G_NT = 0, G_C = 3, G_CU = 4, G_U = 5, G_CV = 8, G_V = 9, G_ALPHA = 12, G_CM = 13, G_CI = 14 };

struct Pose {
    float r[9];  // row-major rotation sensor -> world
    float t[3];
};

struct RasterParams {
    float k2;  // cutoff_sigma^2
    float alpha_thr, alpha_max, T_min, near, den_eps, drop_tau;
    float cutoff;
};

struct Grid {
    int H, W;    // rays
    int TH, TW;  // tiles
    int T;       // TH * TW
};

// Tile numbering is column-major so that consecutive tiles form azimuth sectors.
__host__ __device__ inline int tile_id(int tr, int tc, int TH) { return tc * TH + tr; }

// ----------------------------------------------------------------------------------------
// error-free transformations (float32)
// ----------------------------------------------------------------------------------------

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void two_prod(float a, float b, float &p, float &e)
{
    p = a * b;
    e = fmaf(a, b, -p);
}

// a*b - c*d with about one rounding (Kahan's FMA difference of products)
__device__ __forceinline__ float diff_prod(float a, float b, float c, float d)
{
    float w = c * d;
    float e = fmaf(-c, d, w);
    float f = fmaf(a, b, -w);
    return f + e;
}

// Unevaluated float pair h + l.  Sums are not renormalised after every step: the pairs
// below combine a handful of terms and are rounded once at the end.
struct F2 {
    float h, l;
};

__device__ __forceinline__ F2 f2_mul(float a, float b)
{
    F2 r;
    two_prod(a, b, r.h, r.l);
    return r;
}

__device__ __forceinline__ F2 f2_add(F2 x, F2 y)
{
    F2 r;
    two_sum(x.h, y.h, r.h, r.l);
    r.l += x.l + y.l;
    return r;
}

__device__ __forceinline__ F2 f2_neg(F2 x) { return F2{-x.h, -x.l}; }
__device__ __forceinline__ F2 f2_twice(F2 x) { return F2{2.f * x.h, 2.f * x.l}; }

// x y for pairs, to about 2^-46 relative: the low-order cross terms are added to the exact
// product of the high parts
__device__ __forceinline__ F2 f2_mul2(F2 x, F2 y)
{
    F2 r = f2_mul(x.h, y.h);
    r.l = fmaf(x.h, y.l, fmaf(x.l, y.h, r.l));
    return r;
}

// o = x cross y, float32 inputs, exact as float pairs
__device__ __forceinline__ void cross_f2(const float *x, const float *y, F2 *o)
{
    o[0] = f2_add(f2_mul(x[1], y[2]), f2_neg(f2_mul(x[2], y[1])));
    o[1] = f2_add(f2_mul(x[2], y[0]), f2_neg(f2_mul(x[0], y[2])));
    o[2] = f2_add(f2_mul(x[0], y[1]), f2_neg(f2_mul(x[1], y[0])));
}

// o = x cross y for pair vectors
__device__ __forceinline__ void cross_f2f2(const F2 *x, const F2 *y, F2 *o)
{
    o[0] = f2_add(f2_mul2(x[1], y[2]), f2_neg(f2_mul2(x[2], y[1])));
    o[1] = f2_add(f2_mul2(x[2], y[0]), f2_neg(f2_mul2(x[0], y[2])));
    o[2] = f2_add(f2_mul2(x[0], y[1]), f2_neg(f2_mul2(x[1], y[0])));
}

// ----------------------------------------------------------------------------------------
// per-surfel projection (shared by the projection and the chain-rule kernels)
// ----------------------------------------------------------------------------------------

// Sensor-frame rotation columns a' = R^T a, b' = R^T b, n' = R^T n of the normalised
// quaternion q / |q|, each component rounded once.  With qq = |q|^2 the columns of R(q/|q|)
// are the columns of the homogeneous quaternion matrix divided by qq:
//   a = (w2+x2-y2-z2, 2(xy+wz), 2(xz-wy)) / qq,  b = (2(xy-wz), w2-x2+y2-z2, 2(yz+wx)) / qq,
//   n = (2(xz+wy), 2(yz-wx), w2-x2-y2+z2) / qq.
// Every product of two inputs is exact as a float pair, so the numerators, the rotation by
// the pose and the division carry errors of order 2^-44, far below one float32 rounding.
__device__ __forceinline__ void sensor_frame(const float *q, const Pose &P, float *a, float *b, float *n)
{
    const float w = q[0], x = q[1], y = q[2], z = q[3];
    const F2 ww = f2_mul(w, w), xx = f2_mul(x, x), yy = f2_mul(y, y), zz = f2_mul(z, z);
    const F2 xy = f2_mul(x, y), wz = f2_mul(w, z), xz = f2_mul(x, z), wy = f2_mul(w, y);
    const F2 yz = f2_mul(y, z), wx = f2_mul(w, x);
    const F2 wwxx = f2_add(ww, xx), yyzz = f2_add(yy, zz), wwyy = f2_add(ww, yy), xxzz = f2_add(xx, zz);
    const F2 wwzz = f2_add(ww, zz), xxyy = f2_add(xx, yy);
    F2 col[3][3];  // world columns times qq: col[c][k], c = a, b, n
    col[0][0] = f2_add(wwxx, f2_neg(yyzz));
    col[0][1] = f2_twice(f2_add(xy, wz));
    col[0][2] = f2_twice(f2_add(xz, f2_neg(wy)));
    col[1][0] = f2_twice(f2_add(xy, f2_neg(wz)));
    col[1][1] = f2_add(wwyy, f2_neg(xxzz));
    col[1][2] = f2_twice(f2_add(yz, wx));
    col[2][0] = f2_twice(f2_add(xz, wy));
    col[2][1] = f2_twice(f2_add(yz, f2_neg(wx)));
    col[2][2] = f2_add(wwzz, f2_neg(xxyy));
    const F2 qq = f2_add(wwxx, yyzz);
    const float iq = 1.f / qq.h;
    float *out[3] = {a, b, n};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // (R^T col)_j = sum_k R[k][j] col[k]
            F2 acc = f2_mul(P.r[j], col[c][0].h);
            acc.l = fmaf(P.r[j], col[c][0].l, acc.l);
#pragma unroll
            for (int k = 1; k < 3; ++k) {
                F2 t = f2_mul(P.r[3 * k + j], col[c][k].h);
                t.l = fmaf(P.r[3 * k + j], col[c][k].l, t.l);
                acc = f2_add(acc, t);
            }
            // (acc.h + acc.l) / (qq.h + qq.l): one correction of the rounded quotient
            const float q0 = acc.h * iq;
            const float rem = fmaf(-q0, qq.h, acc.h) + fmaf(-q0, qq.l, acc.l);
            out[c][j] = fmaf(rem, iq, q0);
        }
    }
}

struct Geom {
    float mh[3], ml[3];  // mu' = mh + ml (compensated)
    float a[3], b[3], n[3];
    float qh[4], qn;
    float s0, s1, alpha, r, sigma;
    bool valid;
};

// v = R v'
__device__ __forceinline__ void rot(const Pose &P, const float *v, float *o)
{
    for (int i = 0; i < 3; ++i) o[i] = fmaf(P.r[3 * i], v[0], fmaf(P.r[3 * i + 1], v[1], P.r[3 * i + 2] * v[2]));
}

__device__ __forceinline__ Geom project_geom(const float *__restrict__ means, const float *__restrict__ quats,
                                             const float *__restrict__ log_scales,
                                             const float *__restrict__ logits, int64_t i, const Pose &P,
                                             float near)
{
    Geom g;
    float q[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
    float qq = fmaf(q[0], q[0], fmaf(q[1], q[1], fmaf(q[2], q[2], q[3] * q[3])));
    g.qn = sqrtf(qq);
    g.valid = g.qn > 0.f && isfinite(g.qn);
    float inv = g.valid ? 1.f / g.qn : 0.f;
    for (int c = 0; c < 4; ++c) g.qh[c] = q[c] * inv;
    if (g.valid) {
        sensor_frame(q, P, g.a, g.b, g.n);
    } else {
        for (int c = 0; c < 3; ++c) g.a[c] = g.b[c] = g.n[c] = 0.f;
    }
    // mu - t exactly as a float pair, then R^T (.) with compensated sums
    float dh[3], dl[3];
    for (int c = 0; c < 3; ++c) two_sum(means[3 * i + c], -P.t[c], dh[c], dl[c]);
    for (int j = 0; j < 3; ++j) {
        float s = 0.f, comp = 0.f;
        for (int k = 0; k < 3; ++k) {
            float p, pe, se;
            two_prod(P.r[3 * k + j], dh[k], p, pe);
            two_sum(s, p, s, se);
            comp += pe + se + P.r[3 * k + j] * dl[k];
        }
        float hi, lo;
        two_sum(s, comp, hi, lo);
        g.mh[j] = hi;
        g.ml[j] = lo;
    }
    g.s0 = expf(log_scales[2 * i]);
    g.s1 = expf(log_scales[2 * i + 1]);
    g.alpha = 1.f / (1.f + expf(-logits[i]));
    // r = |mu'| from the compensated centre: r^2 as a pair (exact squares of the high parts,
    // cross terms 2 mh ml), then one Newton correction of the float32 square root.  The range
    // key orders the lists, so r is within about half an ulp of |mu'|: two centres can only
    // compare in the wrong order when their ranges differ by less than 2^-22 relative.
    {
        F2 rr = f2_add(f2_add(f2_mul(g.mh[0], g.mh[0]), f2_mul(g.mh[1], g.mh[1])), f2_mul(g.mh[2], g.mh[2]));
        rr.l = fmaf(2.f * g.mh[0], g.ml[0], fmaf(2.f * g.mh[1], g.ml[1], fmaf(2.f * g.mh[2], g.ml[2], rr.l)));
        const float r0 = sqrtf(rr.h);
        const float res = fmaf(-r0, r0, rr.h) + rr.l;
        g.r = r0 > 0.f ? fmaf(res, 0.5f / r0, r0) : r0;
    }
    float nm = fmaf(g.n[0], g.mh[0], fmaf(g.n[1], g.mh[1], g.n[2] * g.mh[2]))
             + fmaf(g.n[0], g.ml[0], fmaf(g.n[1], g.ml[1], g.n[2] * g.ml[2]));
    g.sigma = nm <= 0.f ? 1.f : -1.f;
    g.valid = g.valid && g.r >= near && isfinite(g.r) && isfinite(g.s0) && isfinite(g.s1) && g.s0 > 0.f &&
              g.s1 > 0.f && isfinite(g.alpha);
    return g;
}

// Record of a projected surfel (layout above).
// The record quantities of a projected surfel.  The chain rule calls this too, so both see
// bit-identical values.
struct RecParts {
    float nt[3], c, m[3], w[3], na[3], bn[3], U[3], cu, V[3], cv;
};

__device__ __forceinline__ RecParts record_parts(const Geom &g)
{
    RecParts q;
    for (int k = 0; k < 3; ++k) q.nt[k] = g.sigma * g.n[k];
    q.c = fmaf(q.nt[0], g.mh[0], fmaf(q.nt[1], g.mh[1], q.nt[2] * g.mh[2]))
        + fmaf(q.nt[0], g.ml[0], fmaf(q.nt[1], g.ml[1], q.nt[2] * g.ml[2]));
    float ir = 1.f / g.r;
    for (int k = 0; k < 3; ++k) q.m[k] = g.mh[k] * ir;
    // w = mu' x m, small: accurate difference of products on the high part + low part
    q.w[0] = diff_prod(g.mh[1], q.m[2], g.mh[2], q.m[1]) + (g.ml[1] * q.m[2] - g.ml[2] * q.m[1]);
    q.w[1] = diff_prod(g.mh[2], q.m[0], g.mh[0], q.m[2]) + (g.ml[2] * q.m[0] - g.ml[0] * q.m[2]);
    q.w[2] = diff_prod(g.mh[0], q.m[1], g.mh[1], q.m[0]) + (g.ml[0] * q.m[1] - g.ml[1] * q.m[0]);
    float i0 = g.sigma / g.s0, i1 = g.sigma / g.s1;
    // na = n' x a' (b' for an orthonormal frame), bn = b' x n' (a'), exact as float pairs
    F2 na[3], bn[3];
    cross_f2(g.n, g.a, na);
    cross_f2(g.b, g.n, bn);
    // U = sigma (na x mu') / s0, V = sigma (mu' x bn) / s1 from the pairs and the compensated
    // centre, rounded once.  A grazing ray (small n'.d) would amplify any rounding of na, bn
    // or mu' inside U, V by 1 / |n'.d|: U.d / den changes by (delta x mu').d / den for an
    // error delta in na; only errors of the form R^T(delta a) cancel against den.
    const F2 mu[3] = {{g.mh[0], g.ml[0]}, {g.mh[1], g.ml[1]}, {g.mh[2], g.ml[2]}};
    F2 Uc[3], Vc[3];
    cross_f2f2(na, mu, Uc);
    cross_f2f2(mu, bn, Vc);
    for (int k = 0; k < 3; ++k) {
        q.na[k] = na[k].h + na[k].l;
        q.bn[k] = bn[k].h + bn[k].l;
        q.U[k] = fmaf(Uc[k].h, i0, Uc[k].l * i0);
        q.V[k] = fmaf(Vc[k].h, i1, Vc[k].l * i1);
    }
    // U . m = sigma na.(mu' x m) / s0,   V . m = -sigma bn.(mu' x m) / s1
    q.cu = fmaf(q.na[0], q.w[0], fmaf(q.na[1], q.w[1], q.na[2] * q.w[2])) * i0;
    q.cv = -fmaf(q.bn[0], q.w[0], fmaf(q.bn[1], q.w[1], q.bn[2] * q.w[2])) * i1;
    return q;
}

__device__ __forceinline__ void make_record(const Geom &g, float *rec)
{
    const RecParts q = record_parts(g);
    rec[R_NT + 0] = q.nt[0]; rec[R_NT + 1] = q.nt[1]; rec[R_NT + 2] = q.nt[2];
    rec[R_C] = q.c;
    rec[R_U + 0] = q.U[0]; rec[R_U + 1] = q.U[1]; rec[R_U + 2] = q.U[2];
    rec[R_CU] = q.cu;
    rec[R_V + 0] = q.V[0]; rec[R_V + 1] = q.V[1]; rec[R_V + 2] = q.V[2];
    rec[R_CV] = q.cv;
    rec[R_M + 0] = q.m[0]; rec[R_M + 1] = q.m[1]; rec[R_M + 2] = q.m[2];
    rec[R_ALPHA] = g.alpha;
}

// ----------------------------------------------------------------------------------------
// rays and the per-(ray, surfel) hit test (shared bit-for-bit by forward and backward)
// ----------------------------------------------------------------------------------------

struct Ray {
    float dh[3];  // float32 direction
    float dl[2];  // exact residuals of the two products (the z component is exact)
};

__device__ __forceinline__ Ray make_ray(const float *__restrict__ rows, const float *__restrict__ cols, int k, int j)
{
    Ray r;
    float sp = rows[2 * k], cp = rows[2 * k + 1];
    float st = cols[2 * j], ct = cols[2 * j + 1];
    r.dh[0] = cp * ct;
    r.dh[1] = cp * st;
    r.dh[2] = sp;
    r.dl[0] = fmaf(cp, ct, -r.dh[0]);
    r.dl[1] = fmaf(cp, st, -r.dh[1]);
    return r;
}

struct Hit {
    float e[3];  // d - m
    float den, inv, nu, nv, t, G, aG, ah;
    bool pass;
};

// Record fields are passed by value so that wave-uniform loads stay in scalar registers.
struct Rec {
    float nt0, nt1, nt2, c, U0, U1, U2, cu, V0, V1, V2, cv, m0, m1, m2, alpha;
};

__device__ __forceinline__ Rec load_rec(const float *__restrict__ recs, uint32_t id)
{
    const float4 *p = reinterpret_cast<const float4 *>(recs + (size_t)id * kRec);
    float4 x = p[0], y = p[1], z = p[2], w = p[3];
    return Rec{x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w, z.x, z.y, z.z, z.w, w.x, w.y, w.z, w.w};
}

// -log2(e) / 2: G = exp(-q2 / 2) = exp2(q2 * kNegHalfLog2e)
constexpr float kNegHalfLog2e = -0.72134752044448170f;

// The hit test in two parts: the geometry (hit distance, footprint coordinates, and the
// tests that need no Gaussian), then the opacity; a wave in which no lane passes the first
// part can skip the second.  hit_test runs both, bit for bit as the two parts.
__device__ __forceinline__ float hit_geom(Hit &h, const Rec &s, const Ray &ray, const RasterParams &p)
{
    h.e[0] = (ray.dh[0] - s.m0) + ray.dl[0];
    h.e[1] = (ray.dh[1] - s.m1) + ray.dl[1];
    h.e[2] = ray.dh[2] - s.m2;
    // den with the exact ray direction (the residuals of its two rounded products): at
    // grazing incidence t, u and v inherit the relative error of den multiplied by 1 / |den|
    h.den = fmaf(s.nt0, ray.dl[0], fmaf(s.nt1, ray.dl[1], fmaf(s.nt0, ray.dh[0], fmaf(s.nt1, ray.dh[1], s.nt2 * ray.dh[2]))));
    h.nu = fmaf(s.U0, h.e[0], fmaf(s.U1, h.e[1], fmaf(s.U2, h.e[2], s.cu)));
    h.nv = fmaf(s.V0, h.e[0], fmaf(s.V1, h.e[1], fmaf(s.V2, h.e[2], s.cv)));
    h.inv = __builtin_amdgcn_rcpf(h.den);
    h.t = s.c * h.inv;
    float u = h.nu * h.inv, v = h.nv * h.inv;
    float q2 = fmaf(u, u, v * v);
    // |den| >= den_eps, t >= near, q2 <= k^2
    h.pass = (fabsf(h.den) >= p.den_eps) && (h.t >= p.near) && (q2 <= p.k2);
    return q2;
}

// alpha_hat >= alpha_thr completes h.pass
__device__ __forceinline__ void hit_opacity(Hit &h, float q2, const Rec &s, const RasterParams &p)
{
    h.G = __builtin_amdgcn_exp2f(q2 * kNegHalfLog2e);
    h.aG = s.alpha * h.G;
    h.ah = fminf(h.aG, p.alpha_max);
    h.pass = h.pass && (h.ah >= p.alpha_thr);
}

__device__ __forceinline__ Hit hit_test(const Rec &s, const Ray &ray, const RasterParams &p)
{
    Hit h;
    const float q2 = hit_geom(h, s, ray, p);
    hit_opacity(h, q2, s, p);
    return h;
}

// Wave sub-tile vs a surfel's conservative ray rectangle (rows r0..r1, columns c0..c0+cw-1
// modulo W).  Two arcs of a circle meet iff one contains the other's first element.
__device__ __forceinline__ bool sub_overlap(uint2 rc, int sr0, int sc0, int W)
{
    int r0 = (int)(rc.x & 0xFFFFu), r1 = (int)(rc.x >> 16);
    int c0 = (int)(rc.y & 0xFFFFu), cw = (int)(rc.y >> 16);
    if (cw == 0 || r0 >= sr0 + kSub || r1 < sr0) return false;
    int d1 = sc0 - c0;
    if (d1 < 0) d1 += W;
    int d2 = c0 - sc0;
    if (d2 < 0) d2 += W;
    return d1 < cw || d2 < kSub;
}

}  // namespace lgsr
