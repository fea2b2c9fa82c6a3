/*
 * lgsr_ref.c -- plain FP64 CPU oracle of the spherical surfel range-image renderer.
 *
 * TEST INFRASTRUCTURE ONLY (see lgsr_ref.h).  Deliberately simple: every ray is tested
 * against every surfel, in float64, with no tiles, no culling and no reformulation.
 * It shares no code with the GPU path.
 *
 * Paper: "Real-Time LiDAR Gaussian Splatting SLAM via Geometry-Aware Covariance
 * Coupling" (arXiv 2607.04127).  Readings taken where the paper is silent:
 *   R1 primitive: a planar Gaussian with density G = exp(-(u^2 + v^2) / 2), (u, v) the
 *      ray/plane hit in the primitive's tangent axes measured in units of its two scales
 *      (2DGS, cited in Sec. 1), cut off at u^2 + v^2 <= k^2 (k = 3).
 *   R2 intersection: exact ray/plane intersection along each beam direction.
 *   R3 order: surfels composited front to back by ascending sensor-frame centre range,
 *      equal ranges by ascending index.
 *   R4 stabilisers: alpha_hat = min(alpha_max, alpha G); hits with alpha_hat < alpha_thr
 *      skipped; stop after the hit that takes the transmittance below T_min.
 *   R5 outputs (Sec. 3.1, Sec. 3.4 "predicted depth, opacity, and normals"): opacity
 *      A = sum of weights; depth = opacity-normalised expected range; normal = opacity-
 *      normalised sum of surfel normals turned to face the sensor, sensor frame, not
 *      renormalised.  Rendered ray drop = [A < drop_tau].  No hit: all zero, drop = 1.
 *   R6 parameters: s = exp(s~) (Sec. 3.3), alpha = sigmoid(o), q = (w, x, y, z) normalised
 *      inside, rotation columns (a, b, n) with a the major tangent axis (Sec. 3.5 uses
 *      a = R(q) e_0).
 *   R7 pose: T_ws maps sensor to world; the pose gradient is taken in the tangent of the
 *      right perturbation T_ws * Exp(xi), xi = (rho, omega).
 *   R8 beams: a pixel is one ray with direction (cos phi cos th, cos phi sin th, sin phi)
 *      built from the beam tables.
 */
#include "lgsr_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double mu[3], a[3], b[3], n[3]; /* centre and axes in the sensor frame */
    double nt[3];                   /* normal turned to face the sensor */
    double sigma;                   /* +1 or -1: nt = sigma * n */
    double s0, s1, alpha, r;
    double qhat[4], qnorm;
    int valid;
    int near_cut; /* a valid rotation, but the centre is nearer than `near` (R11): not rendered */
} surf_t;

typedef struct {
    int64_t i;
    double t, u, v, G, aG, ahat, T, den, delta[3];
} hit_t;

typedef struct {
    double A, SD, SN[3], T, margin, order_gap, den_min;
    int32_t K, n_hits;
} ray_t;

static double dot3(const double *x, const double *y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; }

static void cross3(const double *x, const double *y, double *o)
{
    o[0] = x[1] * y[2] - x[2] * y[1];
    o[1] = x[2] * y[0] - x[0] * y[2];
    o[2] = x[0] * y[1] - x[1] * y[0];
}

/* Rotation of a unit quaternion (w, x, y, z); columns returned as a, b, n (R6). */
static void quat_axes(const double *q, double *a, double *b, double *n)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    a[0] = 1 - 2 * (y * y + z * z); a[1] = 2 * (x * y + w * z);     a[2] = 2 * (x * z - w * y);
    b[0] = 2 * (x * y - w * z);     b[1] = 1 - 2 * (x * x + z * z); b[2] = 2 * (y * z + w * x);
    n[0] = 2 * (x * z + w * y);     n[1] = 2 * (y * z - w * x);     n[2] = 1 - 2 * (x * x + y * y);
}

/* v_sensor = R_p^T v_world, with pose rows R_p[i][j] = pose[4 i + j]. */
static void world_to_sensor_dir(const double *pose, const double *v, double *o)
{
    for (int j = 0; j < 3; ++j) o[j] = pose[j] * v[0] + pose[4 + j] * v[1] + pose[8 + j] * v[2];
}

static void sensor_to_world_dir(const double *pose, const double *v, double *o)
{
    for (int i = 0; i < 3; ++i) o[i] = pose[4 * i] * v[0] + pose[4 * i + 1] * v[1] + pose[4 * i + 2] * v[2];
}

/* Per-surfel quantities of the map Theta (Sec. 3.1) under the pose. */
static void setup_surfels(const lgsr_ref_map *map, const double *pose, const lgsr_ref_params *p, surf_t *S)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < map->n; ++i) {
        surf_t *s = &S[i];
        const double *q = map->quats + 4 * i;
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        s->qnorm = qn;
        s->valid = 0;
        if (!(qn > 0)) continue;
        for (int c = 0; c < 4; ++c) s->qhat[c] = q[c] / qn;
        double aw[3], bw[3], nw[3], dm[3];
        quat_axes(s->qhat, aw, bw, nw);
        for (int c = 0; c < 3; ++c) dm[c] = map->means[3 * i + c] - pose[4 * c + 3];
        world_to_sensor_dir(pose, dm, s->mu);
        world_to_sensor_dir(pose, aw, s->a);
        world_to_sensor_dir(pose, bw, s->b);
        world_to_sensor_dir(pose, nw, s->n);
        s->s0 = exp(map->log_scales[2 * i]);
        s->s1 = exp(map->log_scales[2 * i + 1]);
        s->alpha = 1.0 / (1.0 + exp(-map->opacity_logits[i]));
        s->r = sqrt(dot3(s->mu, s->mu));
        s->sigma = dot3(s->n, s->mu) <= 0 ? 1.0 : -1.0;
        for (int c = 0; c < 3; ++c) s->nt[c] = s->sigma * s->n[c];
        s->valid = s->r >= p->near;
        s->near_cut = !s->valid;
    }
}

static const surf_t *g_sort_S; /* comparator context (sorting is single threaded) */

static int cmp_range(const void *x, const void *y)
{
    int64_t i = *(const int64_t *)x, j = *(const int64_t *)y;
    double ri = g_sort_S[i].r, rj = g_sort_S[j].r;
    if (ri < rj) return -1;
    if (ri > rj) return 1;
    return (i > j) - (i < j);
}

/* Valid surfels in compositing order (R3); returns their count.  When cut != NULL the
 * surfels dropped only for their centre range (near_cut) are listed there, count in *n_cut. */
static int64_t sort_surfels(const surf_t *S, int64_t n, int64_t *order, int64_t *cut, int64_t *n_cut)
{
    int64_t m = 0, mc = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (S[i].valid) order[m++] = i;
        else if (cut && S[i].near_cut) cut[mc++] = i;
    }
    if (n_cut) *n_cut = mc;
    g_sort_S = S;
    qsort(order, (size_t)m, sizeof(int64_t), cmp_range);
    return m;
}

/* Copies of the surfels ids[0 .. m) in that order, so that a ray's walk in compositing order
 * reads memory front to back (the visit order and the arithmetic are those of the walk over
 * S[ids[k]]; only the layout differs).  NULL on allocation failure when m > 0. */
static surf_t *in_order(const surf_t *S, const int64_t *ids, int64_t m)
{
    surf_t *Q = (surf_t *)malloc(sizeof(surf_t) * (size_t)(m > 0 ? m : 1));
    if (Q)
        for (int64_t k = 0; k < m; ++k) Q[k] = S[ids[k]];
    return Q;
}

/* One surfel's per-hit tests on ray d (R1, R4, R11): the hit quantities, whether each test
 * accepts (|n'.d| >= den_eps, t >= near, q2 <= k^2, alpha_hat >= alpha_thr) and its relative
 * gap to its threshold.  The Gaussian is evaluated where the support test accepts, or where
 * its gap is below gap_below (a caller that needs the opacity test's gap of a surfel the
 * support test rejects only when that gap could matter); otherwise G = 0. */
typedef struct {
    double den, t, delta[3], u, v, q2, G, aG, ahat;
    int ok[4];
    double gap[4];
} eval_t;

static double rel_gap(double x, double thr) { return fabs(x - thr) / fabs(thr); }

static void eval_hit(const surf_t *s, const double *d, const lgsr_ref_params *p, double gap_below, eval_t *e)
{
    double k2 = p->cutoff_sigma * p->cutoff_sigma;
    e->den = dot3(s->n, d);
    e->t = dot3(s->n, s->mu) / e->den;
    for (int c = 0; c < 3; ++c) e->delta[c] = e->t * d[c] - s->mu[c];
    e->u = dot3(s->a, e->delta) / s->s0;
    e->v = dot3(s->b, e->delta) / s->s1;
    e->q2 = e->u * e->u + e->v * e->v;
    e->G = (e->q2 <= k2 || rel_gap(e->q2, k2) < gap_below) ? exp(-0.5 * e->q2) : 0.0;
    e->aG = s->alpha * e->G;
    e->ahat = e->aG < p->alpha_max ? e->aG : p->alpha_max;
    e->ok[0] = fabs(e->den) >= p->den_eps;
    e->ok[1] = e->t >= p->near;
    e->ok[2] = e->q2 <= k2;
    e->ok[3] = e->ahat >= p->alpha_thr;
    e->gap[0] = rel_gap(fabs(e->den), p->den_eps);
    e->gap[1] = rel_gap(e->t, p->near);
    e->gap[2] = rel_gap(e->q2, k2);
    e->gap[3] = rel_gap(e->aG, p->alpha_thr);
}

static int accepted(const eval_t *e) { return e->ok[0] && e->ok[1] && e->ok[2] && e->ok[3]; }

/* How far the tests' decision on a surfel is from flipping: for an accepted surfel any one
 * test crossing its threshold rejects it (the smallest gap); for a rejected one every test
 * that rejects it has to cross (the largest of their gaps, an undefined gap counting as
 * infinite). */
static double flip_gap(const eval_t *e)
{
    int acc = accepted(e);
    double g = acc ? INFINITY : 0.0;
    for (int k = 0; k < 4; ++k) {
        double x = isnan(e->gap[k]) ? INFINITY : e->gap[k];
        if (acc) g = fmin(g, x);
        else if (!e->ok[k]) g = fmax(g, x);
    }
    return g;
}

static void ray_dir(const lgsr_ref_beams *B, int64_t rid, double *d)
{
    int64_t k = rid / B->W, j = rid % B->W;
    double sp = B->row_sincos[2 * k], cp = B->row_sincos[2 * k + 1];
    double st = B->col_sincos[2 * j], ct = B->col_sincos[2 * j + 1];
    d[0] = cp * ct;
    d[1] = cp * st;
    d[2] = sp;
}

/* Front-to-back compositing of one ray over every surfel (R1-R5).  Q[0 .. m) are the valid
 * surfels in compositing order and order[k] the id of Q[k]; C[0 .. n_cut) the surfels cut for
 * their centre range only.  When hits != NULL the composited hits are recorded in order
 * (capacity: the number of valid surfels).
 * margin: the smallest relative distance by which some threshold decision would have to
 * move to change the ray's result: for every surfel the ray reaches before it stops, how far
 * the per-hit tests' decision is from flipping (flip_gap); for a composited surfel also its
 * alpha G against alpha_max, its centre range against `near` and the transmittance after it
 * against T_min; for a surfel cut for its centre range, the largest of that range's gap and
 * the gaps of the hit tests that reject it.  order_gap: the smallest relative gap between
 * the centre ranges of consecutive composited surfels.  A small value flags a ray whose
 * result may legitimately differ when computed in lower precision.  den_min: the smallest
 * |n'.d| over the composited hits (the ray/plane intersection amplifies errors of the plane
 * normal by 1 / |n'.d|). */
static void render_ray(const surf_t *Q, const int64_t *order, int64_t m, const surf_t *C, int64_t n_cut,
                       const double *d, const lgsr_ref_params *p, int want_extra, ray_t *out, hit_t *hits)
{
    double T = 1, A = 0, SD = 0, SN[3] = {0, 0, 0}, margin = INFINITY, order_gap = INFINITY;
    double den_min = INFINITY;
    eval_t e;
    if (want_extra)
        for (int64_t ci = 0; ci < n_cut; ++ci) {
            eval_hit(&C[ci], d, p, INFINITY, &e);
            double need = rel_gap(C[ci].r, p->near);
            if (!accepted(&e)) need = fmax(need, flip_gap(&e));
            margin = fmin(margin, need);
        }
    int32_t K = 0, nh = 0;
    int stopped = 0;
    double prev_r = -1;
    for (int64_t oi = 0; oi < m; ++oi) {
        const surf_t *s = &Q[oi];
        /* a surfel the support test rejects with a gap of at least the margin so far cannot
         * lower the margin, whatever its opacity test's gap: its Gaussian is not needed */
        eval_hit(s, d, p, want_extra && !stopped ? margin : 0.0, &e);
        if (want_extra && !stopped) margin = fmin(margin, flip_gap(&e));
        if (!accepted(&e)) continue;
        nh++;
        if (stopped) {
            if (!want_extra) break;
            continue;
        }
        double t = e.t, ahat = e.ahat;
        if (hits) {
            hit_t *h = &hits[K];
            h->i = order[oi];
            h->t = t; h->u = e.u; h->v = e.v; h->G = e.G; h->aG = e.aG; h->ahat = ahat; h->T = T; h->den = e.den;
            for (int c = 0; c < 3; ++c) h->delta[c] = e.delta[c];
        }
        if (want_extra && prev_r >= 0) order_gap = fmin(order_gap, rel_gap(s->r, prev_r));
        prev_r = s->r;
        if (want_extra) {
            margin = fmin(margin, rel_gap(e.aG, p->alpha_max));
            margin = fmin(margin, rel_gap(s->r, p->near));
            den_min = fmin(den_min, fabs(e.den));
        }
        double w = T * ahat;
        A += w;
        SD += w * t;
        for (int c = 0; c < 3; ++c) SN[c] += w * s->nt[c];
        T *= (1 - ahat);
        K++;
        if (want_extra) margin = fmin(margin, rel_gap(T, p->T_min));
        if (T < p->T_min) {
            stopped = 1;
            if (!want_extra) break;
        }
    }
    out->A = A; out->SD = SD; out->T = T; out->K = K; out->n_hits = nh; out->margin = margin;
    out->order_gap = order_gap;
    out->den_min = den_min;
    for (int c = 0; c < 3; ++c) out->SN[c] = SN[c];
}

static int check_args(const lgsr_ref_map *map, const double *pose, const lgsr_ref_beams *beams,
                      const lgsr_ref_params *prm, int64_t n_rays, const int64_t *ray_ids)
{
    if (!map || !pose || !beams || !prm || map->n < 0 || n_rays < 0) return -1;
    if (map->n > 0 && (!map->means || !map->quats || !map->log_scales || !map->opacity_logits)) return -1;
    if (beams->H <= 0 || beams->W <= 0 || !beams->row_sincos || !beams->col_sincos) return -1;
    int64_t total = (int64_t)beams->H * beams->W;
    if (!ray_ids && n_rays != total) return -1;
    if (ray_ids)
        for (int64_t i = 0; i < n_rays; ++i)
            if (ray_ids[i] < 0 || ray_ids[i] >= total) return -1;
    return 0;
}

int lgsr_ref_forward(const lgsr_ref_map *map, const double pose[12], const lgsr_ref_beams *beams,
                     const lgsr_ref_params *prm, int64_t n_rays, const int64_t *ray_ids,
                     double *depth, double *opacity, double *normal, uint8_t *drop,
                     double *t_final, int32_t *n_contrib, double *margin, double *order_gap,
                     int32_t *n_hits, double *den_min)
{
    if (check_args(map, pose, beams, prm, n_rays, ray_ids)) return -1;
    if (n_rays > 0 && (!depth || !opacity || !normal || !drop)) return -1;
    surf_t *S = (surf_t *)calloc((size_t)(map->n > 0 ? map->n : 1), sizeof(surf_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(map->n > 0 ? map->n : 1));
    int64_t *cut = (int64_t *)malloc(sizeof(int64_t) * (size_t)(map->n > 0 ? map->n : 1));
    if (!S || !order || !cut) { free(S); free(order); free(cut); return -1; }
    setup_surfels(map, pose, prm, S);
    int64_t n_cut = 0;
    int64_t m = sort_surfels(S, map->n, order, cut, &n_cut);
    surf_t *Q = in_order(S, order, m), *C = in_order(S, cut, n_cut);
    if (!Q || !C) { free(S); free(order); free(cut); free(Q); free(C); return -1; }
    int want_extra = (margin != NULL) || (n_hits != NULL) || (order_gap != NULL) || (den_min != NULL);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_rays; ++i) {
        int64_t rid = ray_ids ? ray_ids[i] : i;
        double d[3];
        ray_dir(beams, rid, d);
        ray_t r;
        render_ray(Q, order, m, C, n_cut, d, prm, want_extra, &r, NULL);
        if (r.K == 0) {
            depth[i] = 0; opacity[i] = 0;
            normal[3 * i] = normal[3 * i + 1] = normal[3 * i + 2] = 0;
            drop[i] = 1;
        } else {
            opacity[i] = r.A;
            depth[i] = r.SD / r.A;
            for (int c = 0; c < 3; ++c) normal[3 * i + c] = r.SN[c] / r.A;
            drop[i] = r.A < prm->drop_tau;
        }
        if (t_final) t_final[i] = r.T;
        if (n_contrib) n_contrib[i] = r.K;
        if (margin) margin[i] = r.margin;
        if (order_gap) order_gap[i] = r.order_gap;
        if (n_hits) n_hits[i] = r.n_hits;
        if (den_min) den_min[i] = r.den_min;
    }
    free(S);
    free(order);
    free(cut);
    free(Q);
    free(C);
    return 0;
}

/* Sec. 3.4: masked depth L1 (Eq. 10, left) and G-ICP normal cosine term (Eq. 11, first term),
 * L = w_depth * L_depth + lambda_n * lambda_ng * mean_{Omega_N}(1 - Nhat^T N / |Nhat|).
 * Empty masks give a zero term; sign(0) = 0; a zero rendered normal costs 1 with no gradient. */
int lgsr_ref_loss(int64_t n_rays, const double *depth, const double *opacity, const double *normal,
                  const double *target_depth, const double *target_normal, const double *ray_weight,
                  double w_depth, double lambda_n, double lambda_ng, double loss[5],
                  double *g_depth, double *g_opacity, double *g_normal)
{
    if (n_rays < 0 || !loss) return -1;
    if (n_rays > 0 && (!depth || !opacity || !normal || !target_depth || !target_normal)) return -1;
    (void)opacity;
    double cntD = 0, cntN = 0, sumD = 0, sumN = 0;
    for (int64_t i = 0; i < n_rays; ++i) {
        double wgt = ray_weight ? ray_weight[i] : 1.0;
        double mD = (target_depth[i] > 0) ? wgt : 0.0;
        const double *N = target_normal + 3 * i, *Nh = normal + 3 * i;
        double mN = (dot3(N, N) > 0) ? mD : 0.0;
        cntD += mD;
        cntN += mN;
        sumD += mD * fabs(depth[i] - target_depth[i]);
        double nn = sqrt(dot3(Nh, Nh));
        sumN += mN * (nn > 0 ? 1.0 - dot3(Nh, N) / nn : 1.0);
    }
    double termD = cntD > 0 ? w_depth * sumD / cntD : 0.0;
    double termN = cntN > 0 ? lambda_n * lambda_ng * sumN / cntN : 0.0;
    loss[0] = termD + termN;
    loss[1] = termD;
    loss[2] = termN;
    loss[3] = cntD;
    loss[4] = cntN;
    for (int64_t i = 0; i < n_rays; ++i) {
        double wgt = ray_weight ? ray_weight[i] : 1.0;
        double mD = (target_depth[i] > 0) ? wgt : 0.0;
        const double *N = target_normal + 3 * i, *Nh = normal + 3 * i;
        double mN = (dot3(N, N) > 0) ? mD : 0.0;
        double diff = depth[i] - target_depth[i];
        double sgn = diff > 0 ? 1.0 : (diff < 0 ? -1.0 : 0.0);
        if (g_depth) g_depth[i] = cntD > 0 ? w_depth * mD * sgn / cntD : 0.0;
        if (g_opacity) g_opacity[i] = 0.0;
        if (g_normal) {
            double nn = sqrt(dot3(Nh, Nh));
            for (int c = 0; c < 3; ++c) g_normal[3 * i + c] = 0.0;
            if (nn > 0 && cntN > 0 && mN != 0) {
                double cosv = dot3(Nh, N) / nn;
                double f = -lambda_n * lambda_ng * mN / (cntN * nn);
                for (int c = 0; c < 3; ++c) g_normal[3 * i + c] = f * (N[c] - cosv * Nh[c] / nn);
            }
        }
    }
    return 0;
}

/* Per-surfel gradient accumulators in the sensor frame. */
typedef struct {
    double mu[3], a[3], b[3], n[3], s0, s1, alpha;
} sgrad_t;

static void atomic_add(double *x, double v)
{
#pragma omp atomic
    *x += v;
}

/* Chain rule from sensor-frame gradients g of one surfel to its raw parameters and to the
 * pose tangent (rho, omega) of the right perturbation (R6, R7):
 *   mu' = R_p^T (mu - t_p), a' = R_p^T a, ...: world gradient = R_p times sensor gradient;
 *   (a, b, n) = columns of R(qhat); q -> qhat = q / |q|; s = exp(s~); alpha = sigmoid(o);
 *   mu' -> mu' - rho + mu' x omega, a' -> a' + a' x omega, ... to first order. */
static void chain_params(const surf_t *s, const double *pose, const sgrad_t *g, double *dm, double *dq,
                         double *dl, double *dlog, double *dpose)
{
    double Ga[3], Gb[3], Gn[3];
    sensor_to_world_dir(pose, g->mu, dm);
    sensor_to_world_dir(pose, g->a, Ga);
    sensor_to_world_dir(pose, g->b, Gb);
    sensor_to_world_dir(pose, g->n, Gn);
    double w = s->qhat[0], x = s->qhat[1], y = s->qhat[2], z = s->qhat[3];
    double dw = Ga[1] * 2 * z - Ga[2] * 2 * y - Gb[0] * 2 * z + Gb[2] * 2 * x + Gn[0] * 2 * y - Gn[1] * 2 * x;
    double dx = Ga[1] * 2 * y + Ga[2] * 2 * z + Gb[0] * 2 * y - Gb[1] * 4 * x + Gb[2] * 2 * w
              + Gn[0] * 2 * z - Gn[1] * 2 * w - Gn[2] * 4 * x;
    double dy = -Ga[0] * 4 * y + Ga[1] * 2 * x - Ga[2] * 2 * w + Gb[0] * 2 * x + Gb[2] * 2 * z
              + Gn[0] * 2 * w + Gn[1] * 2 * z - Gn[2] * 4 * y;
    double dz = -Ga[0] * 4 * z + Ga[1] * 2 * w + Ga[2] * 2 * x - Gb[0] * 2 * w - Gb[1] * 4 * z
              + Gb[2] * 2 * y + Gn[0] * 2 * x + Gn[1] * 2 * y;
    double dqh[4] = {dw, dx, dy, dz};
    double radial = dqh[0] * s->qhat[0] + dqh[1] * s->qhat[1] + dqh[2] * s->qhat[2] + dqh[3] * s->qhat[3];
    for (int c = 0; c < 4; ++c) dq[c] = (dqh[c] - radial * s->qhat[c]) / s->qnorm;
    dl[0] = s->s0 * g->s0;
    dl[1] = s->s1 * g->s1;
    *dlog = s->alpha * (1 - s->alpha) * g->alpha;
    double c1[3], c2[3], c3[3], c4[3];
    cross3(s->mu, g->mu, c1);
    cross3(s->a, g->a, c2);
    cross3(s->b, g->b, c3);
    cross3(s->n, g->n, c4);
    for (int c = 0; c < 3; ++c) {
        dpose[c] = -g->mu[c];
        dpose[3 + c] = -(c1[c] + c2[c] + c3[c] + c4[c]);
    }
}

/* chain_params on magnitudes: every coefficient and input taken by absolute value, so the
 * result bounds the size of the terms that the signed chain adds up (running error bound). */
static void chain_params_abs(const surf_t *s, const double *pose, const sgrad_t *g, double *dm, double *dq,
                             double *dl, double *dlog, double *dpose)
{
    double P[12];
    for (int c = 0; c < 12; ++c) P[c] = fabs(pose[c]);
    double Ga[3], Gb[3], Gn[3];
    sensor_to_world_dir(P, g->mu, dm);
    sensor_to_world_dir(P, g->a, Ga);
    sensor_to_world_dir(P, g->b, Gb);
    sensor_to_world_dir(P, g->n, Gn);
    double w = fabs(s->qhat[0]), x = fabs(s->qhat[1]), y = fabs(s->qhat[2]), z = fabs(s->qhat[3]);
    double dw = 2 * (Ga[1] * z + Ga[2] * y + Gb[0] * z + Gb[2] * x + Gn[0] * y + Gn[1] * x);
    double dx = 2 * (Ga[1] * y + Ga[2] * z + Gb[0] * y + Gb[2] * w + Gn[0] * z + Gn[1] * w) + 4 * x * (Gb[1] + Gn[2]);
    double dy = 2 * (Ga[1] * x + Ga[2] * w + Gb[0] * x + Gb[2] * z + Gn[0] * w + Gn[1] * z) + 4 * y * (Ga[0] + Gn[2]);
    double dz = 2 * (Ga[1] * w + Ga[2] * x + Gb[0] * w + Gb[2] * y + Gn[0] * x + Gn[1] * y) + 4 * z * (Ga[0] + Gb[1]);
    double dqh[4] = {dw, dx, dy, dz}, qa[4] = {w, x, y, z};
    double radial = dqh[0] * w + dqh[1] * x + dqh[2] * y + dqh[3] * z;
    for (int c = 0; c < 4; ++c) dq[c] = (dqh[c] + radial * qa[c]) / s->qnorm;
    dl[0] = s->s0 * g->s0;
    dl[1] = s->s1 * g->s1;
    *dlog = s->alpha * (1 - s->alpha) * g->alpha;
    const double *vec[4] = {s->mu, s->a, s->b, s->n};
    const double *gv[4] = {g->mu, g->a, g->b, g->n};
    for (int c = 0; c < 3; ++c) {
        dpose[c] = g->mu[c];
        double acc = 0;
        int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        for (int k = 0; k < 4; ++k) acc += fabs(vec[k][c1]) * gv[k][c2] + fabs(vec[k][c2]) * gv[k][c1];
        dpose[3 + c] = acc;
    }
}

static double norm_n(const double *v, int n)
{
    double q = 0;
    for (int c = 0; c < n; ++c) q += v[c] * v[c];
    return sqrt(q);
}

int lgsr_ref_backward(const lgsr_ref_map *map, const double pose[12], const lgsr_ref_beams *beams,
                      const lgsr_ref_params *prm, int64_t n_rays, const int64_t *ray_ids,
                      const double *g_depth, const double *g_opacity, const double *g_normal,
                      double *d_means, double *d_quats, double *d_log_scales,
                      double *d_opacity_logits, double d_pose[6], double *mass, double *pose_mass)
{
    if (check_args(map, pose, beams, prm, n_rays, ray_ids)) return -1;
    if (n_rays > 0 && (!g_depth || !g_opacity || !g_normal)) return -1;
    if (map->n > 0 && (!d_means || !d_quats || !d_log_scales || !d_opacity_logits)) return -1;
    if (!d_pose) return -1;
    int64_t n = map->n;
    size_t nn = (size_t)(n > 0 ? n : 1);
    surf_t *S = (surf_t *)calloc(nn, sizeof(surf_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * nn);
    sgrad_t *Gs = (sgrad_t *)calloc(nn, sizeof(sgrad_t));
    if (!S || !order || !Gs) { free(S); free(order); free(Gs); return -1; }
    if (mass)
        for (int64_t i = 0; i < 4 * n; ++i) mass[i] = 0;
    if (pose_mass)
        for (int c = 0; c < 6; ++c) pose_mass[c] = 0;
    setup_surfels(map, pose, prm, S);
    int64_t m = sort_surfels(S, n, order, NULL, NULL);
    surf_t *Q = in_order(S, order, m);
    if (!Q) { free(S); free(order); free(Gs); return -1; }

#pragma omp parallel
    {
        hit_t *hits = (hit_t *)malloc(sizeof(hit_t) * (size_t)(m > 0 ? m : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n_rays; ++i) {
            int64_t rid = ray_ids ? ray_ids[i] : i;
            double d[3];
            ray_dir(beams, rid, d);
            ray_t r;
            render_ray(Q, order, m, NULL, 0, d, prm, 0, &r, hits);
            if (r.K == 0) continue;
            /* dL = gD dDhat + gA dA + gN.dNhat with Dhat = SD/A, Nhat = SN/A:
             * dL = (gD/A) dSD + (gN/A).dSN + (gA - (gD Dhat + gN.Nhat)/A) dA. */
            double A = r.A, Dh = r.SD / A, Nh[3];
            for (int c = 0; c < 3; ++c) Nh[c] = r.SN[c] / A;
            const double *gN = g_normal + 3 * i;
            double gbD = g_depth[i] / A, gbN[3];
            for (int c = 0; c < 3; ++c) gbN[c] = gN[c] / A;
            double gbA = g_opacity[i] - (g_depth[i] * Dh + dot3(gN, Nh)) / A;
            double B = 0; /* sum over later hits of w_i c_i */
            /* magnitudes of the same quantities before any cancellation (test tolerances) */
            double abD = fabs(g_depth[i]) / A, abN[3], abA, Babs = 0;
            for (int c = 0; c < 3; ++c) abN[c] = fabs(gN[c]) / A;
            abA = fabs(g_opacity[i]) + (fabs(g_depth[i]) * fabs(Dh) + fabs(gN[0] * Nh[0]) + fabs(gN[1] * Nh[1])
                                         + fabs(gN[2] * Nh[2])) / A;
            for (int j = r.K - 1; j >= 0; --j) {
                const hit_t *h = &hits[j];
                const surf_t *s = &S[h->i];
                double cj = gbD * h->t + dot3(gbN, s->nt) + gbA;
                double w = h->T * h->ahat;
                /* w_j = T_j ahat_j and every later weight carries the factor (1 - ahat_j) */
                double d_ahat = h->T * cj - B / (1 - h->ahat);
                B += w * cj;
                double d_t = gbD * w, d_nt[3];
                for (int c = 0; c < 3; ++c) d_nt[c] = gbN[c] * w;
                double d_alpha = 0, d_G = 0;
                if (h->aG < prm->alpha_max) { d_alpha = d_ahat * h->G; d_G = d_ahat * s->alpha; }
                double d_q2 = -0.5 * h->G * d_G;
                double d_u = 2 * h->u * d_q2, d_v = 2 * h->v * d_q2;
                /* u = a'.Delta / s0, v = b'.Delta / s1, Delta = t d - mu', t = n'.mu' / n'.d */
                double gDelta[3], g_mu[3], g_a[3], g_b[3], g_n[3];
                for (int c = 0; c < 3; ++c) {
                    gDelta[c] = d_u * s->a[c] / s->s0 + d_v * s->b[c] / s->s1;
                    g_a[c] = d_u * h->delta[c] / s->s0;
                    g_b[c] = d_v * h->delta[c] / s->s1;
                }
                double g_t = d_t + dot3(gDelta, d);
                for (int c = 0; c < 3; ++c) {
                    g_mu[c] = -gDelta[c] + g_t * s->n[c] / h->den;
                    g_n[c] = -g_t * h->delta[c] / h->den + s->sigma * d_nt[c];
                }
                sgrad_t *g = &Gs[h->i];
                for (int c = 0; c < 3; ++c) {
                    atomic_add(&g->mu[c], g_mu[c]);
                    atomic_add(&g->a[c], g_a[c]);
                    atomic_add(&g->b[c], g_b[c]);
                    atomic_add(&g->n[c], g_n[c]);
                }
                atomic_add(&g->s0, -d_u * h->u / s->s0);
                atomic_add(&g->s1, -d_v * h->v / s->s1);
                atomic_add(&g->alpha, d_alpha);
                if (mass || pose_mass) {
                    /* the same contribution evaluated on magnitudes: a running error bound of
                     * the terms a finite-precision evaluation adds up (test tolerances) */
                    double ca = abD * fabs(h->t) + fabs(abN[0] * s->nt[0]) + fabs(abN[1] * s->nt[1])
                              + fabs(abN[2] * s->nt[2]) + abA;
                    double ahA = h->T * ca + Babs / (1 - h->ahat);
                    Babs += w * ca;
                    double aA = 0, aG = 0;
                    if (h->aG < prm->alpha_max) { aA = ahA * h->G; aG = ahA * s->alpha; }
                    double aq2 = 0.5 * h->G * aG, au = 2 * fabs(h->u) * aq2, av = 2 * fabs(h->v) * aq2;
                    double aT = abD * w, aDel[3], aTt, ad = fabs(h->den);
                    sgrad_t one;
                    for (int c = 0; c < 3; ++c) {
                        aDel[c] = au * fabs(s->a[c]) / s->s0 + av * fabs(s->b[c]) / s->s1;
                        one.a[c] = au * fabs(h->delta[c]) / s->s0;
                        one.b[c] = av * fabs(h->delta[c]) / s->s1;
                    }
                    aTt = aT + aDel[0] * fabs(d[0]) + aDel[1] * fabs(d[1]) + aDel[2] * fabs(d[2]);
                    for (int c = 0; c < 3; ++c) {
                        one.mu[c] = aDel[c] + aTt * fabs(s->n[c]) / ad;
                        one.n[c] = aTt * fabs(h->delta[c]) / ad + abN[c] * w;
                    }
                    one.s0 = au * fabs(h->u) / s->s0;
                    one.s1 = av * fabs(h->v) / s->s1;
                    one.alpha = aA;
                    double dm[3], dq[4], dl[2], dlog, dp[6];
                    chain_params_abs(s, pose, &one, dm, dq, dl, &dlog, dp);
                    if (mass) {
                        atomic_add(&mass[4 * h->i + 0], norm_n(dm, 3));
                        atomic_add(&mass[4 * h->i + 1], norm_n(dq, 4));
                        atomic_add(&mass[4 * h->i + 2], norm_n(dl, 2));
                        atomic_add(&mass[4 * h->i + 3], fabs(dlog));
                    }
                    if (pose_mass)
                        for (int c = 0; c < 6; ++c) atomic_add(&pose_mass[c], fabs(dp[c]));
                }
            }
        }
        free(hits);
    }

    /* Chain rule to the raw parameters and the pose. */
    double pr[3] = {0, 0, 0}, pw[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        const surf_t *s = &S[i];
        double *dm = d_means + 3 * i, *dq = d_quats + 4 * i, *dl = d_log_scales + 2 * i;
        if (!s->valid) {
            dm[0] = dm[1] = dm[2] = 0;
            dq[0] = dq[1] = dq[2] = dq[3] = 0;
            dl[0] = dl[1] = 0;
            d_opacity_logits[i] = 0;
            continue;
        }
        double dp[6];
        chain_params(s, pose, &Gs[i], dm, dq, dl, &d_opacity_logits[i], dp);
        for (int c = 0; c < 3; ++c) {
            pr[c] += dp[c];
            pw[c] += dp[3 + c];
        }
    }
    for (int c = 0; c < 3; ++c) { d_pose[c] = pr[c]; d_pose[3 + c] = pw[c]; }
    free(S);
    free(Q);
    free(order);
    free(Gs);
    return 0;
}

/* ---- full mapping objective (Sec. 3.4, Eq. 10-13) -------------------------------------- */

/* The four neighbours of pixel (k, j) used by N_surf: right/left columns (azimuth wraps over
 * the full turn) and the rows above/below (index k + 1 / k - 1, no wrap). */
typedef struct {
    int64_t r, l, u, d;
} nbr_t;

/* R12 (Sec. 3.4, normal loss, N_surf): the normal of the rendered surface at pixel (k, j),
 * from the points P = D^ d of the rendered range image at the four neighbours:
 * v = (P_r - P_l) x (P_u - P_d), N_surf = v / |v| turned to face the sensor (v.d_p > 0 flips
 * it).  Defined for 1 <= k <= H - 2 when the four neighbours rendered a range (D^ > 0) and
 * v != 0.  Returns 1 when defined; a, b, v receive the two differences and their cross
 * product, *sgn the turn (+1 or -1), *flip_margin |v.d_p| / |v| (how close the turn is to a
 * tie). */
static int surf_normal(const lgsr_ref_beams *B, const double *depth, int64_t k, int64_t j, nbr_t *nb,
                       double a[3], double b[3], double v[3], double *sgn, double *flip_margin)
{
    const int64_t H = B->H, W = B->W;
    if (k < 1 || k > H - 2) return 0;
    nb->r = k * W + (j + 1) % W;
    nb->l = k * W + (j + W - 1) % W;
    nb->u = (k + 1) * W + j;
    nb->d = (k - 1) * W + j;
    if (!(depth[nb->r] > 0) || !(depth[nb->l] > 0) || !(depth[nb->u] > 0) || !(depth[nb->d] > 0)) return 0;
    double dr[3], dl[3], du[3], dd[3], dp[3];
    ray_dir(B, nb->r, dr);
    ray_dir(B, nb->l, dl);
    ray_dir(B, nb->u, du);
    ray_dir(B, nb->d, dd);
    ray_dir(B, k * W + j, dp);
    for (int c = 0; c < 3; ++c) {
        a[c] = depth[nb->r] * dr[c] - depth[nb->l] * dl[c];
        b[c] = depth[nb->u] * du[c] - depth[nb->d] * dd[c];
    }
    cross3(a, b, v);
    double vn = sqrt(dot3(v, v));
    if (!(vn > 0)) return 0;
    double vd = dot3(v, dp);
    *sgn = vd > 0 ? -1.0 : 1.0;
    *flip_margin = fabs(vd) / vn;
    return 1;
}

int lgsr_ref_surf_normal(const lgsr_ref_beams *B, const double *depth, double *n_surf, uint8_t *defined,
                         double *flip_margin)
{
    if (!B || !depth || !n_surf || B->H < 0 || B->W < 0) return -1;
    const int64_t H = B->H, W = B->W;
    for (int64_t k = 0; k < H; ++k)
        for (int64_t j = 0; j < W; ++j) {
            int64_t i = k * W + j;
            nbr_t nb;
            double a[3], b[3], v[3], sgn = 1, fm = INFINITY;
            int ok = surf_normal(B, depth, k, j, &nb, a, b, v, &sgn, &fm);
            double vn = ok ? sqrt(dot3(v, v)) : 1.0;
            for (int c = 0; c < 3; ++c) n_surf[3 * i + c] = ok ? sgn * v[c] / vn : 0.0;
            if (defined) defined[i] = (uint8_t)ok;
            if (flip_margin) flip_margin[i] = ok ? fm : INFINITY;
        }
    return 0;
}

/* Eq. 10 (depth L1 and positive-only opacity BCE), Eq. 11 (both normal terms) and their
 * weights in Eq. 13:
 *   L = w_depth / |Omega_D| sum_{Omega_D} |D^ - D|
 *     - lambda_alpha / |Omega_D| sum_{Omega_D} log(A^ + eps)
 *     + lambda_n lambda_ng / |Omega_N| sum_{Omega_N} (1 - N^ . N_gicp / |N^|)
 *     + lambda_n lambda_ns / |Omega_D| sum_{Omega_D, N_surf defined} (1 - N^ . N_surf / |N^|).
 * The gradient is the full derivative: through N^ and, inside N_surf, through the rendered
 * depth of the four neighbours. */
int lgsr_ref_objective(const lgsr_ref_beams *B, const double *depth, const double *opacity, const double *normal,
                       const double *target_depth, const double *target_normal, double w_depth,
                       double lambda_alpha, double eps, double lambda_n, double lambda_ng, double lambda_ns,
                       double loss[8], double *g_depth, double *g_opacity, double *g_normal)
{
    if (!B || !loss || B->H < 0 || B->W < 0) return -1;
    const int64_t n = (int64_t)B->H * B->W;
    if (n > 0 && (!depth || !opacity || !normal || !target_depth || !target_normal)) return -1;
    double cntD = 0, cntN = 0, cntS = 0, sumD = 0, sumA = 0, sumNg = 0, sumNs = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!(target_depth[i] > 0)) continue;
        const double *Nt = target_normal + 3 * i, *Nh = normal + 3 * i;
        double nh = sqrt(dot3(Nh, Nh));
        cntD += 1;
        sumD += fabs(depth[i] - target_depth[i]);
        sumA += log(opacity[i] + eps);
        if (dot3(Nt, Nt) > 0) {
            cntN += 1;
            sumNg += nh > 0 ? 1.0 - dot3(Nh, Nt) / nh : 1.0;
        }
        nbr_t nb;
        double a[3], b[3], v[3], sgn, fm;
        if (surf_normal(B, depth, i / B->W, i % B->W, &nb, a, b, v, &sgn, &fm)) {
            double vn = sqrt(dot3(v, v));
            double Ns[3] = {sgn * v[0] / vn, sgn * v[1] / vn, sgn * v[2] / vn};
            cntS += 1;
            sumNs += nh > 0 ? 1.0 - dot3(Nh, Ns) / nh : 1.0;
        }
    }
    double tD = cntD > 0 ? w_depth * sumD / cntD : 0.0;
    double tA = cntD > 0 ? -lambda_alpha * sumA / cntD : 0.0;
    double tNg = cntN > 0 ? lambda_n * lambda_ng * sumNg / cntN : 0.0;
    double tNs = cntD > 0 ? lambda_n * lambda_ns * sumNs / cntD : 0.0;
    loss[0] = tD + tA + tNg + tNs;
    loss[1] = tD;
    loss[2] = tA;
    loss[3] = tNg;
    loss[4] = tNs;
    loss[5] = cntD;
    loss[6] = cntN;
    loss[7] = cntS;
    if (!g_depth && !g_opacity && !g_normal) return 0;
    if (!g_depth || !g_opacity || !g_normal) return -1;
    for (int64_t i = 0; i < n; ++i) {
        g_depth[i] = 0;
        g_opacity[i] = 0;
        g_normal[3 * i] = g_normal[3 * i + 1] = g_normal[3 * i + 2] = 0;
    }
    if (!(cntD > 0)) return 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!(target_depth[i] > 0)) continue;
        const double *Nt = target_normal + 3 * i, *Nh = normal + 3 * i;
        double nh = sqrt(dot3(Nh, Nh));
        double diff = depth[i] - target_depth[i];
        g_depth[i] += w_depth * (diff > 0 ? 1.0 : (diff < 0 ? -1.0 : 0.0)) / cntD;
        g_opacity[i] = -lambda_alpha / (cntD * (opacity[i] + eps));
        if (dot3(Nt, Nt) > 0 && nh > 0) {
            double cosv = dot3(Nh, Nt) / nh;
            double f = -lambda_n * lambda_ng / (cntN * nh);
            for (int c = 0; c < 3; ++c) g_normal[3 * i + c] += f * (Nt[c] - cosv * Nh[c] / nh);
        }
        nbr_t nb;
        double a[3], b[3], v[3], sgn, fm;
        if (nh > 0 && surf_normal(B, depth, i / B->W, i % B->W, &nb, a, b, v, &sgn, &fm)) {
            double vn = sqrt(dot3(v, v));
            double u[3] = {v[0] / vn, v[1] / vn, v[2] / vn};
            double Ns[3] = {sgn * u[0], sgn * u[1], sgn * u[2]};
            double cosv = dot3(Nh, Ns) / nh;
            double c0 = lambda_n * lambda_ns / cntD;
            for (int c = 0; c < 3; ++c) g_normal[3 * i + c] += -c0 * (Ns[c] - cosv * Nh[c] / nh) / nh;
            /* dl/dN_surf = -c0 N^/|N^|; through N_surf = sgn v/|v| to v, then to a and b */
            double gN[3] = {-c0 * Nh[0] / nh, -c0 * Nh[1] / nh, -c0 * Nh[2] / nh};
            double gu = dot3(gN, u);
            double gv[3], ga[3], gb[3];
            for (int c = 0; c < 3; ++c) gv[c] = sgn * (gN[c] - gu * u[c]) / vn;
            cross3(b, gv, ga); /* d(a x b) . gv = da . (b x gv) */
            cross3(gv, a, gb); /* (a x db) . gv = db . (gv x a) */
            double dr[3], dl[3], du[3], dd[3];
            ray_dir(B, nb.r, dr);
            ray_dir(B, nb.l, dl);
            ray_dir(B, nb.u, du);
            ray_dir(B, nb.d, dd);
            g_depth[nb.r] += dot3(dr, ga);
            g_depth[nb.l] -= dot3(dl, ga);
            g_depth[nb.u] += dot3(du, gb);
            g_depth[nb.d] -= dot3(dd, gb);
        }
    }
    return 0;
}

/* Eq. 12 with its weight from Eq. 13: lambda_s sum_i max(0, max(s_x, s_y) - s_max), s =
 * exp(log_scales).  The gradient goes to the larger scale (the first on a tie): lambda_s s_k
 * when it exceeds s_max.  margin (NULL to skip): |max(s) - s_max| / s_max per surfel. */
int lgsr_ref_scale_reg(int64_t n, const double *log_scales, double lambda_s, double s_max, double *loss,
                       double *g_log_scales, double *margin)
{
    if (n < 0 || !loss || (n > 0 && !log_scales) || !(s_max > 0)) return -1;
    double sum = 0;
    for (int64_t i = 0; i < n; ++i) {
        double sx = exp(log_scales[2 * i]), sy = exp(log_scales[2 * i + 1]);
        int k = sy > sx ? 1 : 0;
        double smax = k ? sy : sx;
        if (smax > s_max) sum += smax - s_max;
        if (g_log_scales) {
            g_log_scales[2 * i] = g_log_scales[2 * i + 1] = 0;
            if (smax > s_max) g_log_scales[2 * i + k] = lambda_s * smax;
        }
        if (margin) margin[i] = fabs(smax - s_max) / s_max;
    }
    *loss = lambda_s * sum;
    return 0;
}

/* ---- scan to range image (Sec. 3.1) and target covariance (Sec. 3.2) ------------------ */

/* R15: the spherical projection pi_s of a scan onto the H x W grid of a spinning LiDAR:
 * rows uniform in elevation from el_max (row 0) down to el_min (row H - 1), columns uniform
 * over the full turn (column j at azimuth 2 pi j / W).  A point goes to the nearest row and
 * column (f = (el_max - el) / step, k = floor(f + 1/2); g = az W / (2 pi), j = floor(g +
 * 1/2) mod W), is kept when 0 <= k < H and r_min <= r <= r_max, and the nearest return wins
 * each pixel (equal ranges: the lower point index).  The pixel takes that point's range and
 * its normal turned to face the sensor (n.p > 0 flips it).  bin_margin (per point, NULL to
 * skip) is the distance of f and g to their rounding boundaries in bins and of r to the
 * range gates relative to r: how close the point is to landing elsewhere. */
int lgsr_ref_scan_to_range(int64_t n, const double *points, const double *normals, int32_t H, int32_t W,
                           double el_min, double el_max, double r_min, double r_max, double *depth,
                           double *normal, int64_t *index, double *bin_margin)
{
    if (n < 0 || H < 2 || W < 1 || !(el_max > el_min) || !depth || !index || (n > 0 && !points)) return -1;
    const int64_t P = (int64_t)H * W;
    for (int64_t i = 0; i < P; ++i) {
        depth[i] = 0;
        index[i] = -1;
        if (normal) normal[3 * i] = normal[3 * i + 1] = normal[3 * i + 2] = 0;
    }
    const double step = (el_max - el_min) / (H - 1);
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t i = 0; i < n; ++i) {
        const double *p = points + 3 * i;
        double rxy = sqrt(p[0] * p[0] + p[1] * p[1]);
        double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        double el = atan2(p[2], rxy);
        double az = atan2(p[1], p[0]);
        double f = (el_max - el) / step;
        double g = az * W / two_pi;
        double kf = floor(f + 0.5), jf = floor(g + 0.5);
        if (bin_margin) {
            double m = fmin(fabs(f + 0.5 - kf), fabs(kf + 0.5 - f));
            m = fmin(m, fmin(fabs(g + 0.5 - jf), fabs(jf + 0.5 - g)));
            if (r > 0) m = fmin(m, fmin(fabs(r - r_min), fabs(r - r_max)) / r);
            bin_margin[i] = m;
        }
        if (!(r >= r_min && r <= r_max) || kf < 0 || kf > H - 1) continue;
        int64_t j = (int64_t)jf % W;
        if (j < 0) j += W;
        int64_t pix = (int64_t)kf * W + j;
        if (index[pix] < 0 || r < depth[pix]) {
            depth[pix] = r;
            index[pix] = i;
        }
    }
    if (normal && normals)
        for (int64_t q = 0; q < P; ++q) {
            if (index[q] < 0) continue;
            const double *nv = normals + 3 * index[q], *p = points + 3 * index[q];
            double sgn = dot3(nv, p) > 0 ? -1.0 : 1.0;
            for (int c = 0; c < 3; ++c) normal[3 * q + c] = sgn * nv[c];
        }
    return 0;
}

/* Sec. 3.2, target covariance: Sigma = R diag(s_x^2, s_y^2, eps^2) R^T with R = [a b n]
 * the rotation of the normalised quaternion (w, x, y, z) and s = exp(log_scales); a zero
 * quaternion (no orientation) gives a zero covariance.  cov: n x 6 = (xx, xy, xz, yy, yz, zz). */
int lgsr_ref_target_cov(int64_t n, const double *quats, const double *log_scales, double eps, double *cov)
{
    if (n < 0 || !(eps >= 0) || (n > 0 && (!quats || !log_scales || !cov))) return -1;
    for (int64_t i = 0; i < n; ++i) {
        const double *q = quats + 4 * i;
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        if (!(qn > 0)) { /* no orientation: no target */
            for (int c = 0; c < 6; ++c) cov[6 * i + c] = 0;
            continue;
        }
        double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
        double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                          {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                          {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
        double d[3] = {exp(2 * log_scales[2 * i]), exp(2 * log_scales[2 * i + 1]), eps * eps};
        double S[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) S[r][c] = R[r][0] * d[0] * R[c][0] + R[r][1] * d[1] * R[c][1] + R[r][2] * d[2] * R[c][2];
        double *o = cov + 6 * i;
        o[0] = S[0][0];
        o[1] = S[0][1];
        o[2] = S[0][2];
        o[3] = S[1][1];
        o[4] = S[1][2];
        o[5] = S[2][2];
    }
    return 0;
}

/* The valid surfels in compositing order (R3) with their sensor-frame centre ranges. */
int lgsr_ref_order(const lgsr_ref_map *map, const double pose[12], const lgsr_ref_params *prm, int64_t *order,
                   double *range, int64_t *m_out)
{
    if (!map || !pose || !prm || !m_out || map->n < 0) return -1;
    if (map->n > 0 && (!order || !range || !map->means || !map->quats || !map->log_scales || !map->opacity_logits))
        return -1;
    surf_t *S = (surf_t *)calloc((size_t)(map->n > 0 ? map->n : 1), sizeof(surf_t));
    if (!S) return -1;
    setup_surfels(map, pose, prm, S);
    int64_t m = sort_surfels(S, map->n, order, NULL, NULL);
    for (int64_t k = 0; k < m; ++k) range[k] = S[order[k]].r;
    *m_out = m;
    free(S);
    return 0;
}

/* The composited surfels of each of n_rays rays, front to back: ray i's ids in
 * ids[i * cap .. i * cap + min(count[i], cap)), count[i] its hit count K. */
int lgsr_ref_contributors(const lgsr_ref_map *map, const double pose[12], const lgsr_ref_beams *beams,
                          const lgsr_ref_params *prm, int64_t n_rays, const int64_t *ray_ids, int64_t *ids,
                          int64_t cap, int32_t *count)
{
    if (check_args(map, pose, beams, prm, n_rays, ray_ids) || cap < 0 || (n_rays > 0 && (!count || (cap && !ids))))
        return -1;
    surf_t *S = (surf_t *)calloc((size_t)(map->n > 0 ? map->n : 1), sizeof(surf_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(map->n > 0 ? map->n : 1));
    if (!S || !order) { free(S); free(order); return -1; }
    setup_surfels(map, pose, prm, S);
    int64_t m = sort_surfels(S, map->n, order, NULL, NULL);
    surf_t *Q = in_order(S, order, m);
    if (!Q) { free(S); free(order); return -1; }
    int fail = 0;
#pragma omp parallel
    {
        hit_t *hits = (hit_t *)malloc(sizeof(hit_t) * (size_t)(m > 0 ? m : 1));
        if (!hits) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < n_rays; ++i) {
            if (!hits) continue;
            double d[3];
            ray_dir(beams, ray_ids ? ray_ids[i] : i, d);
            ray_t r;
            render_ray(Q, order, m, NULL, 0, d, prm, 0, &r, hits);
            count[i] = r.K;
            for (int64_t k = 0; k < r.K && k < cap; ++k) ids[i * cap + k] = hits[k].i;
        }
        free(hits);
    }
    free(S);
    free(order);
    free(Q);
    return fail ? -1 : 0;
}

void lgsr_ref_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int lgsr_ref_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
