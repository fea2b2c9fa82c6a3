/*
 * lgsr_ref.h -- plain FP64 CPU oracle of the spherical surfel range-image renderer.
 *
 * TEST INFRASTRUCTURE ONLY.  This library defines what the GPU renderer must compute and
 * is used by the test-suite, the smoke check and the benchmark's CPU-baseline leg.  The
 * product path never links, loads or calls it, and it shares no code with the GPU path.
 *
 * What it follows (arXiv 2607.04127):
 *   - map representation Theta = {mu, q, s~, alpha} of 2D Gaussian primitives (Sec. 3.1);
 *   - rendering under the spherical projection into predicted depth, opacity and normals
 *     on the scan's grid (Sec. 3.1, Sec. 3.4), with the surfel (2D Gaussian) ray
 *     intersection of the cited 2DGS work;
 *   - log-scale parameterisation s = exp(s~) (Sec. 3.3, range-adaptive scale init);
 *   - valid-depth mask M_D = [D > 0], masked depth L1 and the cosine normal loss with
 *     mask M_N = M_D * [|N| > 0] (Sec. 3.4, Eq. 10 left and Eq. 11 first term);
 *   - weights lambda_n = 1 and lambda_{n,g} = 0.05 (Sec. 4.1, implementation details).
 * Readings where the paper is silent (compositing order, stabilisers, beam model, pose
 * convention) are stated beside each function in lgsr_ref.c.
 *
 * All arrays are HOST memory in float64.  Inputs that the GPU receives as float32 are
 * promoted exactly by the caller.  Functions return 0 on success and -1 on bad arguments.
 */
#ifndef LGSR_REF_H
#define LGSR_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double cutoff_sigma; /* a hit counts while u^2 + v^2 <= cutoff_sigma^2 */
    double alpha_thr;    /* a hit with alpha_hat < alpha_thr is skipped */
    double alpha_max;    /* alpha_hat = min(alpha_max, alpha * G) */
    double T_min;        /* stop once the transmittance drops below T_min (that hit included) */
    double near;         /* surfels whose centre is nearer than this are dropped; hits with t < near skipped */
    double den_eps;      /* |n'.d| < den_eps: ray parallel to the surfel plane, skipped */
    double drop_tau;     /* rendered ray drop = [A < drop_tau] */
} lgsr_ref_params;

typedef struct {
    int64_t n;
    const double *means;          /* n x 3, world frame */
    const double *quats;          /* n x 4, (w, x, y, z), any nonzero norm */
    const double *log_scales;     /* n x 2 */
    const double *opacity_logits; /* n */
} lgsr_ref_map;

typedef struct {
    int32_t H, W;
    const double *row_sincos; /* H x 2: (sin phi_k, cos phi_k), row 0 = top beam */
    const double *col_sincos; /* W x 2: (sin th_j, cos th_j) */
} lgsr_ref_beams;

/* Render n_rays rays (ray_ids[i] = k * W + j, or all H*W rays in order when ray_ids is NULL).
 * Outputs per ray: depth, opacity, normal (x3, sensor frame), drop; optional (NULL to skip):
 * t_final (transmittance after the last hit), n_contrib (hits composited), margin (smallest
 * relative distance of any threshold decision to its threshold, see lgsr_ref.c), order_gap
 * (smallest relative centre-range gap between consecutive composited surfels), n_hits
 * (hits passing every test when early termination is ignored), den_min (smallest |n'.d| over
 * the composited hits, infinity without one). */
int lgsr_ref_forward(const lgsr_ref_map *map, const double pose[12], const lgsr_ref_beams *beams,
                     const lgsr_ref_params *prm, int64_t n_rays, const int64_t *ray_ids,
                     double *depth, double *opacity, double *normal, uint8_t *drop,
                     double *t_final, int32_t *n_contrib, double *margin, double *order_gap,
                     int32_t *n_hits, double *den_min);

/* Loss over n_rays rays and its gradient with respect to the rendered depth, opacity and
 * normal.  ray_weight (NULL = all ones) multiplies the valid masks; it restricts the loss to
 * a ray subset.  loss[5] = {total, depth term, normal term, |Omega_D|, |Omega_N|}. */
int lgsr_ref_loss(int64_t n_rays, const double *depth, const double *opacity, const double *normal,
                  const double *target_depth, const double *target_normal, const double *ray_weight,
                  double w_depth, double lambda_n, double lambda_ng, double loss[5],
                  double *g_depth, double *g_opacity, double *g_normal);

/* Backward of lgsr_ref_forward: given dL/d(depth, opacity, normal) per ray, accumulate the
 * gradient with respect to every surfel parameter (outputs are overwritten) and the pose in
 * the right-perturbation tangent (rho, omega) of T_ws * Exp(xi).
 * Optional (NULL to skip), for test tolerances: mass (n x 4) receives per surfel, for the
 * gradient of means, quats, log_scales and opacity_logit, the sum over rays of the norm of
 * each ray's contribution evaluated on magnitudes (every term and coefficient by absolute
 * value, before any cancellation: a running error bound); pose_mass[6] likewise per pose
 * component. */
int lgsr_ref_backward(const lgsr_ref_map *map, const double pose[12], const lgsr_ref_beams *beams,
                      const lgsr_ref_params *prm, int64_t n_rays, const int64_t *ray_ids,
                      const double *g_depth, const double *g_opacity, const double *g_normal,
                      double *d_means, double *d_quats, double *d_log_scales,
                      double *d_opacity_logits, double d_pose[6], double *mass, double *pose_mass);

/* Normals of the rendered surface (Sec. 3.4, N_surf) for every pixel of an H x W range
 * image: n_surf (H*W x 3, zero where undefined), defined (H*W, may be NULL), flip_margin
 * (H*W, may be NULL: |v.d| / |v| of the orientation decision, +inf where undefined). */
int lgsr_ref_surf_normal(const lgsr_ref_beams *beams, const double *depth, double *n_surf, uint8_t *defined,
                         double *flip_margin);

/* Frame terms of the mapping objective (Eq. 10, Eq. 11, weighted as in Eq. 13) over the full
 * H x W image of `beams`, and their gradient with respect to the rendered depth, opacity and
 * normal (all three NULL to skip; overwritten).  loss[8] = {total, depth term, opacity term,
 * G-ICP normal term, rendered-surface normal term, |Omega_D|, |Omega_N|, |Omega_S|} with
 * Omega_S the rays of Omega_D whose N_surf is defined. */
int lgsr_ref_objective(const lgsr_ref_beams *beams, const double *depth, const double *opacity,
                       const double *normal, const double *target_depth, const double *target_normal,
                       double w_depth, double lambda_alpha, double eps, double lambda_n, double lambda_ng,
                       double lambda_ns, double loss[8], double *g_depth, double *g_opacity, double *g_normal);

/* Scale regulariser (Eq. 12, times lambda_s): *loss, and g_log_scales (n x 2, NULL to skip,
 * overwritten); margin (n, NULL to skip) = |max(s) - s_max| / s_max. */
int lgsr_ref_scale_reg(int64_t n, const double *log_scales, double lambda_s, double s_max, double *loss,
                       double *g_log_scales, double *margin);

/* Spherical projection of a scan (n points, sensor frame, n x 3; normals n x 3 or NULL) onto
 * the H x W grid with rows from el_max (row 0) to el_min and columns over the full turn:
 * nearest return per pixel.  depth (H*W, 0 = none), normal (H*W x 3, may be NULL: the
 * winner's normal turned to face the sensor, zero if none), index (H*W, the winning point,
 * -1 if none), bin_margin (n, may be NULL). */
int lgsr_ref_scan_to_range(int64_t n, const double *points, const double *normals, int32_t H, int32_t W,
                           double el_min, double el_max, double r_min, double r_max, double *depth,
                           double *normal, int64_t *index, double *bin_margin);

/* Target covariances of surfels (n x 6: xx, xy, xz, yy, yz, zz), thickness eps. */
int lgsr_ref_target_cov(int64_t n, const double *quats, const double *log_scales, double eps, double *cov);

/* The surfels that render (valid rotation, centre range >= near) in compositing order:
 * ascending sensor-frame centre range, equal ranges by ascending index (R3); order[k] the
 * surfel index, range[k] its range (both capacity n), *m the count. */
int lgsr_ref_order(const lgsr_ref_map *map, const double pose[12], const lgsr_ref_params *prm, int64_t *order,
                   double *range, int64_t *m);

/* The composited surfels of each ray, front to back: ray i's ids in ids[i cap ..], at most
 * cap of them; count[i] = its number of composited hits K. */
int lgsr_ref_contributors(const lgsr_ref_map *map, const double pose[12], const lgsr_ref_beams *beams,
                          const lgsr_ref_params *prm, int64_t n_rays, const int64_t *ray_ids, int64_t *ids,
                          int64_t cap, int32_t *count);

/* Set the number of OpenMP threads later calls run with (n > 0). */
void lgsr_ref_set_threads(int n);

/* Number of OpenMP threads the oracle runs with. */
int lgsr_ref_threads(void);

#ifdef __cplusplus
}
#endif
#endif
