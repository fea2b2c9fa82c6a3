/*
 * lgsr.h -- C ABI of the MI355X (gfx950) spherical surfel range-image renderer.
 *
 * The library renders a map of surface-oriented 2D anisotropic Gaussians (surfels) into
 * a spinning-LiDAR range image -- per-ray depth, opacity, normal and ray-drop mask -- and
 * back-propagates a range-image loss to every surfel parameter and to the 6-DoF sensor
 * pose.  It follows arXiv 2607.04127 ("Real-Time LiDAR Gaussian Splatting SLAM via
 * Geometry-Aware Covariance Coupling"):
 *   Sec. 3.1  map Theta = {(mu_i, q_i, s~_i, alpha_i)} rendered under the spherical
 *             projection pi_s into (D^, A^, N^) on the scan's grid;
 *   Sec. 3.3  log-scale parameterisation s~ = log s;
 *   Sec. 3.4  mapping: rasterise, compare with the observations on valid pixels
 *             M_D = [D > 0] (masked depth L1, Eq. 10 left; G-ICP normal cosine term with
 *             M_N = M_D [|N| > 0], Eq. 11 first term), optimise Theta;
 *   Sec. 4.1  loss weights lambda_n = 1, lambda_{n,g} = 0.05.
 * The primitive is the 2DGS surfel cited in Sec. 1: a planar Gaussian
 * G = exp(-(u^2 + v^2) / 2) at the exact ray/plane hit (u, v) in units of its two scales,
 * composited front to back by ascending sensor-frame centre range (ties: lower index),
 * with alpha_hat = min(alpha_max, alpha G), hits below alpha_thr skipped and traversal
 * stopped after the hit that takes the transmittance below T_min.  Outputs: opacity
 * A = sum of weights, depth = opacity-normalised expected range, normal = opacity-
 * normalised sum of sensor-facing surfel normals (sensor frame), drop = [A < drop_tau];
 * a ray with no hit renders all zeros and drop = 1.
 *
 * Conventions
 *   - float32 everywhere; sizes int64 / int32.  Pointers are DEVICE pointers unless marked
 *     HOST.  The caller owns every input and output buffer; the library owns its context
 *     workspace and the lgsr_state objects it returns.
 *   - surfel layout (structure of arrays, row-major, contiguous): means n x 3 (world),
 *     quats n x 4 as (w, x, y, z) of any nonzero norm whose rotation's columns are
 *     (major tangent a, minor tangent b, normal n), log_scales n x 2, opacity_logits n
 *     (opacity = sigmoid(logit)).  A surfel with a zero quaternion or whose centre lies
 *     nearer than `near` renders nothing and gets zero gradient.
 *   - pose: 3 x 4 row-major [R | t] mapping sensor coordinates to world coordinates.
 *     Pose gradients are in the tangent (rho, omega) of the right perturbation
 *     T * Exp(xi): mu' -> mu' - rho + mu' x omega to first order.
 *   - beams: row_sincos H x 2 holds (sin phi_k, cos phi_k), row 0 the highest beam, rows
 *     strictly decreasing in elevation within (-90, 90) degrees; col_sincos W x 2 holds
 *     (sin th_j, cos th_j) with th_j = 2 pi j / W (uniform azimuth, counter-clockwise from
 *     +x).  Pixel (k, j), ray index k * W + j, is one ray of direction
 *     (cos phi_k cos th_j, cos phi_k sin th_j, sin phi_k).  The library relies on this
 *     layout for culling; other tables give undefined images.  1 <= H, W <= 32768.
 *   - per-ray images are row-major H x W (normals H x W x 3).
 *   - all calls are asynchronous on the context's HIP stream unless stated; errors are
 *     status codes (no exception crosses the ABI) with a message from lgsr_last_error.
 *     Arguments are validated before anything is launched.  A kernel fault surfaces as
 *     LGSR_EDEVICE at a later synchronising call.
 *   - one context may be used by one host thread at a time; calls on one context are
 *     ordered on its stream.
 */
#ifndef LGSR_H
#define LGSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LGSR_OK = 0,
    LGSR_EINVAL = -1,     /* invalid argument (null pointer, size out of range, bad option) */
    LGSR_ENOMEM = -2,     /* device or pinned-host allocation failed */
    LGSR_EDEVICE = -3,    /* HIP runtime error: no device, launch failure, earlier kernel fault */
    LGSR_ECAPACITY = -4,  /* the (surfel, tile) pair list would exceed the configured limit */
    LGSR_ESTATE = -5,     /* state from another context, or used after its context changed device */
    LGSR_EINTERNAL = -6
} lgsr_status;

typedef struct {
    int64_t n;
    const float *means;          /* n x 3 */
    const float *quats;          /* n x 4 */
    const float *log_scales;     /* n x 2 */
    const float *opacity_logits; /* n */
} lgsr_surfels;

typedef struct {
    int32_t H, W;
    const float *row_sincos; /* H x 2 */
    const float *col_sincos; /* W x 2 */
} lgsr_beams;

typedef struct {
    float cutoff_sigma; /* hits count while u^2 + v^2 <= cutoff_sigma^2      (default 3)      */
    float alpha_thr;    /* hits with alpha_hat < alpha_thr are skipped         (default 1/255)  */
    float alpha_max;    /* alpha_hat = min(alpha_max, alpha G)                 (default 0.99)   */
    float T_min;        /* stop after the hit taking transmittance below T_min (default 1e-4)   */
    float near;         /* centres nearer than this are dropped; hits at t < near skipped (0.2) */
    float den_eps;      /* |n . d| < den_eps: ray parallel to the surfel, skipped (1e-6)        */
    float drop_tau;     /* rendered drop = [A < drop_tau]                      (default 0.5)    */
    int32_t chunk;      /* list entries per parallel chunk; 0 = chosen from the pair count, else
                           16..65536.  Results do not depend on it beyond float32 rounding.     */
    int32_t flags;      /* 0, or LGSR_FLAG_BATCH_FUSED (lgsr_render_batch only; others ignore it) */
} lgsr_raster_opts;

/* lgsr_render_batch: composite all requests of the batch with one launch per stage (chunks,
 * merge, fix-up) after every request's lists are built, instead of each request on its own
 * stream as soon as its lists are ready.  Same results. */
#define LGSR_FLAG_BATCH_FUSED 1

typedef struct {
    float *depth;   /* H x W   */
    float *opacity; /* H x W   */
    float *normal;  /* H x W x 3, sensor frame */
    uint8_t *drop;  /* H x W   */
} lgsr_frame;

typedef struct {
    float w_depth;   /* weight of the masked depth L1 term            (default 1)    */
    float lambda_n;  /* weight of the normal loss                     (default 1)    */
    float lambda_ng; /* weight of the G-ICP normal cosine term inside (default 0.05) */
} lgsr_loss_weights;

/* Weights of the full mapping objective (Eq. 13 with Eq. 10-11; values of Sec. 4.1).  eps
 * is not given numerically in the paper; lambda_ns is zero until densification starts
 * (Sec. 3.4), which is the caller's schedule. */
typedef struct {
    float w_depth;      /* masked depth L1 (Eq. 10 left)                      (default 1)    */
    float lambda_alpha; /* positive-only opacity BCE (Eq. 10 right)           (default 0.1)  */
    float eps;          /* inside log(A^ + eps)                               (default 1e-6) */
    float lambda_n;     /* normal loss (Eq. 13)                               (default 1)    */
    float lambda_ng;    /* G-ICP normal cosine term (Eq. 11)                  (default 0.05) */
    float lambda_ns;    /* rendered-surface normal cosine term (Eq. 11)       (default 0.01) */
} lgsr_objective_weights;

typedef struct {
    float *d_depth;   /* H x W     dL/d depth   */
    float *d_opacity; /* H x W     dL/d opacity */
    float *d_normal;  /* H x W x 3 dL/d normal  */
} lgsr_frame_grad;

typedef struct {
    float *means;          /* n x 3 */
    float *quats;          /* n x 4 */
    float *log_scales;     /* n x 2 */
    float *opacity_logits; /* n     */
} lgsr_surfel_grads;

typedef struct lgsr_ctx lgsr_ctx;     /* library-owned, opaque */
typedef struct lgsr_state lgsr_state; /* library-owned, opaque */

/* Fill *opts / *w with the defaults listed above. */
void lgsr_default_opts(lgsr_raster_opts *opts);
void lgsr_default_loss_weights(lgsr_loss_weights *w);
void lgsr_default_objective_weights(lgsr_objective_weights *w);

/* Create a context on HIP device `device` issuing all work on `hip_stream` (a hipStream_t;
 * NULL = the device's null stream).  Allocates a small workspace; later calls grow it.
 * Errors: EINVAL (out == NULL), EDEVICE (no such device), ENOMEM. */
lgsr_status lgsr_create(lgsr_ctx **out, int device, void *hip_stream);

/* Wait for the context's stream, then free the context, its workspace and every state it
 * created (live or freed); handles of those states must not be used afterwards.  NULL is a
 * no-op. */
void lgsr_destroy(lgsr_ctx *ctx);

/* Switch the stream later calls are issued on (NULL = null stream). */
lgsr_status lgsr_set_stream(lgsr_ctx *ctx, void *hip_stream);

/* Message of the last failed call on ctx; valid until the next call on ctx. */
const char *lgsr_last_error(const lgsr_ctx *ctx);

/* Render the surfels seen from pose_ws (Sec. 3.1, Sec. 3.4 rasterisation).
 *   pose_ws: 12 floats, HOST memory when pose_on_device == 0, DEVICE memory otherwise.
 *   out: caller-owned frame buffers, fully overwritten.
 *   state: if not NULL, receives a new state holding what lgsr_backward needs (sorted
 *          (surfel, tile) lists, per-surfel records, per-ray transmittance); it refers to
 *          the surfel buffers and the beam tables, which must stay unchanged until the
 *          backward has been issued.  Free it with lgsr_state_free.
 * The call reads back one integer (the number of (surfel, tile) pairs) to size the pair
 * list, so it waits for the projection kernels of this call; everything else is async.
 * Errors: EINVAL, ENOMEM, ECAPACITY (more than 2^31 - 1 pairs), EDEVICE. */
lgsr_status lgsr_forward(lgsr_ctx *ctx, const lgsr_surfels *surfels, const float *pose_ws,
                         int32_t pose_on_device, const lgsr_beams *beams,
                         const lgsr_raster_opts *opts, lgsr_frame *out, lgsr_state **state);

/* Loss of a rendered frame against targets (Sec. 3.4, Eq. 10 left and Eq. 11 first term):
 *   L = w_depth / |Omega_D| sum M_D |D^ - D|
 *     + lambda_n lambda_ng / |Omega_N| sum M_N (1 - N^ . N / |N^|),
 * M_D = [D > 0], M_N = M_D [|N| > 0]; an empty mask gives a zero term; |0| has zero
 * slope; a ray rendering a zero normal costs 1 with zero gradient.
 *   n_rays: number of rays (H * W), >= 0.
 *   target_depth: n_rays (0 = no return); target_normal: n_rays x 3, unit, sensor frame.
 *   loss_out: DEVICE float[5] = {total, depth term, normal term, |Omega_D|, |Omega_N|}.
 *   grad_out: caller-owned dL/d(depth, opacity, normal); d_opacity is zero for this loss.
 * Errors: EINVAL, EDEVICE. */
lgsr_status lgsr_loss(lgsr_ctx *ctx, int64_t n_rays, const lgsr_frame *pred,
                      const float *target_depth, const float *target_normal,
                      const lgsr_loss_weights *weights, float *loss_out, lgsr_frame_grad *grad_out);

/* lgsr_loss without any device allocation, for callers that cannot allocate: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * result and errors as lgsr_loss, on the context's stream.  The loss's partial sums go to a
 * static device array of 4096 floats (16 KiB, one per device, held until the process ends)
 * instead of the context's workspace; the loss needs at most 4 per workgroup and at most
 * 1024 workgroups for any n_rays, and a larger need is refused with ECAPACITY.  Every call on
 * one device shares that array: calls that overlap on one device (several streams or host
 * threads) race and must be serialised by the caller.  Nothing in the array has to start at
 * zero.  ESTATE if the array's address could not be taken when the context was created. */
lgsr_status lgsr_loss_noalloc(lgsr_ctx *ctx, int64_t n_rays, const lgsr_frame *pred,
                              const float *target_depth, const float *target_normal,
                              const lgsr_loss_weights *weights, float *loss_out, lgsr_frame_grad *grad_out);

/* Frame terms of the full mapping objective (Sec. 3.4: Eq. 10, Eq. 11, weighted as in
 * Eq. 13) and their gradient:
 *   L = w_depth / |Omega_D| sum_{Omega_D} |D^ - D|
 *     - lambda_alpha / |Omega_D| sum_{Omega_D} log(A^ + eps)
 *     + lambda_n lambda_ng / |Omega_N| sum_{Omega_N} (1 - N^ . N / |N^|)
 *     + lambda_n lambda_ns / |Omega_D| sum_{Omega_D, N_surf defined} (1 - N^ . N_surf / |N^|)
 * N_surf (Sec. 3.4 (ii)) at pixel (k, j) is the unit normal of the rendered surface:
 * v = (P(k, j+1) - P(k, j-1)) x (P(k+1, j) - P(k-1, j)), P = D^ d (d from the beam tables;
 * columns wrap around the full turn), turned to face the sensor; defined on rows 1..H-2
 * when the four neighbours rendered a range (D^ > 0) and v != 0.  The gradient is the full
 * derivative, through N^ and through the neighbours' D^ inside N_surf.
 *   beams: the H x W beam model the frame was rendered with (device tables).
 *   pred: the rendered frame (depth, opacity, normal read; drop unused).
 *   target_depth: H x W (0 = no return); target_normal: H x W x 3 (zero = none), sensor frame.
 *   loss_out: DEVICE float[8] = {total, depth term, opacity term, G-ICP normal term,
 *             surface normal term, |Omega_D|, |Omega_N|, |Omega_S|} (Omega_S: rays of Omega_D
 *             whose N_surf is defined).
 *   grad_out: caller-owned dL/d(depth, opacity, normal), overwritten; NULL = loss only.
 * Errors: EINVAL (NULL or inconsistent arguments, eps < 0), EDEVICE. */
lgsr_status lgsr_objective(lgsr_ctx *ctx, const lgsr_beams *beams, const lgsr_frame *pred,
                           const float *target_depth, const float *target_normal,
                           const lgsr_objective_weights *weights, float *loss_out,
                           lgsr_frame_grad *grad_out);

/* Scale regulariser (Sec. 3.4, Eq. 12, times lambda_s of Eq. 13):
 *   L = lambda_s sum_i max(0, max(s_x, s_y) - s_max),  s = exp(log_scales).
 *   log_scales: DEVICE n x 2, 8-byte aligned.  s_max > 0 (not given numerically in the paper).
 *   loss_out: DEVICE float[1].
 *   grad_log_scales: DEVICE n x 2, 8-byte aligned, ACCUMULATED into (dL/dlog s_k = lambda_s s_k
 *     for the larger scale when it exceeds s_max, the first one on a tie); NULL = loss only.
 *     Issue it after lgsr_backward to add the regulariser to the rendering gradient.
 * Errors: EINVAL, EDEVICE. */
lgsr_status lgsr_scale_reg(lgsr_ctx *ctx, int64_t n, const float *log_scales, float lambda_s, float s_max,
                           float *loss_out, float *grad_log_scales);

/* The spherical grid a scan is projected onto (Sec. 3.1): H rows uniform in elevation from
 * el_max (row 0) down to el_min (row H - 1), W columns uniform over the full turn (column j
 * at azimuth 2 pi j / W, azimuth measured from +x towards +y), the grid the renderer's beam
 * tables describe.  Angles in radians; returns with range outside [r_min, r_max] are dropped. */
typedef struct {
    int32_t H, W;  /* H >= 2, W >= 1 */
    float el_min, el_max;  /* el_max > el_min */
    float r_min, r_max;    /* 0 <= r_min <= r_max (r_max may be +inf) */
} lgsr_scan_grid;

/* Scan to range image (Sec. 3.1; the target image D and G-ICP normal image of Sec. 3.4): each
 * point (sensor frame) goes to the nearest row and column of `grid`, is kept inside the rows
 * and the range gates, and the nearest return wins each pixel (equal ranges: the lower point
 * index).  A pixel takes the winner's range and its normal turned to face the sensor.
 *   points: DEVICE n x 3 float; normals: DEVICE n x 3 (e.g. the smallest principal axes of
 *     the tracker's point covariances) or NULL (normal image zero).
 *   depth: DEVICE H x W (0 = no return); normal: DEVICE H x W x 3 or NULL;
 *   index: DEVICE H x W int32 (winning point, -1 = none) or NULL.
 * n < 2^31.  Uses 8 bytes of workspace per pixel.  Errors: EINVAL, ENOMEM, EDEVICE. */
lgsr_status lgsr_scan_to_range(lgsr_ctx *ctx, int64_t n, const float *points, const float *normals,
                               const lgsr_scan_grid *grid, float *depth, float *normal, int32_t *index);

/* Target covariances for covariance-weighted G-ICP (Sec. 3.2): per surfel
 * Sigma = R diag(s_x^2, s_y^2, eps^2) R^T, R = [a b n] the rotation of the normalised
 * quaternion, s = exp(log_scales), eps the thickness along the normal (not given numerically
 * in the paper); a zero quaternion gives a zero covariance.
 *   quats: DEVICE n x 4 (w, x, y, z), 16-byte aligned; log_scales: DEVICE n x 2, 8-byte aligned.
 *   cov: DEVICE n x 6 = (xx, xy, xz, yy, yz, zz), world frame, 8-byte aligned.
 * Errors: EINVAL, EDEVICE. */
lgsr_status lgsr_target_cov(lgsr_ctx *ctx, int64_t n, const float *quats, const float *log_scales, float eps,
                            float *cov);

/* Backward of the forward that produced `state`: given dL/d(depth, opacity, normal) per
 * ray, write dL/d every surfel parameter into `out` (overwritten; zero for surfels that
 * render nothing) and dL/d(rho, omega) into grad_pose (DEVICE float[6], overwritten).
 * Per-surfel gradients are summed with float atomics, so the last bits can vary from run
 * to run.  Errors: EINVAL, ESTATE, ENOMEM, EDEVICE. */
lgsr_status lgsr_backward(lgsr_ctx *ctx, lgsr_state *state, const lgsr_frame_grad *grad_in,
                          lgsr_surfel_grads *out, float *grad_pose);

/* Release a state (its buffers return to the context's pool).  NULL is a no-op. */
void lgsr_state_free(lgsr_state *state);

/* Counters of the forward that produced `state` (waits for it), HOST int64[8]:
 *   out[0] (surfel, tile) pairs            out[1] surfels that survived culling
 *   out[2] bytes of device workspace held by the context and the state
 *   out[3] longest per-tile list           out[4] ray-surfel tests the raster performs
 *          (64 per pair and overlapping 8 x 8 wave sub-tile)
 *   out[5] composited hits (sum over rays of the hit count)
 *   out[6] rays with at least one hit
 *   out[7] ray tests a front-to-back walk needs: as out[4], but per wave sub-tile only up to
 *          the last contributor of its slowest ray (the whole list if a ray never drops
 *          below T_min). */
lgsr_status lgsr_query(lgsr_ctx *ctx, const lgsr_state *state, int64_t out[8]);

/* Depth of the per-ray lists of the forward that produced `state` (waits for it), HOST
 * int64[2]: out[0] the (ray, surfel) hits that pass every per-hit test (cut-off, alpha_thr,
 * near, den_eps) summed over rays, counting the hits behind the point where the ray's
 * transmittance fell below T_min as well; out[1] the rays with at least one such hit.  The
 * beam tables and the surfel arrays of that forward must still hold their values.
 * Errors: EINVAL, ESTATE, EDEVICE. */
lgsr_status lgsr_count_hits(lgsr_ctx *ctx, const lgsr_state *state, int64_t out[2]);

/* The sorted list of one 16 x 16-ray tile (tile row tile_row covers ray rows 16 tile_row ..
 * 16 tile_row + 15, likewise columns) of the forward that produced `state`: the ids of the
 * surfels whose conservative ray rectangle meets the tile, in compositing order (ascending
 * sensor-frame centre range, ties by lower index; Sec. 3.1 rendering order as read above).
 * Every surfel that contributes to a ray of the tile must be in it.  Copies
 * min(*count, cap) ids into ids (HOST) and sets *count to the list length; waits for the
 * stream.  Errors: EINVAL (tile outside the grid, NULL count, ids NULL with cap > 0),
 * ESTATE, EDEVICE. */
lgsr_status lgsr_tile_list(lgsr_ctx *ctx, const lgsr_state *state, int32_t tile_row, int32_t tile_col,
                           uint32_t *ids, int64_t cap, int64_t *count);

/* Streaming probe, outside the rendering path: the HBM bandwidth a plain streaming kernel
 * reaches on this device, the denominator of the path's HBM fraction, and a cache flush
 * between timed steps.  kind 0 (copy): a[i] = b[i] (8 bytes per float); kind 1 (triad):
 * a[i] = b[i] + 3 c[i] (12 bytes per float), both with non-temporal 4-vector accesses per
 * lane; kinds 2 and 3: the same with plain one-vector accesses.  blocks: 256-lane
 * workgroups striding over the arrays (0 = 4096).  n floats, a multiple of 4; a, b, c
 * DEVICE, 16-byte aligned, not overlapping.  Asynchronous on the context's stream.
 * Errors: EINVAL, EDEVICE. */
lgsr_status lgsr_stream_probe(lgsr_ctx *ctx, int32_t kind, const float *b, const float *c, float *a, int64_t n,
                              int32_t blocks);

/* Stage timers.  lgsr_profile selects stages by bit mask (bit k = stage k, 0 = off, -1 =
 * all); each selected stage is then bracketed by HIP events on the context's stream (a
 * stage may span several kernel launches; every event costs a little stream time).
 * lgsr_profile_read waits for the stream, adds up the elapsed times per stage since the
 * last read (HOST double[10], milliseconds) and the number of times each stage ran (HOST
 * int64[10]), then resets them. */
enum {
    LGSR_STAGE_PROJECT = 0,    /* projection, records, rectangles, per-tile pair counts */
    LGSR_STAGE_SCAN = 1,       /* tile offsets, list bounds and the pair count */
    LGSR_STAGE_READBACK = 2,   /* the one device-to-host read (pair count, longest list) */
    LGSR_STAGE_EMIT = 3,       /* surfel ids into the tile lists */
    LGSR_STAGE_TILE_SORT = 4,  /* each tile list by (range, index) */
    LGSR_STAGE_RASTER_FWD = 5, /* forward compositing: chunk list, chunks, merge, fix-up */
    LGSR_STAGE_LOSS = 6,       /* loss and its per-ray gradient */
    LGSR_STAGE_BWD_PREP = 7,   /* clearing the record gradients (after a new allocation only) */
    LGSR_STAGE_RASTER_BWD = 8, /* backward compositing */
    LGSR_STAGE_CHAIN = 9,      /* parameter and pose gradients */
    LGSR_NUM_STAGES = 10
};
lgsr_status lgsr_profile(lgsr_ctx *ctx, int32_t stage_mask);
lgsr_status lgsr_profile_read(lgsr_ctx *ctx, double ms[10], int64_t calls[10]);

/* Wait for all work issued on the context's stream; reports an earlier kernel fault. */
lgsr_status lgsr_sync(lgsr_ctx *ctx);

/* A batch of render or render + gradient requests (the rendering-service path).  Each
 * request names its own map, pose, beam model and outputs; requests of one batch may mix
 * maps and resolutions.  Every request's projection and tile offsets are issued first,
 * spread over four streams, then the library waits once per request for its pair count
 * and issues the rest (lists, compositing and, for a request with targets, lgsr_loss and
 * lgsr_backward) on the same streams.  One host wait per request instead of one per stage
 * chain, and kernels of different requests overlap on the GPU.  Sec. 3.4's mapping step
 * renders and differentiates many keyframes this way.
 * All pointers in a request are DEVICE pointers except pose_ws (by value) and the request
 * array itself (HOST).  target_depth == NULL: render only (the gradient fields are then
 * ignored).  With targets, loss_out (float[5]), frame_grad (H x W scratch that receives
 * dL/d(frame)), grads (n) and grad_pose (6) must be set.  Outputs of different requests
 * must not overlap.  The call returns once everything is issued; the context's stream
 * orders after all of it (lgsr_sync waits for it).  Arguments of every request are
 * validated before anything is issued (LGSR_EINVAL, naming the request). */
typedef struct {
    lgsr_surfels surfels;
    float pose_ws[12]; /* 3 x 4 row-major [R | t], sensor to world */
    lgsr_beams beams;
    lgsr_frame out;
    const float *target_depth;  /* H x W or NULL */
    const float *target_normal; /* H x W x 3 */
    float *loss_out;            /* device float[5] */
    lgsr_frame_grad frame_grad; /* H x W scratch */
    lgsr_surfel_grads grads;    /* n, overwritten */
    float *grad_pose;           /* device float[6] */
} lgsr_request;
lgsr_status lgsr_render_batch(lgsr_ctx *ctx, int32_t n, const lgsr_request *requests /* HOST */,
                              const lgsr_raster_opts *opts, const lgsr_loss_weights *weights);

/* Device bytes one request holds beyond its inputs and outputs (host computation, no
 * device needed): the buffers of its state (records, rectangles, keys, pair lists and sort
 * workspace, chunk list and per-chunk summaries, per-ray state) for a map of n surfels, an
 * H x W beam model and P (surfel, tile) pairs at the automatic chunk length, and, when
 * with_grad, the loss and backward scratch, each sized as the library allocates it.  A
 * service admits requests against an HBM budget with it.  Errors: EINVAL. */
lgsr_status lgsr_request_bytes(int64_t n, int32_t H, int32_t W, int64_t P, int32_t with_grad, int64_t *bytes);

/* Completion of the requests of the most recent lgsr_render_batch on the context, without
 * waiting: done[i] (HOST int32, n entries) = 1 once request i's kernels have finished and its
 * outputs hold their values, else 0.  A service can hand each result on as soon as it is
 * ready instead of at the end of the whole batch.  n must not exceed the number of requests
 * that batch issued.  Errors: EINVAL, EDEVICE (a kernel of the batch faulted). */
lgsr_status lgsr_batch_poll(lgsr_ctx *ctx, int32_t n, int32_t *done);

/* Device bytes held by `state` (HOST int64 out); no GPU work, no wait.  A caller that keeps
 * states from forward to backward can budget HBM with it, and recompute (run the forward
 * again, which is deterministic) instead of keeping a state when the budget is spent.
 * state == NULL: the bytes the context itself retains (its workspace, the scratch of the
 * loss and backward, the states of earlier batches kept for reuse). */
lgsr_status lgsr_state_bytes(lgsr_ctx *ctx, const lgsr_state *state, int64_t *bytes);

/* One Adam step (Kingma and Ba; the map optimisation of Sec. 3.4 does not name its
 * optimiser, this is the usual choice for Gaussian maps) over up to 8 groups of float32
 * arrays in one launch.  Per element, with t = step >= 1:
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   p -= lr * (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
 * All pointers DEVICE, n elements each; param, m and v are updated in place (m, v start at
 * zero).  Arrays of different groups must not overlap.  LGSR_EINVAL for n_groups outside
 * [0, 8], a NULL array with n > 0, step < 1, or beta outside [0, 1). */
typedef struct {
    int64_t n;
    float *param;
    const float *grad;
    float *m;
    float *v;
    float lr;
} lgsr_adam_group;
lgsr_status lgsr_adam_step(lgsr_ctx *ctx, int32_t n_groups, const lgsr_adam_group *groups /* HOST */, float beta1,
                           float beta2, float eps, int32_t step);

#ifdef __cplusplus
}
#endif
#endif
