// lgsr_kernels.h -- host-side launchers of the renderer's kernels (internal interface
// between the C-ABI layer and the kernel files).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lgsr_internal.h"

namespace lgsr {

// ---- sort.hip ----
size_t scan_tmp_words(int64_t n);
// out[i] = sum_{k<i} x_k with x_k = in[k] (or in[gather[k]]); *total (device, may be null)
// receives the sum of all n.  n <= 4096 * 4096.  In-place (out == in) is allowed.
hipError_t scan_u32(const uint32_t *in, const uint32_t *gather, uint32_t *out, uint32_t *total, int64_t n,
                    uint32_t *tmp, hipStream_t s);
size_t radix_hist_words(int64_t n);
// Stable sort by the low `bits` bits of keys; on return *in_alt tells whether the sorted
// data ended in (keys_alt, vals_alt).
hipError_t radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt, int64_t n,
                            int bits, uint32_t *hist, uint32_t *scan_tmp, hipStream_t s, bool *in_alt);

// ---- project.hip ----
struct SurfelPtrs {
    const float *means, *quats, *log_scales, *logits;
    int64_t n;
};

hipError_t launch_project(const SurfelPtrs &S, const Pose &pose_val, const float *pose_dev, float *pose_out,
                          const float *rows, const Grid &g, const RasterParams &p, float *recs, uint2 *rects,
                          uint32_t *keys, uint32_t *vals, uint32_t *cnt, hipStream_t s);
hipError_t launch_emit(const uint32_t *sorted_ids, const uint32_t *cnt, const uint32_t *offs, const uint2 *rects,
                       int64_t n, const Grid &g, uint32_t *pair_keys, uint32_t *pair_vals, hipStream_t s);
hipError_t launch_ranges(const uint32_t *sorted_keys, int64_t P, int T, uint2 *ranges, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_count_visible(const uint2 *rects, int64_t n, uint32_t *out, hipStream_t s);
hipError_t launch_max_range(const uint2 *ranges, int T, uint32_t *out, hipStream_t s);
// out[0] ray-surfel tests, out[1] composited hits, out[2] rays with a hit (u64, zeroed here)
hipError_t launch_work_counts(const uint32_t *tile_keys, const uint32_t *ids, const uint2 *rects, int64_t P,
                              const float4 *st1, const Grid &g, unsigned long long *out, hipStream_t s);

// ---- raster.hip ----
struct RasterBufs {
    const uint32_t *ids;  // sorted pair surfel ids
    const float *recs;
    const uint2 *rects, *ranges;
    const float *rows, *cols;
    uint4 *chunks;         // items_max x (tile, first, end, 0)
    uint32_t *chunk_base;  // T + 1
    uint32_t *n_items;     // device counter
    float *slots;          // chunk_slot_floats(items_max)
    float4 *st0, *st1;     // per ray
    float4 *fixA, *fixB;   // per ray
    int seg;
    int64_t items_max;
};
int chunk_size(int64_t P, int requested);
int64_t chunk_items_max(int64_t P, int T, int seg);
size_t chunk_slot_floats(int64_t items_max);
hipError_t launch_raster_fwd(const RasterBufs &R, const Grid &g, const RasterParams &p, float *depth,
                             float *opacity, float *normal, uint8_t *drop, hipStream_t s);
hipError_t launch_raster_bwd_prep(const RasterBufs &R, const Grid &g, const float *gD, const float *gA,
                                  const float *gN, float4 *gb0, float *gb1, hipStream_t s);
hipError_t launch_raster_bwd(const RasterBufs &R, const Grid &g, const RasterParams &p, const float4 *gb0,
                             const float *gb1, float *recgrad, hipStream_t s);

// ---- loss.hip ----
int loss_blocks(int64_t n_rays);
hipError_t launch_loss(int64_t n_rays, const float *depth, const float *normal, const float *td, const float *tn,
                       float w_depth, float lambda_n, float lambda_ng, float *partials, float *loss_out,
                       float *gD, float *gA, float *gN, hipStream_t s);

// ---- chain.hip ----
int chain_blocks(int64_t n);
hipError_t launch_chain(const SurfelPtrs &S, const float *pose_dev, const RasterParams &p, const float *recgrad,
                        float *d_means, float *d_quats, float *d_log_scales, float *d_logits, float *pose_partials,
                        float *grad_pose, hipStream_t s);

}  // namespace lgsr
