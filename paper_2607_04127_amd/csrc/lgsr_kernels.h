// lgsr_kernels.h -- host-side launchers of the renderer's kernels (internal interface
// between the C-ABI layer and the kernel files).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lgsr_internal.h"

namespace lgsr {

// ---- sort.hip ----
// Lists longer than this are sorted in chunks of this size and merged.
int tile_sort_capacity();
// Chunks of a list of `longest` entries.
int tile_sort_chunks(int64_t longest);
// cnt, cursor: T x kShards.  ranges[t] = [first, end) of tile t's list and cursor[t kShards
// + s] = first slot of its shard s, from the exclusive prefix sum of cnt in (tile, shard)
// order; cnt is left zero; out (device, 4 words) receives the total as two 32-bit words (low, high), the
// largest tile count and the number of tiles longer than tile_sort_capacity(), whose ids go
// to long_tiles (T words).  host_out, when not null, is the device address of 4 words of
// host memory that receive the same words.
hipError_t launch_tile_scan(uint32_t *cnt, int T, uint2 *ranges, uint32_t *cursor, uint32_t *out,
                            uint32_t *long_tiles, uint32_t *host_out, hipStream_t s);
// Puts the cursors of launch_tile_scan back after an emission advanced them.
hipError_t launch_restore_cursors(const uint2 *ranges, int T, uint32_t *cursor, hipStream_t s);
// The raster's chunk list, built alongside the tile sort: chunks of seg list entries
// (items_max x uint4), chunk_base (T + 1), n_items (device word).
struct ChunkList {
    int seg;
    uint4 *chunks;
    uint32_t *chunk_base;
    uint32_t *n_items;
    int64_t cap_items;  // chunks the buffer holds
};
// Orders every tile's list ids[ranges[t].x .. ranges[t].y) by (keys[id], id) ascending
// (keys has n entries) and builds the chunk list.  Lists longer than tile_sort_capacity()
// are left to launch_tile_sort_long; lists reaching past cap_pairs (the ids buffer) are
// skipped; sort_lists = false builds the chunk list only.
hipError_t launch_tile_sort(const uint2 *ranges, int T, const uint32_t *keys, int64_t n, uint32_t *ids,
                            int64_t cap_pairs, bool sort_lists, const ChunkList &cl, hipStream_t s);
// The lists longer than tile_sort_capacity(): the n_long of them in long_tiles,
// nch = tile_sort_chunks(longest), tmp (P x 8 bytes).
hipError_t launch_tile_sort_long(const uint2 *ranges, const uint32_t *keys, int64_t n, uint32_t *ids,
                                 const uint32_t *long_tiles, int n_long, int nch, unsigned long long *tmp,
                                 hipStream_t s);

// ---- project.hip ----
struct SurfelPtrs {
    const float *means, *quats, *log_scales, *logits;
    int64_t n;
};

// Workgroups of the projection and of the emission for n surfels on a device of n_cu compute
// units: one per CU at most (workgroup b takes surfels [b n / B, (b + 1) n / B)); both
// launches of one frame must use the same count.
int surfel_blocks(int64_t n, int n_cu);
// records, range keys (float bits of the sensor range), ray rectangles, and per-(tile,
// shard) pair counts added to tile_cnt (T x kShards, zero it first)
hipError_t launch_project(const SurfelPtrs &S, const Pose &pose_val, const float *pose_dev, float *pose_out,
                          const float *rows, const Grid &g, const RasterParams &p, float *recs, uint2 *rects,
                          uint32_t *keys, uint32_t *tile_cnt, int blocks, hipStream_t s);
// surfel ids into the tile lists; cursor (T x kShards) from launch_tile_scan, pv holds P words
hipError_t launch_emit(const uint2 *rects, int64_t n, const Grid &g, uint32_t *cursor, uint32_t *pv, int64_t P,
                       int blocks, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_count_visible(const uint2 *rects, int64_t n, uint32_t *out, hipStream_t s);
hipError_t launch_max_range(const uint2 *ranges, int T, uint32_t *out, hipStream_t s);
// out[0] ray-surfel tests, out[1] composited hits, out[2] rays with a hit (u64; out[0..3] zeroed here)
hipError_t launch_work_counts(const uint2 *ranges, const uint32_t *ids, const uint2 *rects, int64_t P,
                              const float4 *st1, const Grid &g, unsigned long long *out, hipStream_t s);

// ---- raster.hip ----
// Most chunks one tile's list is cut into (the merge keeps a 64-bit set of chunks per ray).
constexpr int kTileChunks = 64;
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
    float4 *fixA, *fixB;   // per ray: the merge's fix-up record; after the fix-up, the
                           // sums of the chunk it re-walked (fixB.w: that chunk, or -1)
    uint32_t *fixflag;     // 4 x items_max, per (chunk, sub-tile): nonzero when a ray's fix-up
                           // falls there; zero between forwards (the fix-up clears what the
                           // merge set)
    uint64_t *kmask;       // 4 x items_max, per (chunk, sub-tile): the lanes whose ray has a
                           // composite in the chunk (written by the forward chunk tasks)
    int seg;
    int64_t items_max;
};
// One request of a batched forward raster: its buffers, grid and outputs; block0 and tile0
// (its first block in the chunk-task launches and in the merge launch) are filled by the
// launcher.
struct FwdJob {
    RasterBufs R;
    Grid g;
    float *depth, *opacity, *normal;
    uint8_t *drop;
    uint32_t block0, tile0;
};
constexpr int kMaxFwdJobs = 16;
struct FwdJobs {
    FwdJob j[kMaxFwdJobs];
    int n;
};
static_assert(sizeof(FwdJobs) <= 4096, "the job table travels as a kernel argument");
// The forward raster (chunks, merge, fix-up) of up to kMaxFwdJobs requests, one launch per
// stage for all of them.
hipError_t launch_raster_fwd_multi(FwdJobs &J, const RasterParams &p, hipStream_t s);
int chunk_size(int64_t P, int requested);
int64_t chunk_items_max(int64_t P, int T, int seg);
size_t chunk_slot_floats(int64_t items_max);
hipError_t launch_raster_fwd(const RasterBufs &R, const Grid &g, const RasterParams &p, float *depth,
                             float *opacity, float *normal, uint8_t *drop, hipStream_t s);
// out (u64, device) += ray tests needed up to each wave's last contributor (query only)
hipError_t launch_work_needed(const RasterBufs &R, const Grid &g, const RasterParams &p, unsigned long long *out,
                              hipStream_t s);
// out[0] (u64) = list entries passing every per-hit test summed over rays, ignoring early
// termination; out[1] = rays with at least one (query only)
hipError_t launch_count_hits(const RasterBufs &R, const Grid &g, const RasterParams &p, unsigned long long *out,
                             hipStream_t s);
// record gradients += the backward of the raster for per-ray upstream gradients gD, gA (per
// ray) and gN (3 per ray)
hipError_t launch_raster_bwd(const RasterBufs &R, const Grid &g, const RasterParams &p, const float *gD,
                             const float *gA, const float *gN, float *recgrad, hipStream_t s);

// ---- loss.hip ----
int loss_blocks(int64_t n_rays);
hipError_t launch_loss(int64_t n_rays, const float *depth, const float *normal, const float *td, const float *tn,
                       float w_depth, float lambda_n, float lambda_ng, float *partials, float *loss_out,
                       float *gD, float *gA, float *gN, hipStream_t s);

// ---- objective.hip ----
struct ObjectiveWeights {
    float w_depth, lambda_alpha, eps, lambda_n, lambda_ng, lambda_ns;
};
int objective_partial_floats(int64_t n_rays);
hipError_t launch_objective(int H, int W, const float *rows, const float *cols, const float *depth,
                            const float *opacity, const float *normal, const float *td, const float *tn,
                            const ObjectiveWeights &w, float *partials, float *loss_out, float *gD, float *gA,
                            float *gN, hipStream_t s);
int scale_reg_blocks(int64_t n);
hipError_t launch_scale_reg(int64_t n, const float *log_scales, float lambda_s, float s_max, float *partials,
                            float *loss_out, float *grad_log_scales, hipStream_t s);

// ---- scan.hip ----
struct ScanGridF {
    int H, W;
    float el_max, rows_per_rad, cols_per_rad, r_min, r_max;
};
hipError_t launch_scan_to_range(int64_t n, const float *pts, const float *nrm, const ScanGridF &g,
                                unsigned long long *slots, float *depth, float *normal, int32_t *index, hipStream_t s);
hipError_t launch_target_cov(int64_t n, const float *quats, const float *log_scales, float eps, float *cov,
                             hipStream_t s);

// ---- chain.hip ----
int chain_blocks(int64_t n);
// reads the record-gradient slots of surfels with a non-empty ray rectangle and clears them
hipError_t launch_chain(const SurfelPtrs &S, const float *pose_dev, const RasterParams &p, const uint2 *rects,
                        float *recgrad,
                        float *d_means, float *d_quats, float *d_log_scales, float *d_logits, float *pose_partials,
                        float *grad_pose, hipStream_t s);

// ---- adam.hip ----
struct AdamGroup {
    int64_t n;
    float *param;
    const float *grad;
    float *m, *v;
    float lr;
};
struct AdamBatch {
    AdamGroup g[8];
    int64_t first_block[8];  // filled by launch_adam
    int count;
};
hipError_t launch_adam(AdamBatch B, float beta1, float beta2, float eps, int step, hipStream_t s);

// ---- probe.hip ----
// kind 0 copy a = b (non-temporal, 4 vectors per lane), 1 triad a = b + 3 c (same), 2 copy
// and 3 triad with plain loads and stores, one vector per lane; blocks <= 0: 4096
hipError_t launch_stream_probe(int kind, const float *b, const float *c, float *a, int64_t n, int blocks,
                               hipStream_t s);

}  // namespace lgsr
