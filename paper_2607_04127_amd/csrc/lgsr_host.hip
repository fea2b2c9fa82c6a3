// lgsr_host.hip -- the C ABI of include/lgsr.h: argument validation, contexts, pooled
// states and the ordering of the stages on HIP streams.
//
// Forward stages (on the context's stream, or on a lane stream within a batch):
//   project      per-surfel record, conservative ray rectangle, range key, per-tile counts
//   scan         tile counts -> [start, end) of every tile's list, total P, longest list
//   (P and the longest list are read back once to size the pair buffers)
//   emit         surfel ids into their tiles' lists (unordered)
//   tile_sort    every list by (range, index), one workgroup per tile
//   raster_fwd   compositing, frame outputs and per-ray backward state
// Backward: zero record gradients, raster_bwd, chain (parameters + pose).
// A forward is split in two: begin (everything up to the read-back of the pair count) and
// end (the rest).  A batch runs every request's begin first, spread over kLanes streams,
// then waits once per request for its count and issues the ends (with loss and backward
// for gradient requests) on the same lanes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lgsr.h"
#include "lgsr_internal.h"
#include "lgsr_kernels.h"

using namespace lgsr;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

hipError_t ensure(DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (bytes <= b.cap) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (e != hipSuccess) return e;
    }
    size_t want = bytes + bytes / 4;
    want = (want + 4095) & ~(size_t)4095;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return e;
    }
    b.cap = want;
    return hipSuccess;
}

void release(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

template <class T>
T *as(DevBuf &b)
{
    return static_cast<T *>(b.p);
}

}  // namespace

struct lgsr_state {
    lgsr_ctx *ctx = nullptr;
    bool live = false;
    // forward products kept for the backward
    DevBuf recs, rects, pk, pv, ranges, long_tiles, st0, st1, pose, chunks, chunk_base, slots, fixA, fixB, fixflag,
        kmask;
    bool fixflag_clean = false;  // every word of fixflag is zero (the fix-up clears what the merge sets)
    void *fixflag_seen = nullptr;
    // per-forward scratch: range keys, per-(tile, shard) counts and cursors, read-back words
    DevBuf keys, cnt, offs, counters;
    bool cnt_clean = false;      // every word of cnt is zero (the tile scan leaves it so)
    void *cnt_seen = nullptr;    // the cnt allocation cnt_clean refers to
    uint32_t *pinned = nullptr;      // host copy of counters[0..3], written by the tile scan
    uint32_t *pinned_dev = nullptr;  // its device address
    hipEvent_t rb = nullptr;         // recorded after the tile scan
    // lists emitted and sorted ahead of the read-back, on buffers sized from earlier frames
    bool spec = false;
    int spec_seg = 0;
    int64_t spec_cap_pairs = 0, spec_cap_items = 0;
    int64_t last_P = -1;  // pairs of this state's previous forward
    int chunk_req = 0;           // requested chunk size (0: automatic)
    uint32_t *ids = nullptr;  // per-tile lists of surfel ids, front to back (pv)
    SurfelPtrs S{};
    const float *rows = nullptr, *cols = nullptr;
    Grid g{};
    RasterParams prm{};
    RasterBufs R{};
    int64_t P = 0;
};

// A stream with the scratch of the loss and the backward; calls on one lane run in order.
struct Lane {
    hipStream_t stream = nullptr;  // lane 0: the context's stream
    bool own = false;              // created by the context (lanes 1..)
    DevBuf recgrad, partials, pose_partials;
    bool recgrad_zero = false;  // every record-gradient slot is zero (the chain clears what it reads)
    hipEvent_t done = nullptr;  // joins a batch back into the context's stream
    std::vector<lgsr_state *> batch_states;  // per-request states of batches on this lane
};

constexpr int kLanes = 4;

struct lgsr_ctx {
    int device = 0;
    int n_cu = 1;  // compute units of the device: projection and emission run one workgroup per CU at most
    hipStream_t stream = nullptr;
    std::string err;
    Lane lanes[kLanes];
    hipEvent_t batch_start = nullptr;
    std::vector<hipEvent_t> req_done;  // per request of the latest batch: recorded after its last kernel
    int32_t batch_n = 0;               // requests of the latest batch
    DevBuf counters;             // lgsr_query's counters
    DevBuf scan_slots;           // lgsr_scan_to_range's per-pixel keys
    uint32_t *pinned = nullptr;  // host-pinned read-back of lgsr_query
    std::vector<lgsr_state *> pool;  // freed states kept for reuse
    std::vector<lgsr_state *> all;   // every state allocated by this context
    lgsr_state scratch_state;        // used when the caller asks for no state
    int live_states = 0;
    // stage timers
    uint32_t prof_mask = 0;  // bit k: time stage k
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    double prof_ms[LGSR_NUM_STAGES] = {};
    int64_t prof_calls[LGSR_NUM_STAGES] = {};
};

namespace {

lgsr_status fail(lgsr_ctx *ctx, lgsr_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

lgsr_status hip_fail(lgsr_ctx *ctx, hipError_t e, const char *where)
{
    lgsr_status st = (e == hipErrorOutOfMemory) ? LGSR_ENOMEM : LGSR_EDEVICE;
    return fail(ctx, st, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(expr, where)                                   \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
    } while (0)

bool finite_pos(float x) { return std::isfinite(x) && x > 0.f; }

lgsr_status check_opts(lgsr_ctx *ctx, const lgsr_raster_opts *o)
{
    if (!o) return fail(ctx, LGSR_EINVAL, "opts is NULL");
    if (!finite_pos(o->cutoff_sigma)) return fail(ctx, LGSR_EINVAL, "cutoff_sigma must be finite and > 0");
    if (!finite_pos(o->alpha_thr) || !finite_pos(o->alpha_max) || o->alpha_max >= 1.f || o->alpha_thr > o->alpha_max)
        return fail(ctx, LGSR_EINVAL, "need 0 < alpha_thr <= alpha_max < 1");
    if (!std::isfinite(o->T_min) || o->T_min < 0.f || o->T_min >= 1.f)
        return fail(ctx, LGSR_EINVAL, "T_min must lie in [0, 1)");
    if (!finite_pos(o->near)) return fail(ctx, LGSR_EINVAL, "near must be finite and > 0");
    if (!std::isfinite(o->den_eps) || o->den_eps < 0.f) return fail(ctx, LGSR_EINVAL, "den_eps must be >= 0");
    if (!std::isfinite(o->drop_tau)) return fail(ctx, LGSR_EINVAL, "drop_tau must be finite");
    if (o->chunk != 0 && (o->chunk < 16 || o->chunk > 65536))
        return fail(ctx, LGSR_EINVAL, "chunk must be 0 or lie in [16, 65536]");
    if ((o->flags & ~LGSR_FLAG_BATCH_FUSED) != 0) return fail(ctx, LGSR_EINVAL, "unknown flags");
    return LGSR_OK;
}

RasterParams to_params(const lgsr_raster_opts *o)
{
    RasterParams p;
    p.cutoff = o->cutoff_sigma;
    p.k2 = o->cutoff_sigma * o->cutoff_sigma;
    p.alpha_thr = o->alpha_thr;
    p.alpha_max = o->alpha_max;
    p.T_min = o->T_min;
    p.near = o->near;
    p.den_eps = o->den_eps;
    p.drop_tau = o->drop_tau;
    return p;
}

lgsr_state *take_state(lgsr_ctx *ctx)
{
    if (!ctx->pool.empty()) {
        lgsr_state *s = ctx->pool.back();
        ctx->pool.pop_back();
        return s;
    }
    lgsr_state *s = new (std::nothrow) lgsr_state;
    if (s) {
        s->ctx = ctx;
        ctx->all.push_back(s);
    }
    return s;
}

void free_state_buffers(lgsr_state *s)
{
    release(s->recs); release(s->rects); release(s->pk); release(s->pv); release(s->long_tiles);
    release(s->ranges); release(s->st0); release(s->st1); release(s->pose);
    release(s->chunks); release(s->chunk_base); release(s->slots); release(s->fixA); release(s->fixB);
    release(s->fixflag);
    release(s->kmask);
    release(s->keys); release(s->cnt); release(s->offs); release(s->counters);
    if (s->pinned) (void)hipHostFree(s->pinned);
    s->pinned = nullptr;
    if (s->rb) (void)hipEventDestroy(s->rb);
    s->rb = nullptr;
}

void free_lane(Lane &L)
{
    release(L.recgrad); release(L.partials); release(L.pose_partials);
    if (L.done) (void)hipEventDestroy(L.done);
    L.done = nullptr;
    if (L.own && L.stream) (void)hipStreamDestroy(L.stream);
    L.stream = nullptr;
    L.own = false;
}

hipEvent_t take_event(lgsr_ctx *ctx)
{
    if (!ctx->ev_free.empty()) {
        hipEvent_t e = ctx->ev_free.back();
        ctx->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Brackets one stage with events on a stream while profiling is on.
struct Stage {
    lgsr_ctx *ctx;
    int id;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Stage(lgsr_ctx *c, int stage, hipStream_t stream) : ctx(c), id(stage), s(stream)
    {
        if (!((ctx->prof_mask >> id) & 1u)) return;
        a = take_event(ctx);
        if (a) (void)hipEventRecord(a, s);
    }
    ~Stage()
    {
        if (!a) return;
        hipEvent_t b = take_event(ctx);
        if (!b) {
            ctx->ev_free.push_back(a);
            return;
        }
        (void)hipEventRecord(b, s);
        ctx->ev_pending.push_back({id, {a, b}});
    }
};

size_t state_bytes(const lgsr_state *s)
{
    return s->recs.cap + s->rects.cap + s->pk.cap + s->pv.cap + s->long_tiles.cap + s->ranges.cap +
           s->st0.cap + s->st1.cap + s->pose.cap + s->chunks.cap + s->chunk_base.cap + s->slots.cap + s->fixA.cap +
           s->fixB.cap + s->fixflag.cap + s->kmask.cap + s->keys.cap + s->cnt.cap + s->offs.cap + s->counters.cap;
}

size_t ctx_bytes(const lgsr_ctx *c)
{
    size_t b = c->counters.cap + c->scan_slots.cap + state_bytes(&c->scratch_state);
    for (const Lane &L : c->lanes) {
        b += L.recgrad.cap + L.partials.cap + L.pose_partials.cap;
        for (const lgsr_state *st : L.batch_states) b += state_bytes(st);
    }
    return b;
}

// ---- validation shared by the single-request and batch entry points ----

lgsr_status check_surfels(lgsr_ctx *ctx, const lgsr_surfels *surfels)
{
    if (!surfels) return fail(ctx, LGSR_EINVAL, "surfels is NULL");
    const int64_t n = surfels->n;
    if (n < 0 || n > (int64_t)0x7FFFFFFF) return fail(ctx, LGSR_EINVAL, "surfel count %lld out of range", (long long)n);
    if (n > 0 && (!surfels->means || !surfels->quats || !surfels->log_scales || !surfels->opacity_logits))
        return fail(ctx, LGSR_EINVAL, "surfel arrays must not be NULL");
    return LGSR_OK;
}

lgsr_status check_beams(lgsr_ctx *ctx, const lgsr_beams *beams)
{
    if (!beams) return fail(ctx, LGSR_EINVAL, "beams is NULL");
    if (beams->H < 1 || beams->W < 1 || beams->H > 32768 || beams->W > 32768)
        return fail(ctx, LGSR_EINVAL, "beam grid %d x %d out of range [1, 32768]", beams->H, beams->W);
    if (!beams->row_sincos || !beams->col_sincos) return fail(ctx, LGSR_EINVAL, "beam tables must not be NULL");
    return LGSR_OK;
}

lgsr_status check_frame(lgsr_ctx *ctx, const lgsr_frame *out)
{
    if (!out || !out->depth || !out->opacity || !out->normal || !out->drop)
        return fail(ctx, LGSR_EINVAL, "frame outputs must not be NULL");
    return LGSR_OK;
}

lgsr_status host_pose(lgsr_ctx *ctx, const float *pose_ws, Pose &P)
{
    for (int c = 0; c < 12; ++c)
        if (!std::isfinite(pose_ws[c])) return fail(ctx, LGSR_EINVAL, "pose has a non-finite entry");
    for (int c = 0; c < 9; ++c) P.r[c] = pose_ws[(c / 3) * 4 + (c % 3)];
    for (int c = 0; c < 3; ++c) P.t[c] = pose_ws[4 * c + 3];
    return LGSR_OK;
}

lgsr_status check_weights(lgsr_ctx *ctx, const lgsr_loss_weights *w)
{
    if (!w) return fail(ctx, LGSR_EINVAL, "weights is NULL");
    if (!std::isfinite(w->w_depth) || !std::isfinite(w->lambda_n) || !std::isfinite(w->lambda_ng))
        return fail(ctx, LGSR_EINVAL, "weights must be finite");
    return LGSR_OK;
}

lgsr_status check_surfel_grads(lgsr_ctx *ctx, int64_t n, const lgsr_surfel_grads *out, const float *grad_pose)
{
    if (!out || (n > 0 && (!out->means || !out->quats || !out->log_scales || !out->opacity_logits)))
        return fail(ctx, LGSR_EINVAL, "surfel gradient outputs are NULL");
    if (!grad_pose) return fail(ctx, LGSR_EINVAL, "grad_pose is NULL");
    return LGSR_OK;
}

// ---- forward, loss and backward on a given stream / lane ----

// Forward, first half: records, rectangles, counts, tile offsets and the asynchronous
// read-back of (P, longest list), after which S->rb is recorded.  pose_dev (device 3 x 4)
// replaces pose_val when not null.
lgsr_status forward_begin(lgsr_ctx *ctx, lgsr_state *S, const lgsr_surfels *surfels, const Pose &pose_val,
                          const float *pose_dev, const lgsr_beams *beams, const lgsr_raster_opts *opts,
                          hipStream_t s)
{
    const int64_t n = surfels->n;
    Grid g;
    g.H = beams->H;
    g.W = beams->W;
    g.TH = (g.H + kTile - 1) / kTile;
    g.TW = (g.W + kTile - 1) / kTile;
    g.T = g.TH * g.TW;
    const int64_t rays = (int64_t)g.H * g.W;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    S->g = g;
    S->prm = to_params(opts);
    S->chunk_req = opts->chunk;
    S->S = SurfelPtrs{surfels->means, surfels->quats, surfels->log_scales, surfels->opacity_logits, n};
    S->rows = beams->row_sincos;
    S->cols = beams->col_sincos;
    S->P = 0;
    HIP_TRY(ensure(S->recs, nn * kRec * sizeof(float)), "alloc records");
    HIP_TRY(ensure(S->rects, nn * sizeof(uint2)), "alloc rects");
    HIP_TRY(ensure(S->ranges, (size_t)g.T * sizeof(uint2)), "alloc ranges");
    HIP_TRY(ensure(S->st0, (size_t)rays * sizeof(float4)), "alloc ray state");
    HIP_TRY(ensure(S->st1, (size_t)rays * sizeof(float4)), "alloc ray state");
    HIP_TRY(ensure(S->pose, 16 * sizeof(float)), "alloc pose");
    HIP_TRY(ensure(S->keys, nn * 4), "alloc keys");
    HIP_TRY(ensure(S->cnt, (size_t)g.T * kShards * 4), "alloc tile counts");
    HIP_TRY(ensure(S->offs, (size_t)g.T * kShards * 4), "alloc tile cursors");
    HIP_TRY(ensure(S->long_tiles, (size_t)g.T * 4), "alloc long tile list");
    HIP_TRY(ensure(S->counters, 16), "alloc counters");
    if (!S->pinned) {
        HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&S->pinned), 16, hipHostMallocCoherent), "pinned");
        HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void **>(&S->pinned_dev), S->pinned, 0), "pinned");
    }
    if (!S->rb) HIP_TRY(hipEventCreateWithFlags(&S->rb, hipEventDisableTiming), "event");
    uint32_t *counters = as<uint32_t>(S->counters);
    {
    Stage st_(ctx, LGSR_STAGE_PROJECT, s);
    if (!(S->cnt_clean && S->cnt_seen == S->cnt.p))
        HIP_TRY(launch_fill_u32(as<uint32_t>(S->cnt), 0u, (int64_t)(S->cnt.cap / 4), s), "clear tile counts");
    S->cnt_clean = false;  // until the scan below has run
    HIP_TRY(launch_project(S->S, pose_val, pose_dev, as<float>(S->pose), beams->row_sincos, g, S->prm,
                           as<float>(S->recs), as<uint2>(S->rects), as<uint32_t>(S->keys), as<uint32_t>(S->cnt),
                           surfel_blocks(S->S.n, ctx->n_cu), s),
            "project");
    }
    {
    Stage st_(ctx, LGSR_STAGE_SCAN, s);
    // a value the scan cannot write (P would be 2^64 - 1): seen after the wait, the words did
    // not arrive and forward_end copies them from the device instead
    for (int k = 0; k < 4; ++k) S->pinned[k] = 0xFFFFFFFFu;
    HIP_TRY(launch_tile_scan(as<uint32_t>(S->cnt), g.T, as<uint2>(S->ranges), as<uint32_t>(S->offs), counters,
                             as<uint32_t>(S->long_tiles), S->pinned_dev, s),
            "tile scan");
    S->cnt_clean = true;
    S->cnt_seen = S->cnt.p;
    HIP_TRY(hipEventRecord(S->rb, s), "readback event");
    }
    // Emission and the per-tile sorts go out before the host waits for the pair count, on
    // buffers sized from this state's previous frame with a margin; forward_end checks the
    // count and redoes them when a buffer was short or the chunk length differs.
    S->spec = false;
    S->ids = as<uint32_t>(S->pv);
    if (S->last_P >= 0 && g.T > 0) {
        const int64_t want = S->last_P + S->last_P / 4 + 4096;
        const int seg = chunk_size(S->last_P, S->chunk_req);
        const int64_t items = chunk_items_max(want, g.T, seg);
        if (want <= (int64_t)0x7FFFFFFF && items <= (int64_t)0x7FFFFFFF) {
            HIP_TRY(ensure(S->pv, (size_t)want * 4), "alloc pairs");
            HIP_TRY(ensure(S->chunks, (size_t)items * sizeof(uint4)), "alloc chunks");
            HIP_TRY(ensure(S->chunk_base, (size_t)(g.T + 1) * sizeof(uint32_t)), "alloc chunks");
            S->ids = as<uint32_t>(S->pv);
            S->spec_cap_pairs = (int64_t)(S->pv.cap / 4);
            S->spec_cap_items = (int64_t)(S->chunks.cap / sizeof(uint4));
            S->spec_seg = seg;
            {
            Stage st_(ctx, LGSR_STAGE_EMIT, s);
            HIP_TRY(launch_emit(as<uint2>(S->rects), n, g, as<uint32_t>(S->offs), S->ids, S->spec_cap_pairs,
                                surfel_blocks(n, ctx->n_cu), s),
                    "emit");
            }
            Stage st_(ctx, LGSR_STAGE_TILE_SORT, s);
            const ChunkList cl{seg, as<uint4>(S->chunks), as<uint32_t>(S->chunk_base), as<uint32_t>(S->pose) + 12,
                               S->spec_cap_items};
            HIP_TRY(launch_tile_sort(as<uint2>(S->ranges), g.T, as<uint32_t>(S->keys), n, S->ids, S->spec_cap_pairs,
                                     true, cl, s),
                    "tile sort");
            S->spec = true;
        }
    }
    return LGSR_OK;
}

// Forward, second half, up to the compositing: waits for the read-back, then emission,
// per-tile order and the chunk list; S->R then describes the raster buffers.
lgsr_status forward_lists(lgsr_ctx *ctx, lgsr_state *S, hipStream_t s)
{
    {
    Stage st_(ctx, LGSR_STAGE_READBACK, s);
    HIP_TRY(hipEventSynchronize(S->rb), "readback wait");
    if (S->pinned[0] == 0xFFFFFFFFu && S->pinned[1] == 0xFFFFFFFFu)
        HIP_TRY(hipMemcpy(S->pinned, S->counters.p, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost), "readback");
    }
    const int64_t P = (int64_t)((uint64_t)S->pinned[0] | ((uint64_t)S->pinned[1] << 32));
    const int64_t longest = (int64_t)S->pinned[2];
    const Grid g = S->g;
    const int64_t n = S->S.n;
    const int64_t rays = (int64_t)g.H * g.W;
    // lists are addressed with 32-bit offsets
    if (P > (int64_t)0x7FFFFFFF) return fail(ctx, LGSR_ECAPACITY, "too many (surfel, tile) pairs");
    const size_t pp = (size_t)(P > 0 ? P : 1);
    const int n_long = (int)S->pinned[3];
    const int nch = tile_sort_chunks(longest);
    if (n_long > 0) {
        if ((int64_t)n_long * nch > (int64_t)0x7FFFFFFF) return fail(ctx, LGSR_ECAPACITY, "tile lists too long");
        HIP_TRY(ensure(S->pk, pp * 8), "alloc sort workspace");
    }
    const int seg = chunk_size(P, S->chunk_req);
    const int64_t items_max = chunk_items_max(P, g.T, seg);
    if (items_max > 0x7FFFFFFF) return fail(ctx, LGSR_ECAPACITY, "too many list chunks");
    // the lists emitted ahead hold when their buffers were large enough; the chunk list also
    // needs this frame's chunk length
    const bool lists_ok = S->spec && P <= S->spec_cap_pairs;
    const bool chunks_ok = lists_ok && seg == S->spec_seg && items_max <= S->spec_cap_items;
    HIP_TRY(ensure(S->chunks, (size_t)(items_max > 0 ? items_max : 1) * sizeof(uint4)), "alloc chunks");
    HIP_TRY(ensure(S->chunk_base, (size_t)(g.T + 1) * sizeof(uint32_t)), "alloc chunks");
    HIP_TRY(ensure(S->slots, chunk_slot_floats(items_max > 0 ? items_max : 1) * sizeof(float)), "alloc slots");
    HIP_TRY(ensure(S->fixA, (size_t)rays * sizeof(float4)), "alloc ray state");
    HIP_TRY(ensure(S->fixB, (size_t)rays * sizeof(float4)), "alloc ray state");
    HIP_TRY(ensure(S->fixflag, (size_t)(items_max > 0 ? 4 * items_max : 1) * sizeof(uint32_t)), "alloc chunk flags");
    HIP_TRY(ensure(S->kmask, (size_t)(items_max > 0 ? 4 * items_max : 1) * sizeof(uint64_t)), "alloc chunk masks");
    if (!(S->fixflag_clean && S->fixflag_seen == S->fixflag.p))
        HIP_TRY(launch_fill_u32(as<uint32_t>(S->fixflag), 0u, (int64_t)(S->fixflag.cap / 4), s), "clear chunk flags");
    S->fixflag_clean = false;  // until the raster below has run
    const ChunkList cl{seg, as<uint4>(S->chunks), as<uint32_t>(S->chunk_base), as<uint32_t>(S->pose) + 12,
                       (int64_t)(S->chunks.cap / sizeof(uint4))};
    if (!lists_ok) {
        HIP_TRY(ensure(S->pv, pp * 4), "alloc pairs");
        S->ids = as<uint32_t>(S->pv);
        if (S->spec) HIP_TRY(launch_restore_cursors(as<uint2>(S->ranges), g.T, as<uint32_t>(S->offs), s), "emit");
        if (P > 0) {
            Stage st_(ctx, LGSR_STAGE_EMIT, s);
            HIP_TRY(launch_emit(as<uint2>(S->rects), n, g, as<uint32_t>(S->offs), S->ids, P, surfel_blocks(n, ctx->n_cu),
                                s),
                    "emit");
        }
        Stage st_(ctx, LGSR_STAGE_TILE_SORT, s);
        HIP_TRY(launch_tile_sort(as<uint2>(S->ranges), g.T, as<uint32_t>(S->keys), n, S->ids, P, true, cl, s),
                "tile sort");
    } else if (!chunks_ok) {
        Stage st_(ctx, LGSR_STAGE_TILE_SORT, s);
        HIP_TRY(launch_tile_sort(as<uint2>(S->ranges), g.T, as<uint32_t>(S->keys), n, S->ids, P, false, cl, s),
                "chunk list");
    }
    if (n_long > 0) {
        Stage st_(ctx, LGSR_STAGE_TILE_SORT, s);
        HIP_TRY(launch_tile_sort_long(as<uint2>(S->ranges), as<uint32_t>(S->keys), n, S->ids,
                                      as<uint32_t>(S->long_tiles), n_long, nch, as<unsigned long long>(S->pk), s),
                "tile sort");
    }
    S->spec = false;
    S->last_P = P;
    RasterBufs &R = S->R;
    R.ids = S->ids;
    R.recs = as<float>(S->recs);
    R.rects = as<uint2>(S->rects);
    R.ranges = as<uint2>(S->ranges);
    R.rows = S->rows;
    R.cols = S->cols;
    R.chunks = as<uint4>(S->chunks);
    R.chunk_base = as<uint32_t>(S->chunk_base);
    R.n_items = as<uint32_t>(S->pose) + 12;
    R.slots = as<float>(S->slots);
    R.st0 = as<float4>(S->st0);
    R.st1 = as<float4>(S->st1);
    R.fixA = as<float4>(S->fixA);
    R.fixB = as<float4>(S->fixB);
    R.fixflag = as<uint32_t>(S->fixflag);
    R.kmask = as<uint64_t>(S->kmask);
    R.seg = seg;
    R.items_max = items_max;
    S->P = P;
    return LGSR_OK;
}

// After the raster forward of S has been issued: the fix-up leaves every chunk flag zero.
void raster_issued(lgsr_state *S)
{
    S->fixflag_clean = true;
    S->fixflag_seen = S->fixflag.p;
}

// Forward, second half: lists (forward_lists), then compositing into `out`.
lgsr_status forward_end(lgsr_ctx *ctx, lgsr_state *S, const lgsr_frame *out, hipStream_t s)
{
    lgsr_status st = forward_lists(ctx, S, s);
    if (st != LGSR_OK) return st;
    Stage st_(ctx, LGSR_STAGE_RASTER_FWD, s);
    HIP_TRY(launch_raster_fwd(S->R, S->g, S->prm, out->depth, out->opacity, out->normal, out->drop, s),
            "raster forward");
    raster_issued(S);
    return LGSR_OK;
}

lgsr_status loss_impl(lgsr_ctx *ctx, Lane &L, int64_t n_rays, const lgsr_frame *pred, const float *target_depth,
                      const float *target_normal, const lgsr_loss_weights *w, float *loss_out,
                      const lgsr_frame_grad *grad_out)
{
    HIP_TRY(ensure(L.partials, (size_t)loss_blocks(n_rays) * 4 * sizeof(float)), "alloc partials");
    Stage st_(ctx, LGSR_STAGE_LOSS, L.stream);
    HIP_TRY(launch_loss(n_rays, pred ? pred->depth : nullptr, pred ? pred->normal : nullptr, target_depth,
                        target_normal, w->w_depth, w->lambda_n, w->lambda_ng, as<float>(L.partials), loss_out,
                        grad_out ? grad_out->d_depth : nullptr, grad_out ? grad_out->d_opacity : nullptr,
                        grad_out ? grad_out->d_normal : nullptr, L.stream),
            "loss");
    return LGSR_OK;
}

lgsr_status backward_impl(lgsr_ctx *ctx, Lane &L, lgsr_state *S, const lgsr_frame_grad *gin,
                          const lgsr_surfel_grads *out, float *grad_pose)
{
    hipStream_t s = L.stream;
    const size_t nn = (size_t)(S->S.n > 0 ? S->S.n : 1);
    if (L.recgrad.cap < nn * kGrad * sizeof(float)) L.recgrad_zero = false;
    HIP_TRY(ensure(L.recgrad, nn * kGrad * sizeof(float)), "alloc record gradients");
    HIP_TRY(ensure(L.pose_partials, (size_t)chain_blocks(S->S.n) * 6 * sizeof(float)), "alloc pose partials");
    {
    // only after a new allocation or a backward that did not finish: the chain clears the
    // slots it reads
    Stage st_(ctx, LGSR_STAGE_BWD_PREP, s);
    if (!L.recgrad_zero)
        HIP_TRY(launch_fill_u32(as<uint32_t>(L.recgrad), 0u, (int64_t)(L.recgrad.cap / sizeof(uint32_t)), s),
                "zero record gradients");
    L.recgrad_zero = false;
    }
    {
    Stage st_(ctx, LGSR_STAGE_RASTER_BWD, s);
    HIP_TRY(launch_raster_bwd(S->R, S->g, S->prm, gin->d_depth, gin->d_opacity, gin->d_normal,
                              as<float>(L.recgrad), s),
            "raster backward");
    }
    Stage st_(ctx, LGSR_STAGE_CHAIN, s);
    HIP_TRY(launch_chain(S->S, as<float>(S->pose), S->prm, as<uint2>(S->rects), as<float>(L.recgrad), out->means,
                         out->quats, out->log_scales, out->opacity_logits, as<float>(L.pose_partials), grad_pose, s),
            "chain");
    L.recgrad_zero = true;
    return LGSR_OK;
}

}  // namespace

extern "C" {

void lgsr_default_opts(lgsr_raster_opts *o)
{
    if (!o) return;
    o->cutoff_sigma = 3.f;
    o->alpha_thr = 1.f / 255.f;
    o->alpha_max = 0.99f;
    o->T_min = 1e-4f;
    o->near = 0.2f;
    o->den_eps = 1e-6f;
    o->drop_tau = 0.5f;
    o->chunk = 0;
    o->flags = 0;
}

void lgsr_default_loss_weights(lgsr_loss_weights *w)
{
    if (!w) return;
    w->w_depth = 1.f;
    w->lambda_n = 1.f;
    w->lambda_ng = 0.05f;
}

// ---- static scratch of lgsr_loss_noalloc ----
// The loss's per-workgroup partial sums (4 floats for each of at most 1024 workgroups) live
// in a file-scope device array, so that lgsr_loss_noalloc allocates nothing.  Every device
// the library runs on holds its own copy until the process ends.  In host code `scratch`
// names a host-side stand-in, not device memory: its device address is taken once per
// device (scratch_setup, from lgsr_create with the device current) and only that address is
// passed to kernels.
constexpr int kNoAllocScratchFloats = 4096;
static __device__ __align__(256) float scratch[kNoAllocScratchFloats];
constexpr int kMaxDevices = 64;
static float *g_scratch_dev[kMaxDevices] = {};
static std::mutex g_scratch_mu;

namespace {

hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = static_cast<float *>(p);
    return hipSuccess;
}

float *scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[device];
}

}  // namespace

lgsr_status lgsr_create(lgsr_ctx **out, int device, void *hip_stream)
{
    if (!out) return LGSR_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return LGSR_EDEVICE;
    }
    if (device < 0 || device >= ndev) return LGSR_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return LGSR_EDEVICE;
    if (scratch_setup(device) != hipSuccess) {
        (void)hipGetLastError();
        return LGSR_EDEVICE;
    }
    lgsr_ctx *ctx = new (std::nothrow) lgsr_ctx;
    if (!ctx) return LGSR_ENOMEM;
    ctx->device = device;
    if (hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        ctx->n_cu < 1) {
        (void)hipGetLastError();
        delete ctx;
        return LGSR_EDEVICE;
    }
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->lanes[0].stream = ctx->stream;
    ctx->scratch_state.ctx = ctx;
    if (hipHostMalloc(reinterpret_cast<void **>(&ctx->pinned), 256, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return LGSR_ENOMEM;
    }
    if (ensure(ctx->counters, 256) != hipSuccess) {
        (void)hipHostFree(ctx->pinned);
        delete ctx;
        return LGSR_ENOMEM;
    }
    *out = ctx;
    return LGSR_OK;
}

void lgsr_destroy(lgsr_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (Lane &L : ctx->lanes)
        if (L.own && L.stream) (void)hipStreamSynchronize(L.stream);
    // every state, freed or not (batch states included): handles of live states become invalid
    for (lgsr_state *s : ctx->all) {
        free_state_buffers(s);
        delete s;
    }
    free_state_buffers(&ctx->scratch_state);
    for (Lane &L : ctx->lanes) free_lane(L);
    release(ctx->counters);
    release(ctx->scan_slots);
    if (ctx->batch_start) (void)hipEventDestroy(ctx->batch_start);
    for (hipEvent_t e : ctx->req_done) (void)hipEventDestroy(e);
    for (auto &pe : ctx->ev_pending) {
        (void)hipEventDestroy(pe.second.first);
        (void)hipEventDestroy(pe.second.second);
    }
    for (hipEvent_t e : ctx->ev_free) (void)hipEventDestroy(e);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

lgsr_status lgsr_set_stream(lgsr_ctx *ctx, void *hip_stream)
{
    if (!ctx) return LGSR_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->lanes[0].stream = ctx->stream;
    return LGSR_OK;
}

const char *lgsr_last_error(const lgsr_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

lgsr_status lgsr_forward(lgsr_ctx *ctx, const lgsr_surfels *surfels, const float *pose_ws, int32_t pose_on_device,
                         const lgsr_beams *beams, const lgsr_raster_opts *opts, lgsr_frame *out,
                         lgsr_state **state)
{
    if (!ctx) return LGSR_EINVAL;
    if (state) *state = nullptr;
    lgsr_status st = check_surfels(ctx, surfels);
    if (st != LGSR_OK) return st;
    if (!pose_ws) return fail(ctx, LGSR_EINVAL, "pose is NULL");
    if ((st = check_beams(ctx, beams)) != LGSR_OK) return st;
    if ((st = check_opts(ctx, opts)) != LGSR_OK) return st;
    if ((st = check_frame(ctx, out)) != LGSR_OK) return st;
    Pose pose_val{};
    if (!pose_on_device && (st = host_pose(ctx, pose_ws, pose_val)) != LGSR_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    lgsr_state *S = state ? take_state(ctx) : &ctx->scratch_state;
    if (!S) return fail(ctx, LGSR_ENOMEM, "out of host memory");
    // on any error below a taken state goes back to the pool
    struct Guard {
        lgsr_ctx *c;
        lgsr_state *s;
        bool keep = false;
        ~Guard()
        {
            if (!keep && s != &c->scratch_state) c->pool.push_back(s);
        }
    } guard{ctx, S};
    st = forward_begin(ctx, S, surfels, pose_val, pose_on_device ? pose_ws : nullptr, beams, opts, ctx->stream);
    if (st != LGSR_OK) return st;
    st = forward_end(ctx, S, out, ctx->stream);
    if (st != LGSR_OK) return st;
    if (state) {
        S->live = true;
        ctx->live_states++;
        guard.keep = true;
        *state = S;
    }
    return LGSR_OK;
}

lgsr_status lgsr_loss(lgsr_ctx *ctx, int64_t n_rays, const lgsr_frame *pred, const float *target_depth,
                      const float *target_normal, const lgsr_loss_weights *w, float *loss_out,
                      lgsr_frame_grad *grad_out)
{
    if (!ctx) return LGSR_EINVAL;
    if (n_rays < 0) return fail(ctx, LGSR_EINVAL, "n_rays must be >= 0");
    lgsr_status st = check_weights(ctx, w);
    if (st != LGSR_OK) return st;
    if (!loss_out) return fail(ctx, LGSR_EINVAL, "loss_out is NULL");
    if (n_rays > 0) {
        if (!pred || !pred->depth || !pred->normal) return fail(ctx, LGSR_EINVAL, "prediction is NULL");
        if (!target_depth || !target_normal) return fail(ctx, LGSR_EINVAL, "targets are NULL");
        if (!grad_out || !grad_out->d_depth || !grad_out->d_opacity || !grad_out->d_normal)
            return fail(ctx, LGSR_EINVAL, "gradient outputs are NULL");
    }
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    return loss_impl(ctx, ctx->lanes[0], n_rays, pred, target_depth, target_normal, w, loss_out, grad_out);
}

lgsr_status lgsr_loss_noalloc(lgsr_ctx *ctx, int64_t n_rays, const lgsr_frame *pred, const float *target_depth,
                              const float *target_normal, const lgsr_loss_weights *w, float *loss_out,
                              lgsr_frame_grad *grad_out)
{
    if (!ctx) return LGSR_EINVAL;
    if (n_rays < 0) return fail(ctx, LGSR_EINVAL, "n_rays must be >= 0");
    lgsr_status st = check_weights(ctx, w);
    if (st != LGSR_OK) return st;
    if (!loss_out) return fail(ctx, LGSR_EINVAL, "loss_out is NULL");
    if (n_rays > 0) {
        if (!pred || !pred->depth || !pred->normal) return fail(ctx, LGSR_EINVAL, "prediction is NULL");
        if (!target_depth || !target_normal) return fail(ctx, LGSR_EINVAL, "targets are NULL");
        if (!grad_out || !grad_out->d_depth || !grad_out->d_opacity || !grad_out->d_normal)
            return fail(ctx, LGSR_EINVAL, "gradient outputs are NULL");
    }
    const int64_t need = (int64_t)loss_blocks(n_rays) * 4;
    if (need > kNoAllocScratchFloats)
        return fail(ctx, LGSR_ECAPACITY, "the loss needs %lld partial sums, the static scratch holds %d",
                    (long long)need, kNoAllocScratchFloats);
    float *part = scratch_of(ctx->device);
    if (!part) return fail(ctx, LGSR_ESTATE, "no static scratch address for device %d", ctx->device);
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(launch_loss(n_rays, pred ? pred->depth : nullptr, pred ? pred->normal : nullptr, target_depth,
                        target_normal, w->w_depth, w->lambda_n, w->lambda_ng, part, loss_out,
                        grad_out ? grad_out->d_depth : nullptr, grad_out ? grad_out->d_opacity : nullptr,
                        grad_out ? grad_out->d_normal : nullptr, ctx->stream),
            "loss");
    return LGSR_OK;
}

void lgsr_default_objective_weights(lgsr_objective_weights *w)
{
    if (!w) return;
    w->w_depth = 1.f;
    w->lambda_alpha = 0.1f;
    w->eps = 1e-6f;
    w->lambda_n = 1.f;
    w->lambda_ng = 0.05f;
    w->lambda_ns = 0.01f;
}

lgsr_status lgsr_objective(lgsr_ctx *ctx, const lgsr_beams *beams, const lgsr_frame *pred,
                           const float *target_depth, const float *target_normal, const lgsr_objective_weights *w,
                           float *loss_out, lgsr_frame_grad *grad_out)
{
    if (!ctx) return LGSR_EINVAL;
    lgsr_status st = check_beams(ctx, beams);
    if (st != LGSR_OK) return st;
    if (!w) return fail(ctx, LGSR_EINVAL, "weights are NULL");
    const float ws[6] = {w->w_depth, w->lambda_alpha, w->eps, w->lambda_n, w->lambda_ng, w->lambda_ns};
    for (float x : ws)
        if (!std::isfinite(x)) return fail(ctx, LGSR_EINVAL, "weights must be finite");
    if (w->eps < 0.f) return fail(ctx, LGSR_EINVAL, "eps must be >= 0");
    if (!loss_out) return fail(ctx, LGSR_EINVAL, "loss_out is NULL");
    const int64_t n_rays = (int64_t)beams->H * beams->W;
    if (n_rays > 0) {
        if (!pred || !pred->depth || !pred->opacity || !pred->normal) return fail(ctx, LGSR_EINVAL, "prediction is NULL");
        if (!target_depth || !target_normal) return fail(ctx, LGSR_EINVAL, "targets are NULL");
        if (grad_out && (!grad_out->d_depth || !grad_out->d_opacity || !grad_out->d_normal))
            return fail(ctx, LGSR_EINVAL, "a gradient output is NULL");
    }
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    Lane &L = ctx->lanes[0];
    HIP_TRY(ensure(L.partials, (size_t)objective_partial_floats(n_rays) * sizeof(float)), "alloc partials");
    const ObjectiveWeights ow{w->w_depth, w->lambda_alpha, w->eps, w->lambda_n, w->lambda_ng, w->lambda_ns};
    Stage st_(ctx, LGSR_STAGE_LOSS, L.stream);
    HIP_TRY(launch_objective(beams->H, beams->W, beams->row_sincos, beams->col_sincos, pred ? pred->depth : nullptr,
                             pred ? pred->opacity : nullptr, pred ? pred->normal : nullptr, target_depth,
                             target_normal, ow, as<float>(L.partials), loss_out,
                             grad_out ? grad_out->d_depth : nullptr, grad_out ? grad_out->d_opacity : nullptr,
                             grad_out ? grad_out->d_normal : nullptr, L.stream),
            "objective");
    return LGSR_OK;
}

lgsr_status lgsr_scale_reg(lgsr_ctx *ctx, int64_t n, const float *log_scales, float lambda_s, float s_max,
                           float *loss_out, float *grad_log_scales)
{
    if (!ctx) return LGSR_EINVAL;
    if (n < 0) return fail(ctx, LGSR_EINVAL, "n must be >= 0");
    if (!loss_out) return fail(ctx, LGSR_EINVAL, "loss_out is NULL");
    if (n > 0 && !log_scales) return fail(ctx, LGSR_EINVAL, "log_scales is NULL");
    if (!std::isfinite(lambda_s) || !(s_max > 0.f) || !std::isfinite(s_max))
        return fail(ctx, LGSR_EINVAL, "lambda_s must be finite and s_max finite and > 0");
    if ((reinterpret_cast<uintptr_t>(log_scales) | reinterpret_cast<uintptr_t>(grad_log_scales)) & 7u)
        return fail(ctx, LGSR_EINVAL, "log_scales and grad_log_scales must be 8-byte aligned");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    Lane &L = ctx->lanes[0];
    HIP_TRY(ensure(L.partials, (size_t)scale_reg_blocks(n) * sizeof(float)), "alloc partials");
    Stage st_(ctx, LGSR_STAGE_LOSS, L.stream);
    HIP_TRY(launch_scale_reg(n, log_scales, lambda_s, s_max, as<float>(L.partials), loss_out, grad_log_scales,
                             L.stream),
            "scale regulariser");
    return LGSR_OK;
}

lgsr_status lgsr_scan_to_range(lgsr_ctx *ctx, int64_t n, const float *points, const float *normals,
                               const lgsr_scan_grid *grid, float *depth, float *normal, int32_t *index)
{
    if (!ctx) return LGSR_EINVAL;
    if (n < 0 || n > (int64_t)0x7FFFFFFF) return fail(ctx, LGSR_EINVAL, "point count %lld out of range", (long long)n);
    if (n > 0 && !points) return fail(ctx, LGSR_EINVAL, "points is NULL");
    if (!grid) return fail(ctx, LGSR_EINVAL, "grid is NULL");
    if (grid->H < 2 || grid->W < 1 || grid->H > 32768 || grid->W > 32768)
        return fail(ctx, LGSR_EINVAL, "grid %d x %d out of range (H in [2, 32768], W in [1, 32768])", grid->H,
                    grid->W);
    if (!std::isfinite(grid->el_min) || !std::isfinite(grid->el_max) || !(grid->el_max > grid->el_min))
        return fail(ctx, LGSR_EINVAL, "need finite el_min < el_max");
    if (!(grid->r_min >= 0.f) || std::isnan(grid->r_max) || !(grid->r_max >= grid->r_min))
        return fail(ctx, LGSR_EINVAL, "need 0 <= r_min <= r_max");
    if (!depth) return fail(ctx, LGSR_EINVAL, "depth is NULL");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    Lane &L = ctx->lanes[0];
    const int64_t P = (int64_t)grid->H * grid->W;
    HIP_TRY(ensure(ctx->scan_slots, (size_t)P * sizeof(unsigned long long)), "alloc scan workspace");
    ScanGridF g;
    g.H = grid->H;
    g.W = grid->W;
    g.el_max = grid->el_max;
    g.rows_per_rad = (float)((double)(grid->H - 1) / ((double)grid->el_max - (double)grid->el_min));
    g.cols_per_rad = (float)((double)grid->W / 6.283185307179586476925286766559);
    g.r_min = grid->r_min;
    g.r_max = grid->r_max;
    HIP_TRY(launch_scan_to_range(n, points, normals, g, as<unsigned long long>(ctx->scan_slots), depth, normal, index,
                                 L.stream),
            "scan to range image");
    return LGSR_OK;
}

lgsr_status lgsr_target_cov(lgsr_ctx *ctx, int64_t n, const float *quats, const float *log_scales, float eps,
                            float *cov)
{
    if (!ctx) return LGSR_EINVAL;
    if (n < 0) return fail(ctx, LGSR_EINVAL, "n must be >= 0");
    if (n > 0 && (!quats || !log_scales || !cov)) return fail(ctx, LGSR_EINVAL, "an array is NULL");
    if (!(eps >= 0.f) || !std::isfinite(eps)) return fail(ctx, LGSR_EINVAL, "eps must be finite and >= 0");
    if ((reinterpret_cast<uintptr_t>(quats) & 15u) || (reinterpret_cast<uintptr_t>(log_scales) & 7u) ||
        (reinterpret_cast<uintptr_t>(cov) & 7u))
        return fail(ctx, LGSR_EINVAL, "quats must be 16-byte, log_scales and cov 8-byte aligned");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(launch_target_cov(n, quats, log_scales, eps, cov, ctx->lanes[0].stream), "target covariance");
    return LGSR_OK;
}

lgsr_status lgsr_backward(lgsr_ctx *ctx, lgsr_state *S, const lgsr_frame_grad *gin, lgsr_surfel_grads *out,
                          float *grad_pose)
{
    if (!ctx) return LGSR_EINVAL;
    if (!S) return fail(ctx, LGSR_EINVAL, "state is NULL");
    if (S->ctx != ctx || !S->live) return fail(ctx, LGSR_ESTATE, "state does not belong to this context");
    if (!gin || !gin->d_depth || !gin->d_opacity || !gin->d_normal)
        return fail(ctx, LGSR_EINVAL, "frame gradients are NULL");
    lgsr_status st = check_surfel_grads(ctx, S->S.n, out, grad_pose);
    if (st != LGSR_OK) return st;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    return backward_impl(ctx, ctx->lanes[0], S, gin, out, grad_pose);
}

lgsr_status lgsr_render_batch(lgsr_ctx *ctx, int32_t n, const lgsr_request *reqs, const lgsr_raster_opts *opts,
                              const lgsr_loss_weights *w)
{
    if (!ctx) return LGSR_EINVAL;
    if (n < 0 || (n > 0 && !reqs)) return fail(ctx, LGSR_EINVAL, "n < 0 or requests is NULL");
    lgsr_status st = check_opts(ctx, opts);
    if (st != LGSR_OK) return st;
    std::vector<Pose> poses((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        const lgsr_request &q = reqs[i];
        if ((st = check_surfels(ctx, &q.surfels)) != LGSR_OK ||
            (st = check_beams(ctx, &q.beams)) != LGSR_OK || (st = check_frame(ctx, &q.out)) != LGSR_OK ||
            (st = host_pose(ctx, q.pose_ws, poses[(size_t)i])) != LGSR_OK) {
            const std::string e = ctx->err;
            return fail(ctx, st, "request %d: %s", i, e.c_str());
        }
        if (q.target_depth || q.target_normal) {
            if (!q.target_depth || !q.target_normal) return fail(ctx, LGSR_EINVAL, "request %d: one target is NULL", i);
            if ((st = check_weights(ctx, w)) != LGSR_OK) return st;
            if (!q.loss_out || !q.frame_grad.d_depth || !q.frame_grad.d_opacity || !q.frame_grad.d_normal)
                return fail(ctx, LGSR_EINVAL, "request %d: loss_out or frame_grad is NULL", i);
            if ((st = check_surfel_grads(ctx, q.surfels.n, &q.grads, q.grad_pose)) != LGSR_OK) {
                const std::string e = ctx->err;
                return fail(ctx, st, "request %d: %s", i, e.c_str());
            }
        }
    }
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    for (int k = 1; k < kLanes; ++k) {
        Lane &L = ctx->lanes[k];
        if (!L.stream) {
            HIP_TRY(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking), "lane stream");
            L.own = true;
        }
    }
    for (Lane &L : ctx->lanes)
        if (!L.done) HIP_TRY(hipEventCreateWithFlags(&L.done, hipEventDisableTiming), "lane event");
    if (!ctx->batch_start) HIP_TRY(hipEventCreateWithFlags(&ctx->batch_start, hipEventDisableTiming), "event");
    while ((int32_t)ctx->req_done.size() < n) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "request event");
        ctx->req_done.push_back(e);
    }
    ctx->batch_n = 0;
    // The lanes start after the work already on the context's stream, and the context's
    // stream continues after the lanes (also when returning early with an error).
    HIP_TRY(hipEventRecord(ctx->batch_start, ctx->stream), "batch start");
    for (int k = 1; k < kLanes; ++k) HIP_TRY(hipStreamWaitEvent(ctx->lanes[k].stream, ctx->batch_start, 0), "join");
    struct Join {
        lgsr_ctx *c;
        uint32_t mask;
        ~Join()
        {
            for (int k = 1; k < kLanes; ++k) {
                Lane &L = c->lanes[k];
                if (hipEventRecord(L.done, L.stream) == hipSuccess) (void)hipStreamWaitEvent(c->stream, L.done, 0);
            }
            c->prof_mask = mask;
        }
    } join{ctx, ctx->prof_mask};
    ctx->prof_mask = 0;  // stage timers describe single calls, not overlapping lanes
    std::vector<lgsr_state *> states((size_t)n);
    int used[kLanes] = {};
    for (int32_t i = 0; i < n; ++i) {
        Lane &L = ctx->lanes[i % kLanes];
        const int r = used[i % kLanes]++;
        if ((int)L.batch_states.size() <= r) {
            lgsr_state *S = new (std::nothrow) lgsr_state;
            if (!S) return fail(ctx, LGSR_ENOMEM, "out of host memory");
            S->ctx = ctx;
            ctx->all.push_back(S);
            L.batch_states.push_back(S);
        }
        states[(size_t)i] = L.batch_states[(size_t)r];
    }
    for (int32_t i = 0; i < n; ++i) {
        const lgsr_request &q = reqs[i];
        st = forward_begin(ctx, states[(size_t)i], &q.surfels, poses[(size_t)i], nullptr, &q.beams, opts,
                           ctx->lanes[i % kLanes].stream);
        if (st != LGSR_OK) return st;
    }
    if (!(opts->flags & LGSR_FLAG_BATCH_FUSED)) {
        // each request's lists, compositing, loss and backward on its lane as soon as its
        // pair count arrives, overlapping with the other lanes and with the host's waits
        for (int32_t i = 0; i < n; ++i) {
            const lgsr_request &q = reqs[i];
            Lane &L = ctx->lanes[i % kLanes];
            lgsr_state *S = states[(size_t)i];
            if ((st = forward_end(ctx, S, &q.out, L.stream)) != LGSR_OK) return st;
            if (q.target_depth) {
                const int64_t rays = (int64_t)q.beams.H * q.beams.W;
                if ((st = loss_impl(ctx, L, rays, &q.out, q.target_depth, q.target_normal, w, q.loss_out,
                                    &q.frame_grad)) != LGSR_OK)
                    return st;
                if ((st = backward_impl(ctx, L, S, &q.frame_grad, &q.grads, q.grad_pose)) != LGSR_OK) return st;
            }
            HIP_TRY(hipEventRecord(ctx->req_done[(size_t)i], L.stream), "request done");
            ctx->batch_n = i + 1;
        }
        return LGSR_OK;
    }
    // LGSR_FLAG_BATCH_FUSED: lists of every request, on its lane, as its pair count arrives
    for (int32_t i = 0; i < n; ++i)
        if ((st = forward_lists(ctx, states[(size_t)i], ctx->lanes[i % kLanes].stream)) != LGSR_OK) return st;
    // the compositing of all requests: one launch per stage (chunks, merge, fix-up) on the
    // context's stream once every lane has its lists
    for (int k = 1; k < kLanes; ++k) {
        HIP_TRY(hipEventRecord(ctx->lanes[k].done, ctx->lanes[k].stream), "lists done");
        HIP_TRY(hipStreamWaitEvent(ctx->stream, ctx->lanes[k].done, 0), "join lists");
    }
    const RasterParams prm = to_params(opts);
    for (int32_t i0 = 0; i0 < n; i0 += kMaxFwdJobs) {
        FwdJobs J{};
        J.n = std::min<int32_t>(kMaxFwdJobs, n - i0);
        for (int k = 0; k < J.n; ++k) {
            const lgsr_request &q = reqs[i0 + k];
            lgsr_state *S = states[(size_t)(i0 + k)];
            J.j[k].R = S->R;
            J.j[k].g = S->g;
            J.j[k].depth = q.out.depth;
            J.j[k].opacity = q.out.opacity;
            J.j[k].normal = q.out.normal;
            J.j[k].drop = q.out.drop;
        }
        HIP_TRY(launch_raster_fwd_multi(J, prm, ctx->stream), "raster forward (batch)");
        for (int k = 0; k < J.n; ++k) raster_issued(states[(size_t)(i0 + k)]);
    }
    HIP_TRY(hipEventRecord(ctx->batch_start, ctx->stream), "frames done");
    for (int k = 1; k < kLanes; ++k) HIP_TRY(hipStreamWaitEvent(ctx->lanes[k].stream, ctx->batch_start, 0), "fork");
    // render-only requests are done with the frames; loss and backward of the others on lanes
    for (int32_t i = 0; i < n; ++i) {
        const lgsr_request &q = reqs[i];
        Lane &L = ctx->lanes[i % kLanes];
        lgsr_state *S = states[(size_t)i];
        if (q.target_depth) {
            const int64_t rays = (int64_t)q.beams.H * q.beams.W;
            if ((st = loss_impl(ctx, L, rays, &q.out, q.target_depth, q.target_normal, w, q.loss_out,
                                &q.frame_grad)) != LGSR_OK)
                return st;
            if ((st = backward_impl(ctx, L, S, &q.frame_grad, &q.grads, q.grad_pose)) != LGSR_OK) return st;
            HIP_TRY(hipEventRecord(ctx->req_done[(size_t)i], L.stream), "request done");
        } else {
            HIP_TRY(hipEventRecord(ctx->req_done[(size_t)i], ctx->stream), "request done");
        }
        ctx->batch_n = i + 1;
    }
    return LGSR_OK;
}

lgsr_status lgsr_request_bytes(int64_t n, int32_t H, int32_t W, int64_t P, int32_t with_grad, int64_t *bytes)
{
    if (!bytes || n < 0 || P < 0 || H < 1 || W < 1 || H > 32768 || W > 32768) return LGSR_EINVAL;
    // every buffer as ensure() sizes it: the request plus a quarter, whole 4 KiB pages
    auto buf = [](size_t b) -> size_t {
        if (b == 0) b = 256;
        return ((b + b / 4) + 4095) & ~(size_t)4095;
    };
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const int TH = (H + kTile - 1) / kTile, TW = (W + kTile - 1) / kTile;
    const int64_t T = (int64_t)TH * TW, rays = (int64_t)H * W;
    const int seg = chunk_size(P, 0);
    const int64_t items = chunk_items_max(P, (int)T, seg);
    const size_t pp = (size_t)(P > 0 ? P : 1);
    size_t b = buf(nn * kRec * sizeof(float)) + buf(nn * sizeof(uint2)) + buf(nn * 4) + buf((size_t)T * sizeof(uint2)) +
               4 * buf((size_t)rays * sizeof(float4)) + buf(16 * sizeof(float)) + 2 * buf((size_t)T * kShards * 4) +
               buf((size_t)T * 4) + buf(16) + buf(pp * 4 + pp) + buf(pp * 8) +
               buf((size_t)(items > 0 ? items : 1) * sizeof(uint4)) + buf((size_t)(T + 1) * sizeof(uint32_t)) +
               buf(chunk_slot_floats(items > 0 ? items : 1) * sizeof(float)) +
               buf((size_t)(items > 0 ? 4 * items : 1) * sizeof(uint32_t)) +
               buf((size_t)(items > 0 ? 4 * items : 1) * sizeof(uint64_t));
    if (with_grad)
        b += buf((size_t)loss_blocks(rays) * 4 * sizeof(float)) + buf(nn * kGrad * sizeof(float)) +
             buf((size_t)chain_blocks(n) * 6 * sizeof(float));
    *bytes = (int64_t)b;
    return LGSR_OK;
}

lgsr_status lgsr_batch_poll(lgsr_ctx *ctx, int32_t n, int32_t *done)
{
    if (!ctx) return LGSR_EINVAL;
    if (n < 0 || (n > 0 && !done)) return fail(ctx, LGSR_EINVAL, "n < 0 or done is NULL");
    if (n > ctx->batch_n) return fail(ctx, LGSR_EINVAL, "the latest batch issued %d requests", ctx->batch_n);
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    for (int32_t i = 0; i < n; ++i) {
        const hipError_t e = hipEventQuery(ctx->req_done[(size_t)i]);
        if (e == hipSuccess) done[i] = 1;
        else if (e == hipErrorNotReady) done[i] = 0;
        else return hip_fail(ctx, e, "request event");
    }
    return LGSR_OK;
}

void lgsr_state_free(lgsr_state *S)
{
    if (!S || !S->ctx) return;
    lgsr_ctx *ctx = S->ctx;
    if (S == &ctx->scratch_state || !S->live) return;
    S->live = false;
    ctx->live_states--;
    ctx->pool.push_back(S);
}

lgsr_status lgsr_query(lgsr_ctx *ctx, const lgsr_state *S, int64_t out[8])
{
    if (!ctx) return LGSR_EINVAL;
    if (!S || !out) return fail(ctx, LGSR_EINVAL, "state or out is NULL");
    if (S->ctx != ctx || !S->live) return fail(ctx, LGSR_ESTATE, "state does not belong to this context");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = ctx->stream;
    uint32_t *counters = as<uint32_t>(ctx->counters);
    lgsr_state *W = const_cast<lgsr_state *>(S);
    unsigned long long *wc = reinterpret_cast<unsigned long long *>(counters + 8);
    HIP_TRY(launch_max_range(as<uint2>(W->ranges), S->g.T, counters + 1, s), "query");
    HIP_TRY(launch_count_visible(as<uint2>(W->rects), S->S.n, counters + 2, s), "query");
    HIP_TRY(launch_work_counts(as<uint2>(W->ranges), W->ids, as<uint2>(W->rects), S->P, as<float4>(W->st1), S->g, wc, s),
            "query");
    if (S->P > 0) HIP_TRY(launch_work_needed(W->R, S->g, S->prm, wc + 3, s), "query");
    HIP_TRY(hipMemcpyAsync(ctx->pinned + 1, counters + 1, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s),
            "readback");
    HIP_TRY(hipMemcpyAsync(ctx->pinned + 4, wc, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
            "readback");
    HIP_TRY(hipStreamSynchronize(s), "query sync");
    const unsigned long long *hw = reinterpret_cast<const unsigned long long *>(ctx->pinned + 4);
    out[0] = S->P;
    out[1] = (int64_t)ctx->pinned[2];
    out[2] = (int64_t)(ctx_bytes(ctx) + state_bytes(S));
    out[3] = (int64_t)ctx->pinned[1];
    out[4] = (int64_t)hw[0];
    out[5] = (int64_t)hw[1];
    out[6] = (int64_t)hw[2];
    out[7] = (int64_t)hw[3];
    return LGSR_OK;
}

lgsr_status lgsr_count_hits(lgsr_ctx *ctx, const lgsr_state *S, int64_t out[2])
{
    if (!ctx) return LGSR_EINVAL;
    if (!S || !out) return fail(ctx, LGSR_EINVAL, "state or out is NULL");
    if (S->ctx != ctx || !S->live) return fail(ctx, LGSR_ESTATE, "state does not belong to this context");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = ctx->stream;
    unsigned long long *wc = reinterpret_cast<unsigned long long *>(as<uint32_t>(ctx->counters) + 8);
    if (S->P > 0) {
        HIP_TRY(launch_count_hits(S->R, S->g, S->prm, wc, s), "count hits");
        HIP_TRY(hipMemcpyAsync(ctx->pinned + 4, wc, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
                "readback");
        HIP_TRY(hipStreamSynchronize(s), "count hits sync");
        const unsigned long long *hw = reinterpret_cast<const unsigned long long *>(ctx->pinned + 4);
        out[0] = (int64_t)hw[0];
        out[1] = (int64_t)hw[1];
    } else {
        out[0] = out[1] = 0;
    }
    return LGSR_OK;
}

lgsr_status lgsr_tile_list(lgsr_ctx *ctx, const lgsr_state *S, int32_t tile_row, int32_t tile_col, uint32_t *ids,
                           int64_t cap, int64_t *count)
{
    if (!ctx) return LGSR_EINVAL;
    if (!S || !count || (cap > 0 && !ids) || cap < 0) return fail(ctx, LGSR_EINVAL, "state, ids or count invalid");
    if (S->ctx != ctx || !S->live) return fail(ctx, LGSR_ESTATE, "state does not belong to this context");
    if (tile_row < 0 || tile_row >= S->g.TH || tile_col < 0 || tile_col >= S->g.TW)
        return fail(ctx, LGSR_EINVAL, "tile (%d, %d) outside the %d x %d tile grid", tile_row, tile_col, S->g.TH,
                    S->g.TW);
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = ctx->stream;
    const int t = tile_id(tile_row, tile_col, S->g.TH);
    uint2 rg{0u, 0u};
    if (S->P > 0) {
        HIP_TRY(hipMemcpyAsync(&rg, as<uint2>(const_cast<lgsr_state *>(S)->ranges) + t, sizeof(uint2),
                               hipMemcpyDeviceToHost, s),
                "tile range");
        HIP_TRY(hipStreamSynchronize(s), "tile range sync");
    }
    const int64_t len = (int64_t)rg.y - (int64_t)rg.x;
    *count = len;
    if (len > 0 && cap > 0) {
        HIP_TRY(hipMemcpyAsync(ids, S->ids + rg.x, (size_t)std::min(len, cap) * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, s),
                "tile list");
        HIP_TRY(hipStreamSynchronize(s), "tile list sync");
    }
    return LGSR_OK;
}

lgsr_status lgsr_stream_probe(lgsr_ctx *ctx, int32_t kind, const float *b, const float *c, float *a, int64_t n,
                              int32_t blocks)
{
    if (!ctx) return LGSR_EINVAL;
    if (n < 0 || (n % 4) != 0) return fail(ctx, LGSR_EINVAL, "n must be a non-negative multiple of 4");
    if (kind < 0 || kind > 3) return fail(ctx, LGSR_EINVAL, "kind must lie in 0..3");
    if (blocks < 0 || blocks > (1 << 20)) return fail(ctx, LGSR_EINVAL, "blocks must lie in 0..2^20");
    if (n > 0 && (!b || !a || ((kind & 1) && !c))) return fail(ctx, LGSR_EINVAL, "NULL array");
    if (((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(c)) & 15u) != 0)
        return fail(ctx, LGSR_EINVAL, "arrays must be 16-byte aligned");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(launch_stream_probe(kind, b, c, a, n, blocks, ctx->stream), "stream probe");
    return LGSR_OK;
}

lgsr_status lgsr_profile(lgsr_ctx *ctx, int32_t stage_mask)
{
    if (!ctx) return LGSR_EINVAL;
    ctx->prof_mask = (uint32_t)stage_mask;
    return LGSR_OK;
}

lgsr_status lgsr_profile_read(lgsr_ctx *ctx, double ms[LGSR_NUM_STAGES], int64_t calls[LGSR_NUM_STAGES])
{
    if (!ctx) return LGSR_EINVAL;
    if (!ms || !calls) return fail(ctx, LGSR_EINVAL, "ms or calls is NULL");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "profile sync");
    for (auto &pe : ctx->ev_pending) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, pe.second.first, pe.second.second) == hipSuccess) {
            ctx->prof_ms[pe.first] += t;
            ctx->prof_calls[pe.first] += 1;
        } else {
            (void)hipGetLastError();
        }
        ctx->ev_free.push_back(pe.second.first);
        ctx->ev_free.push_back(pe.second.second);
    }
    ctx->ev_pending.clear();
    for (int k = 0; k < LGSR_NUM_STAGES; ++k) {
        ms[k] = ctx->prof_ms[k];
        calls[k] = ctx->prof_calls[k];
        ctx->prof_ms[k] = 0.0;
        ctx->prof_calls[k] = 0;
    }
    return LGSR_OK;
}

lgsr_status lgsr_sync(lgsr_ctx *ctx)
{
    if (!ctx) return LGSR_EINVAL;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "sync");
    return LGSR_OK;
}

lgsr_status lgsr_state_bytes(lgsr_ctx *ctx, const lgsr_state *S, int64_t *bytes)
{
    if (!ctx) return LGSR_EINVAL;
    if (!bytes) return fail(ctx, LGSR_EINVAL, "bytes is NULL");
    if (!S) {
        *bytes = (int64_t)ctx_bytes(ctx);
        return LGSR_OK;
    }
    if (S->ctx != ctx || !S->live) return fail(ctx, LGSR_ESTATE, "state does not belong to this context");
    *bytes = (int64_t)state_bytes(S);
    return LGSR_OK;
}

lgsr_status lgsr_adam_step(lgsr_ctx *ctx, int32_t n_groups, const lgsr_adam_group *groups, float beta1, float beta2,
                           float eps, int32_t step)
{
    if (!ctx) return LGSR_EINVAL;
    if (n_groups < 0 || n_groups > 8) return fail(ctx, LGSR_EINVAL, "n_groups must lie in [0, 8]");
    if (n_groups > 0 && !groups) return fail(ctx, LGSR_EINVAL, "groups is NULL");
    if (step < 1) return fail(ctx, LGSR_EINVAL, "step must be >= 1");
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
        return fail(ctx, LGSR_EINVAL, "beta1 and beta2 must lie in [0, 1)");
    if (!std::isfinite(eps) || eps < 0.f) return fail(ctx, LGSR_EINVAL, "eps must be finite and >= 0");
    AdamBatch B{};
    B.count = n_groups;
    for (int k = 0; k < n_groups; ++k) {
        const lgsr_adam_group &G = groups[k];
        if (G.n < 0) return fail(ctx, LGSR_EINVAL, "group %d: n < 0", k);
        if (G.n > 0 && (!G.param || !G.grad || !G.m || !G.v)) return fail(ctx, LGSR_EINVAL, "group %d: NULL array", k);
        if (!std::isfinite(G.lr)) return fail(ctx, LGSR_EINVAL, "group %d: lr must be finite", k);
        B.g[k] = AdamGroup{G.n, G.param, G.grad, G.m, G.v, G.lr};
    }
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(launch_adam(B, beta1, beta2, eps, step, ctx->stream), "adam");
    return LGSR_OK;
}

}  // extern "C"
