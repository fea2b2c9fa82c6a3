"""Benchmark: forward + loss + backward of the spherical surfel renderer on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

One step = lgsr_forward (projection, culling, both sorts, compositing) + lgsr_loss +
lgsr_backward (raster backward, chain rule to every surfel parameter and the pose) over the
64 x 1024-beam, 300,000-surfel synthetic street-block scene; inputs are resident in HBM
before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rendered rays/s fwd+bwd @64×1024, 300k surfels; p50/p99 batched render latency"

# Algorithmic float32 operations of the raster (FMA = 2): per ray-surfel test (ray direction
# offsets, plane denominator with the exact ray direction, two homogeneous tangent
# coordinates, reciprocal, range, squared radius, Gaussian, opacity clamp and the four
# threshold tests), per composited hit forward (weight, the four sums, transmittance, stop
# test) and backward (transmittance recovery, dL/dalpha_hat, the clamp, and the gradients
# w.r.t. the 13 record quantities).
FLOPS_TEST = 41
FLOPS_COMPOSITE_BWD = 65
FLOPS_COMPOSITE_FWD = 13
# MI355X float32 vector peak without packed (dual) float32 math: 256 CUs x 64 lanes x
# 2 flops (FMA) x 2.4 GHz.  The published 157.3 TFLOP/s counts packed float32, which this
# build does not emit.
PEAK_FP32_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
PEAK_FP32_PUBLISHED = 157.3
PEAK_HBM_GBS = 8000.0

# HBM bytes of one raster_bwd launch on the benchmark workload: rocprofv3 FETCH_SIZE and
# WRITE_SIZE per dispatch, each scaled by what the counter reads for a plain 256 MiB device
# copy (profiles/pmc_traffic_raster_bwd_block64x1024_300k.md).  Valid only for the kernel
# sources they were taken with (digest below); reported as null once those change.
TRAFFIC_RASTER_BWD = dict(bytes=77672111,
                          sources_sha256="311327d7e9c240845593e710ae7e44d355accb59b856b7870bf0425f5ea563ec")


# rocprofv3 SQ counters of one raster_bwd launch on the benchmark workload (per dispatch) and
# the kernel's mean duration in the same profiled run; same validity rule as the traffic.
SQ_RASTER_BWD = dict(SQ_INSTS_VALU=25740091, SQ_INSTS_LDS=974275, SQ_LDS_BANK_CONFLICT=305352, ms=0.0678,
                     sources_sha256="311327d7e9c240845593e710ae7e44d355accb59b856b7870bf0425f5ea563ec")


def _sources_digest() -> str:
    """Digest of the sources raster_bwd is compiled from."""
    import hashlib
    d = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2607_04127_amd", "csrc")
    for name in ("raster.hip", "lgsr_internal.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            d.update(name.encode() + b"\0" + f.read())
    return d.hexdigest()


def _bytes_model(n, P, rays):
    """Bytes a tile-binned forward + backward must move (record and gradient layouts of
    this implementation): per surfel the parameters (40 B) read twice, the 64 B record
    written once, the range key written once, the 52 B record gradient zeroed, added and
    read, 40 B of parameter gradients written; per (surfel, tile) pair the 4 B id written by
    emission, read, its range key gathered and written back by the per-tile sort, the
    record, id and ray rectangle read by both rasters; per ray the beam tables, 21 B of
    frame output, 32 B per-ray state written and read, 16 B of targets and 20 B of loss
    gradient written and read."""
    per_surfel = 40 + 64 + 4 + 40 + 3 * 52 + 40
    per_pair = 4 + 12 + 2 * (64 + 4 + 8)
    per_ray = 21 + 2 * 32 + 16 + 2 * 20 + 8
    return n * per_surfel + P * per_pair + rays * per_ray


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="block64x1024_300k")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--service-requests", type=int, default=10000,
                    help="requests per rate of the batched-service phase (0 = skip)")
    ap.add_argument("--no-growth", action="store_true", help="skip the sliding-window and deep-list workloads")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU oracle sample time")
    ap.add_argument("--chunk", type=int, default=0, help="list entries per raster chunk (0 = automatic)")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="bytes of one plain device copy issued before the steps (calibrates counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1 (one process)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import scenegen
    from paper_2607_04127_amd import lgsr

    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    w = scenegen.make_workload(args.workload)
    print(f"# workload {args.workload}: N={w['means'].shape[0]} H={w['H']} W={w['W']} "
          f"(generated in {time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    H, W = w["H"], w["W"]
    rays = H * W
    n = w["means"].shape[0]
    S = {k: torch.from_numpy(w[k]).to(dev) for k in ("means", "quats", "log_scales", "opacity_logits")}
    rows = torch.from_numpy(w["row_sincos"]).to(dev)
    cols = torch.from_numpy(w["col_sincos"]).to(dev)
    pose = torch.from_numpy(w["pose"])
    td = torch.from_numpy(w["target_depth"]).to(dev)
    tn = torch.from_numpy(w["target_normal"]).to(dev)
    frame = dict(depth=torch.empty((H, W), device=dev), opacity=torch.empty((H, W), device=dev),
                 normal=torch.empty((H, W, 3), device=dev), drop=torch.empty((H, W), device=dev, dtype=torch.uint8))
    fgrad = dict(depth=torch.empty((H, W), device=dev), opacity=torch.empty((H, W), device=dev),
                 normal=torch.empty((H, W, 3), device=dev))
    sgrad = dict(means=torch.empty((n, 3), device=dev), quats=torch.empty((n, 4), device=dev),
                 log_scales=torch.empty((n, 2), device=dev), opacity_logits=torch.empty((n,), device=dev))
    loss = torch.empty(5, device=dev)
    gpose = torch.empty(6, device=dev)
    ctx = lgsr.Context(0)
    opts = lgsr.default_opts(chunk=args.chunk)
    if args.calib_copy:
        src = torch.empty(args.calib_copy // 4, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        _, st = lgsr.lgsr_forward(ctx, S, pose, rows, cols, opts=opts, out=frame)
        lgsr.lgsr_loss(ctx, frame, td, tn, loss_out=loss, grad_out=fgrad)
        lgsr.lgsr_backward(ctx, st, fgrad, out=sgrad, grad_pose=gpose)
        st.free()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"# warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    # Timed region: K steps back to back, no stage timers.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = rays / (ms_per_step / 1e3)
    print(f"# timed {args.steps} steps: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)
    # Per-step latency (each step synchronised on its own).
    step_ms = []
    for _ in range(args.steps):
        a = time.perf_counter()
        step()
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - a) * 1e3)
    # The dominant kernel timed with HIP events on the library's stream (events around it only).
    lgsr.lgsr_profile(ctx, ["raster_bwd", "raster_fwd"])
    lgsr.lgsr_profile_read(ctx)
    for _ in range(args.steps):
        step()
    dom = lgsr.lgsr_profile_read(ctx)
    # Stage breakdown (events around every stage; each event adds some stream time).
    lgsr.lgsr_profile(ctx, True)
    for _ in range(args.steps):
        step()
    prof = lgsr.lgsr_profile_read(ctx)
    lgsr.lgsr_profile(ctx, False)

    # work counters of one forward (same inputs, deterministic lists)
    _, st = lgsr.lgsr_forward(ctx, S, pose, rows, cols, opts=opts, out=frame)
    q = lgsr.lgsr_query(ctx, st)
    st.free()
    stages = {k: dict(ms_per_call=(v[0] / v[1] if v[1] else 0.0), calls=v[1]) for k, v in prof.items()}
    bwd_ms = dom["raster_bwd"][0] / max(dom["raster_bwd"][1], 1)
    fwd_ms = dom["raster_fwd"][0] / max(dom["raster_fwd"][1], 1)
    flops_bwd = q["ray_tests"] * FLOPS_TEST + q["composites"] * FLOPS_COMPOSITE_BWD
    flops_fwd = q["ray_tests"] * FLOPS_TEST + q["composites"] * FLOPS_COMPOSITE_FWD
    achieved = flops_bwd / (bwd_ms * 1e-3) / 1e12 if bwd_ms > 0 else 0.0
    bytes_step = _bytes_model(n, q["pairs"], rays)
    p50 = float(np.percentile(step_ms, 50))
    p99 = float(np.percentile(step_ms, 99))

    cold = cache_cold_phase(ctx, step, args.steps)
    hbm = hbm_probe(ctx)

    aux = aux_kernels(ctx, w, S, rows, cols, pose, frame, td, tn, args.steps)

    svc = None
    if args.service_requests > 0:
        svc = service_phase(ctx, args.service_requests)

    growth = None if args.no_growth else growth_phase(ctx)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded street-block scene, virtual-scan surfels, exact raycast targets)",
        "config": {"workload": args.workload, "rays": rays, "H": H, "W": W, "surfels": n, "chunk": args.chunk,
                   "pairs": q["pairs"], "visible_surfels": q["visible"], "max_tile_list": q["max_list"],
                   "ray_tests": q["ray_tests"], "ray_tests_needed": q["ray_tests_needed"],
                   "composites": q["composites"], "rays_hit": q["rays_hit"],
                   "loss": "depth L1 + G-ICP normal cosine", "step_latency_ms_p50": round(p50, 4),
                   "step_latency_ms_p99": round(p99, 4),
                   "batched_latency_ms_p50": svc["at_0.5x"]["batched"]["p50_ms"] if svc else None,
                   "batched_latency_ms_p99": svc["at_0.5x"]["batched"]["p99_ms"] if svc else None,
                   "latency_config": "rendering service at 0.5x single-request capacity (see service)"},
        "service": svc,
        "growth": growth,
        "aux_kernels": aux,
        "roofline": {"kernel": "raster_bwd", "bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(PEAK_FP32_TFLOPS, 1), "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": (TRAFFIC_RASTER_BWD["bytes"]
                                 if TRAFFIC_RASTER_BWD["sources_sha256"] == _sources_digest() else None),
                     "flops_per_launch": flops_bwd, "ms_per_launch": round(bwd_ms, 5),
                     "peak_published_packed": PEAK_FP32_PUBLISHED},
        "stages_ms": {k: round(v["ms_per_call"], 5) for k, v in stages.items() if v["calls"]},
        "raster_fwd": {"ms_per_launch": round(fwd_ms, 5), "flops_per_launch": flops_fwd,
                       "achieved_tflops": round(flops_fwd / (fwd_ms * 1e-3) / 1e12, 3) if fwd_ms > 0 else 0.0},
        "hbm_model": {"bytes_per_step": bytes_step, "achieved_GBps": round(bytes_step / (ms_per_step * 1e-3) / 1e9, 1),
                      "frac_of_8TBps": round(bytes_step / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
        "hbm": hbm_fractions(hbm, n, q["pairs"], rays, bytes_step, ms_per_step, cold, bwd_ms),
        "cache_cold": cold,
        "counters": counter_figures(bwd_ms),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def hbm_probe(ctx):
    """The HBM bandwidth a plain streaming kernel reaches on this device: a copy over 2 x 2 GiB
    and a triad over 3 x 1.5 GiB (working sets far beyond the 256 MB last-level cache), each
    in two access forms (non-temporal 4-vector, plain 1-vector) at 1024, 4096 and 65536
    workgroups, HIP events on the library's stream, the best of 5 repetitions per form after
    one warm-up, then the best form."""
    import torch

    from paper_2607_04127_amd import lgsr

    dev = torch.device("cuda:0")
    out = {}
    for kind, arrays, nbytes_per in (("copy", 2, 8), ("triad", 3, 12)):
        n = (2 if kind == "copy" else 1.5) * 2 ** 30 / 4
        n = int(n) // 4 * 4
        A = [torch.empty(n, device=dev) for _ in range(arrays)]
        for t in A:
            t.fill_(1.0)
        best, form = None, None
        for plain in (False, True):
            for blocks in (1024, 4096, 65536):
                def call():
                    lgsr.lgsr_stream_probe(ctx, kind, A[0], A[1], A[2] if kind == "triad" else None, plain=plain,
                                           blocks=blocks)
                call()
                torch.cuda.synchronize()
                for _ in range(5):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    call()
                    b.record()
                    torch.cuda.synchronize()
                    ms = a.elapsed_time(b)
                    if best is None or ms < best:
                        best, form = ms, f"{'plain 1-vector' if plain else 'non-temporal 4-vector'}, {blocks} workgroups"
        out[f"{kind}_GBps"] = round(nbytes_per * n / (best * 1e-3) / 1e9, 1)
        out[f"{kind}_form"] = form
        out[f"{kind}_working_set_GiB"] = round(arrays * 4 * n / 2 ** 30, 2)
        del A
        torch.cuda.empty_cache()
    out["achievable_GBps"] = max(out["copy_GBps"], out["triad_GBps"])
    print(f"# hbm probe: copy {out['copy_GBps']:.0f} GB/s, triad {out['triad_GBps']:.0f} GB/s", file=sys.stderr,
          flush=True)
    return out


def cache_cold_phase(ctx, step, steps):
    """Step time with the caches flushed before every step: a 1 GiB streaming copy (512 MiB
    read, 512 MiB written) runs first, then HIP events bracket the step alone."""
    import numpy as np
    import torch

    from paper_2607_04127_amd import lgsr

    dev = torch.device("cuda:0")
    n = 2 ** 27  # 512 MiB of float32
    src, dst = torch.ones(n, device=dev), torch.empty(n, device=dev)
    times = []
    for _ in range(steps):
        lgsr.lgsr_stream_probe(ctx, "copy", dst, src)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        step()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    del src, dst
    torch.cuda.empty_cache()
    p50 = float(np.percentile(times, 50))
    print(f"# cache-cold step: p50 {p50:.3f} ms", file=sys.stderr, flush=True)
    return {"ms_per_step_p50": round(p50, 4), "ms_per_step_p90": round(float(np.percentile(times, 90)), 4),
            "flush_bytes": 2 * 4 * n, "steps": steps}


def hbm_fractions(hbm, n, P, rays, bytes_step, ms_per_step, cold, bwd_ms):
    """The step's and raster_bwd's HBM use against the measured achievable bandwidth."""
    bw = hbm["achievable_GBps"]
    # algorithmic bytes of tile-binned splatting at 56 B records (288 N + 156 P + 113 rays)
    b_method = 288 * n + 156 * P + 113 * rays
    compulsory = 80 * n + 37 * rays  # parameters in, targets in, image out, gradients out

    def frac(nbytes, ms):
        return round(nbytes / (ms * 1e-3) / 1e9 / bw, 4) if ms > 0 else None

    out = dict(hbm, b_method_bytes=b_method, compulsory_bytes=compulsory, implementation_model_bytes=bytes_step,
               step_frac_of_achievable=frac(b_method, ms_per_step),
               step_frac_of_achievable_cache_cold=frac(b_method, cold["ms_per_step_p50"]),
               implementation_model_frac_of_achievable=frac(bytes_step, ms_per_step),
               compulsory_frac_of_achievable=frac(compulsory, ms_per_step))
    traffic = TRAFFIC_RASTER_BWD["bytes"] if TRAFFIC_RASTER_BWD["sources_sha256"] == _sources_digest() else None
    out["raster_bwd_traffic_frac_of_achievable"] = frac(traffic, bwd_ms) if traffic else None
    return out


def counter_figures(bwd_ms):
    """VALU issue and LDS bank-conflict figures of raster_bwd from the rocprofv3 SQ counters
    (profiles/sq_counters_block64x1024_300k.md), against the chip's issue capacity: 1024 SIMDs
    at 2.4 GHz, a wave64 VALU instruction holding its SIMD for 4 cycles.  Null once the kernel
    sources differ from those the counters were taken with."""
    if SQ_RASTER_BWD["sources_sha256"] != _sources_digest():
        return None
    c = SQ_RASTER_BWD
    simd_cycles = 1024 * 2.4e9 * c["ms"] * 1e-3
    cu_cycles = 256 * 2.4e9 * c["ms"] * 1e-3
    return {"kernel": "raster_bwd", "counters_ms_per_launch": c["ms"],
            "valu_busy_frac": round(4 * c["SQ_INSTS_VALU"] / simd_cycles, 4),
            "lds_instructions": c["SQ_INSTS_LDS"], "lds_bank_conflict_cycles": c["SQ_LDS_BANK_CONFLICT"],
            "lds_bank_conflict_frac_of_cu_cycles": round(c["SQ_LDS_BANK_CONFLICT"] / cu_cycles, 4)}


def _time_us(fn, reps):
    """Mean microseconds per call of fn over reps calls, HIP events on torch's current stream
    (the stream the library issues on)."""
    import torch
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e3 / reps


def aux_kernels(ctx, w, S, rows, cols, pose, frame, td, tn, reps):
    """The kernels beside the rendering path on the benchmark's shapes, each against the HBM
    roofline with its algorithmic bytes: the full objective of Eq. 13 on the 64 x 1024 frame,
    the scale regulariser and the target covariances over the 300k surfels, and the
    projection of a 64 x 1024 scan of the same street block."""
    import numpy as np
    import torch

    import scenegen
    from paper_2607_04127_amd import lgsr

    dev = rows.device
    H, W = rows.shape[0], cols.shape[0]
    rays, n = H * W, S["means"].shape[0]
    reps = max(reps, 20)
    out = {}

    def entry(us, nbytes, note):
        gbs = nbytes / (us * 1e-6) / 1e9
        return dict(us_per_call=round(us, 3), bytes=int(nbytes), GBps=round(gbs, 1),
                    frac_of_8TBps=round(gbs / PEAK_HBM_GBS, 4), bytes_model=note)

    lgsr.lgsr_forward(ctx, S, pose, rows, cols, out=frame, want_state=False)
    Lo = torch.empty(8, device=dev)
    go = dict(depth=torch.empty((H, W), device=dev), opacity=torch.empty((H, W), device=dev),
              normal=torch.empty((H, W, 3), device=dev))
    wts = lgsr.default_objective_weights()
    us = _time_us(lambda: lgsr.lgsr_objective(ctx, frame, rows, cols, td, tn, wts, loss_out=Lo, grad_out=go), reps)
    out["objective"] = entry(us, rays * (2 * 36 + 20), "per ray: depth, opacity, normal, targets (36 B) read "
                                                       "by both passes, 20 B of gradient written")
    ls = S["log_scales"]
    gls = torch.zeros_like(ls)
    Ls = torch.empty(1, device=dev)
    us = _time_us(lambda: lgsr.lgsr_scale_reg(ctx, ls, 10.0, 1.0, loss_out=Ls, grad_log_scales=gls), reps)
    out["scale_reg"] = entry(us, n * 24, "per surfel: 8 B log-scales read, 16 B gradient read and written")
    cov = torch.empty((n, 6), device=dev)
    us = _time_us(lambda: lgsr.lgsr_target_cov(ctx, S["quats"], ls, 0.01, out=cov), reps)
    out["target_cov"] = entry(us, n * 48, "per surfel: 16 B quaternion and 8 B log-scales read, 24 B written")
    pts, nrm = scenegen.synthetic_scan(w["scene"], w["pose"], H, W, -22.5, 22.5, seed=7)
    pts_d, nrm_d = torch.from_numpy(pts).to(dev), torch.from_numpy(nrm).to(dev)
    so = dict(depth=torch.empty((H, W), device=dev), normal=torch.empty((H, W, 3), device=dev),
              index=torch.empty((H, W), device=dev, dtype=torch.int32))
    el = (np.radians(-22.5), np.radians(22.5))
    us = _time_us(lambda: lgsr.lgsr_scan_to_range(ctx, pts_d, H, W, el[0], el[1], 0.5, 80.0, normals=nrm_d, out=so),
                  reps)
    hits = int((so["index"] >= 0).sum())
    out["scan_to_range"] = entry(us, pts.shape[0] * 20 + rays * 44 + hits * 24,
                                 f"{pts.shape[0]} points: 12 B read, one 8 B atomic; per pixel 8 B key "
                                 f"filled and read, 20 B written; per return 24 B of the winner gathered")
    return out


def service_phase(ctx, n_requests):
    """The batched-service configuration: four resident street-block maps of 100k, 400k, 1M and
    2M surfels, request templates at 32 x 1024 and 64 x 1024 beams (+-22.5 deg) and 128 x 2048
    beams (+-45 deg) with two random poses each and exact raycast targets, Poisson arrivals
    (70% render, 30% render + gradient) at 0.25, 0.5 and 0.9 times the measured
    one-request-per-call capacity and at a fixed 3000 requests/s; n_requests per rate, served
    batched (up to 16 per call, each request's latency taken when its results are ready; at
    0.9x and 3000/s also with one launch per compositing stage for the whole batch) and one
    by one, with p50 / p99 latency and rays/s for each."""
    import torch

    from paper_2607_04127_amd import service as SV

    t = time.perf_counter()
    maps = SV.make_maps([100_000, 400_000, 1_000_000, 2_000_000], seed=41)
    pool = SV.make_pool(maps, poses_per=2, seed=45)
    SV.measure_pairs(ctx, pool)
    torch.cuda.synchronize()
    print(f"# service: {len(maps)} maps, {len(pool)} templates ({time.perf_counter() - t:.1f} s)", file=sys.stderr,
          flush=True)
    cap = SV.capacity(ctx, pool, n=200)
    out = dict(maps=[m["n"] for m in maps], templates=len(pool), requests_per_rate=n_requests, grad_fraction=0.3,
               max_batch=16, single_capacity_rps=round(cap, 1))
    for label, rate in (("at_0.25x", 0.25 * cap), ("at_0.5x", 0.5 * cap), ("at_0.9x", 0.9 * cap),
                        ("fixed_3000rps", 3000.0)):
        stream = SV.poisson_stream(pool, n_requests, rate, grad_fraction=0.3, seed=45)
        entry = dict(rate_rps=round(rate, 1))
        # the fused batch mode (one launch per compositing stage for the whole batch) only
        # differs from the per-stream one where batches hold several requests
        modes = ("batched", "single") if label in ("at_0.25x", "at_0.5x") else ("batched", "fused", "single")
        for mode in modes:
            SV.Service(ctx, pool, mode, max_batch=16).run(stream[:50])  # warm the per-request states
            rep = SV.Service(ctx, pool, mode, max_batch=16).run(stream)
            entry[mode] = dict(p50_ms=round(rep["p50_ms"], 4), p99_ms=round(rep["p99_ms"], 4),
                               rays_per_s=round(rep["rays_per_s"], 1), mean_batch=round(rep["mean_batch"], 2))
            print(f"# service {label} {mode}: p50 {rep['p50_ms']:.3f} ms p99 {rep['p99_ms']:.3f} ms "
                  f"({rep['rays_per_s'] / 1e6:.1f} Mrays/s, mean batch {rep['mean_batch']:.1f})",
                  file=sys.stderr, flush=True)
        out[label] = entry
    del maps, pool
    torch.cuda.empty_cache()
    return out


def growth_phase(ctx):
    """The growth workloads: the sliding window (64 x 2048 beams, 1M surfels, 8 keyframes, 10
    Adam iterations through the autograd layer with the lists recomputed in the backward) and
    the deep-list stress (128 x 2048 beams, 4M surfels with 30% in 0.5 m blobs: forward +
    backward of a fixed random functional of the frame with the pose gradient, lists kept,
    then recomputed)."""
    import numpy as np
    import torch

    import scenegen
    from paper_2607_04127_amd import autograd as AG
    from paper_2607_04127_amd import lgsr
    from paper_2607_04127_amd import window as WN

    out = {}
    t = time.perf_counter()
    w = scenegen.make_workload("window64x2048_1m")
    print(f"# window workload ({time.perf_counter() - t:.1f} s)", file=sys.stderr, flush=True)
    poses, means = WN.perturb(w)
    win = WN.Window(ctx, w, poses, means=means, keep_lists="recompute")
    err0 = WN.pose_errors(win.pose_opt.T0, w["poses"])
    curve, times = [], []
    for _ in range(10):
        torch.cuda.synchronize()
        a = time.perf_counter()
        curve.append(win.step())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - a)
    err1 = WN.pose_errors(win.pose_opt.T0, w["poses"])
    rays = w["H"] * w["W"] * len(w["poses"])
    out["window64x2048_1m"] = dict(
        surfels=int(w["means"].shape[0]), keyframes=len(w["poses"]), iterations=10, keep_lists="recompute",
        s_per_iter=round(float(np.median(times)), 5), rays_per_s=round(rays / float(np.median(times)), 1),
        loss=[round(x, 6) for x in curve], recomputed_backwards=win.renderer.recomputed,
        pose_err_before_m_deg=[round(float(np.mean([e[0] for e in err0])), 5),
                               round(float(np.degrees(np.mean([e[1] for e in err0]))), 4)],
        pose_err_after_m_deg=[round(float(np.mean([e[0] for e in err1])), 5),
                              round(float(np.degrees(np.mean([e[1] for e in err1]))), 4)])
    print(f"# window: {np.median(times) * 1e3:.2f} ms/iteration, loss {curve[0]:.4f} -> {curve[-1]:.4f}",
          file=sys.stderr, flush=True)
    del win, w
    torch.cuda.empty_cache()

    t = time.perf_counter()
    w = scenegen.make_workload("deep128x2048_4m", with_targets=False)
    print(f"# deep workload ({time.perf_counter() - t:.1f} s)", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    H, W = w["H"], w["W"]
    S = {k: torch.from_numpy(np.ascontiguousarray(w[k])).to(dev) for k in AG.SURF_KEYS}
    rows = torch.from_numpy(w["row_sincos"]).to(dev)
    cols = torch.from_numpy(w["col_sincos"]).to(dev)
    pose = torch.from_numpy(w["pose"])
    rng = np.random.default_rng(2024)
    up = dict(depth=torch.from_numpy(rng.uniform(-1, 1, (H, W)).astype(np.float32)).to(dev),
              opacity=torch.from_numpy(rng.uniform(-1, 1, (H, W)).astype(np.float32)).to(dev),
              normal=torch.from_numpy(rng.uniform(-1, 1, (H, W, 3)).astype(np.float32)).to(dev))

    def kept():
        _, st = lgsr.lgsr_forward(ctx, S, pose, rows, cols)
        lgsr.lgsr_backward(ctx, st, up)
        st.free()

    def recomputed():
        lgsr.lgsr_forward(ctx, S, pose, rows, cols, want_state=False)
        _, st = lgsr.lgsr_forward(ctx, S, pose, rows, cols)
        lgsr.lgsr_backward(ctx, st, up)
        st.free()

    res = {}
    for name, fn in (("kept", kept), ("recomputed", recomputed)):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        res[name] = round((time.perf_counter() - a) * 1e3 / 10, 4)
    _, st = lgsr.lgsr_forward(ctx, S, pose, rows, cols)
    q = lgsr.lgsr_query(ctx, st)
    ch = lgsr.lgsr_count_hits(ctx, st)
    st.free()
    out["deep128x2048_4m"] = dict(
        surfels=int(w["means"].shape[0]), rays=H * W, ms_fwd_bwd_lists_kept=res["kept"],
        ms_fwd_bwd_lists_recomputed=res["recomputed"], rays_per_s=round(H * W / (res["kept"] * 1e-3), 1),
        pairs=q["pairs"], max_tile_list=q["max_list"], composites_per_hit_ray=round(q["composites"] / max(q["rays_hit"], 1), 2),
        intersections_per_hit_ray_before_termination=round(ch["hits_all"] / max(ch["rays_with_hits"], 1), 2),
        intersections_per_ray_before_termination=round(ch["hits_all"] / (H * W), 2))
    print(f"# deep: {res['kept']:.3f} ms fwd+bwd (lists kept), {res['recomputed']:.3f} ms (recomputed), "
          f"{out['deep128x2048_4m']['intersections_per_hit_ray_before_termination']} intersections per hit ray",
          file=sys.stderr, flush=True)
    del S, w
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, target_s):
    """The FP64 oracle (forward + loss + backward over every surfel per ray) on a seeded
    ray subset of the same workload, sized to take about target_s seconds."""
    import numpy as np

    from oracle import ref

    H, W = w["H"], w["W"]
    rng = np.random.Generator(np.random.PCG64(1234))
    order = rng.permutation(H * W)

    def run(m):
        ids = np.sort(order[:m])
        t = time.perf_counter()
        ref.loss_and_grad(w, w["pose"], w["row_sincos"], w["col_sincos"], w["target_depth"], w["target_normal"],
                          ray_ids=ids)
        return time.perf_counter() - t

    # the oracle's time is a fixed set-up (projection and ordering of every surfel) plus a
    # per-ray cost: measure both from two short runs, then size the sample
    dt_a, dt_b = run(256), run(1024)
    per_ray = max((dt_b - dt_a) / 768, 1e-7)
    fixed = max(dt_a - 256 * per_ray, 0.0)
    m2 = int(min(H * W, max(1024, (target_s - fixed) / per_ray)))
    dt2 = run(m2)
    cores = ref.threads()
    print(f"# cpu oracle: {m2} rays in {dt2:.1f} s on {cores} threads", file=sys.stderr, flush=True)
    # one thread, on a sample about a fifth as long
    ref.set_threads(1)
    m1 = max(16, int(m2 / cores / 5))
    dt1 = run(m1)
    ref.set_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(m2 / dt2, 1), "unit": "rays/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "one_thread_rays_per_s": round(m1 / dt1, 2),
            "sample": f"{m2} seeded random rays of the {H}x{W} image against all {w['means'].shape[0]} surfels, "
                      f"forward + loss + backward in float64 ({dt2:.1f} s); one thread: {m1} rays ({dt1:.1f} s)"}


if __name__ == "__main__":
    main()
