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
# offsets, plane denominator, two homogeneous tangent coordinates, reciprocal, range,
# squared radius, Gaussian, opacity clamp and the four threshold tests), per composited hit
# forward (weight, the four sums, transmittance, stop test) and backward (transmittance
# recovery, dL/dalpha_hat, the clamp, and the gradients w.r.t. the 13 record quantities).
FLOPS_TEST = 37
FLOPS_COMPOSITE_BWD = 53
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
TRAFFIC_RASTER_BWD = dict(bytes=57538829,
                          sources_sha256="6d58e84aaacbf321e84e7e3db46e8447d3b40160f82dd79dd92be0722e4ac37d")


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
    ap.add_argument("--service-requests", type=int, default=2000,
                    help="requests of the batched-service latency phase (0 = skip)")
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

    aux = aux_kernels(ctx, w, S, rows, cols, pose, frame, td, tn, args.steps)

    svc = None
    if args.service_requests > 0:
        svc = service_phase(ctx, w, S, rows, cols, args.service_requests)

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
                   "batched_latency_ms_p50": svc["batched"]["p50_ms"] if svc else None,
                   "batched_latency_ms_p99": svc["batched"]["p99_ms"] if svc else None},
        "service": svc,
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
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


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


def service_phase(ctx, w, S, rows, cols, n_requests, n_poses=4, seed=45):
    """Batched render latency on the benchmark map: n_requests Poisson arrivals (70% render,
    30% render + gradient) over n_poses poses (random yaw, +-5 m), at 0.7 times the measured
    one-request-per-call capacity, served batched (up to 16 per call) and one by one."""
    import numpy as np
    import torch

    import scenegen
    from paper_2607_04127_amd import service as SV

    rng = np.random.Generator(np.random.PCG64(seed))
    rows_np, cols_np = w["row_sincos"], w["col_sincos"]
    pool = []
    for k in range(n_poses):
        pose = scenegen.make_pose(rng.uniform(0, 2 * np.pi), *rng.uniform(-5, 5, 2))
        td, tn = scenegen.targets_for_pose(w["scene"], pose, rows_np, cols_np, 0.1, 300 + k)
        pool.append(SV.template(S, w["means"].shape[0], rows, cols, pose, torch.from_numpy(td).to(rows.device),
                                torch.from_numpy(tn).to(rows.device)))
    cap = SV.capacity(ctx, pool, n=200)
    rate = 0.7 * cap
    stream = SV.poisson_stream(pool, n_requests, rate, grad_fraction=0.3, seed=seed)
    out = dict(requests=n_requests, rate_rps=round(rate, 1), single_capacity_rps=round(cap, 1),
               grad_fraction=0.3, max_batch=16)
    for mode in ("batched", "single"):
        SV.Service(ctx, pool, mode, max_batch=16).run(stream[:50])  # warm the per-request states
        rep = SV.Service(ctx, pool, mode, max_batch=16).run(stream)
        out[mode] = dict(p50_ms=round(rep["p50_ms"], 4), p99_ms=round(rep["p99_ms"], 4),
                         rays_per_s=round(rep["rays_per_s"], 1), mean_batch=round(rep["mean_batch"], 2))
        print(f"# service {mode}: p50 {rep['p50_ms']:.3f} ms p99 {rep['p99_ms']:.3f} ms "
              f"({rep['rays_per_s'] / 1e6:.1f} Mrays/s, mean batch {rep['mean_batch']:.1f})",
              file=sys.stderr, flush=True)
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

    m = 256
    dt = run(m)
    m2 = int(min(H * W, max(m, m * target_s / max(dt, 1e-3))))
    dt2 = run(m2)
    print(f"# cpu oracle: {m2} rays in {dt2:.1f} s", file=sys.stderr, flush=True)
    return {"value": round(m2 / dt2, 1), "unit": "rays/s", "cores": ref.threads(), "kind": "oracle",
            "sample": f"{m2} seeded random rays of the {H}x{W} image against all {w['means'].shape[0]} surfels, "
                      f"forward + loss + backward in float64 ({dt2:.1f} s)"}


if __name__ == "__main__":
    main()
