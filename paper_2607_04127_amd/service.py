"""Rendering service over several maps kept resident in HBM.

    python -m paper_2607_04127_amd.service [--requests 10000] [--fixed-rate 2000]

Requests (render only, or render + gradient with the loss of Sec. 3.4) arrive as a Poisson
stream, each for a random map, pose and beam model.  The service admits the requests that
have arrived, in arrival order, into a batch until the batch is full or its estimated HBM
working set would exceed the budget, runs the batch with ``lgsr_render_batch`` (one host
wait per request instead of a wait inside every forward, kernels of different requests
overlapping on four streams), and records each request's latency from arrival to the moment
the host sees that request's results ready (``lgsr_batch_poll``).  ``mode="single"`` serves one request per call through lgsr_forward /
lgsr_loss / lgsr_backward, the reference point.

The command-line run builds four maps (100k, 400k, 1M and 2M surfels of the seeded
street-block generator, seeds 41-44), request templates at 32 x 1024 and 64 x 1024 beams
(+-22.5 deg) and 128 x 2048 beams (+-45 deg) with exact raycast targets, measures the
single-request capacity, then serves 10,000 requests (70% render, 30% render + gradient,
stream seed 45) at 0.25, 0.5 and 0.9 times that capacity and at one fixed rate, batched and
one by one, and prints one JSON line with p50 / p99 latency and rays/s.
"""
from __future__ import annotations

import argparse
import collections
import json
import math
import sys
import time

import numpy as np
import torch

from . import lgsr

SURF_KEYS = ("means", "quats", "log_scales", "opacity_logits")
RESOLUTIONS = [(32, 1024, -22.5, 22.5), (64, 1024, -22.5, 22.5), (128, 2048, -45.0, 45.0)]


# ------------------------------------------------------------------------------------------
# maps, request templates, streams
# ------------------------------------------------------------------------------------------

def make_maps(sizes, seed=41, device="cuda:0"):
    """Maps of the street-block generator (scene and surfel seeds seed, seed + 1, ...),
    surfel scales from the 64 x 1024 beam model; parameters resident on the device."""
    import scenegen.scene as SC
    maps = []
    d_az = 2.0 * math.pi / 1024
    d_el = math.radians(45.0) / 63
    for k, n in enumerate(sizes):
        scene = SC.make_scene("block", seed + k, 400)
        surf = SC.sample_surfels(scene, n, seed + k, (-22.5, 22.5), max(d_az, d_el), 40.0, "block")
        dev = {key: torch.from_numpy(np.ascontiguousarray(surf[key])).to(device) for key in SURF_KEYS}
        maps.append(dict(n=int(n), scene=scene, surfels=dev))
    return maps


def make_pool(maps, resolutions=RESOLUTIONS, poses_per=2, seed=45, device="cuda:0"):
    """Request templates: every (map, beam model) with `poses_per` random poses (yaw U(0,
    2 pi), translation U(-5, 5) m) and exact raycast targets with 10% dropped rays."""
    import scenegen.scene as SC
    rng = np.random.Generator(np.random.PCG64(seed))
    tables = [tuple(torch.from_numpy(t).to(device) for t in SC.beam_tables(*r)) for r in resolutions]
    tables_np = [SC.beam_tables(*r) for r in resolutions]
    pool = []
    for mi, m in enumerate(maps):
        for ri, r in enumerate(resolutions):
            for _ in range(poses_per):
                pose = SC.make_pose(rng.uniform(0, 2 * np.pi), *rng.uniform(-5, 5, 2))
                td, tn = SC.targets_for_pose(m["scene"], pose, *tables_np[ri], 0.1, int(rng.integers(1 << 30)))
                pool.append(template(m["surfels"], m["n"], tables[ri][0], tables[ri][1], pose,
                                     torch.from_numpy(td).to(device), torch.from_numpy(tn).to(device), mi, ri))
    return pool


def template(surfels, n, rows, cols, pose, target_depth, target_normal, map_index=0, res_index=0):
    """One request template: a resident map (device tensors, n surfels), device beam tables,
    a host 3 x 4 pose and device targets for render + gradient requests.  `pairs` (the
    (surfel, tile) pairs of its forward) is filled in by measure_pairs."""
    H, W = rows.shape[0], cols.shape[0]
    return dict(map=map_index, res=res_index, rows=rows, cols=cols, pose=np.asarray(pose, np.float32),
                td=target_depth, tn=target_normal, rays=H * W, H=H, W=W, surfels=surfels, n=int(n), pairs=None)


def measure_pairs(ctx, pool):
    """Fill each template's `pairs` from one forward (the admission model's P)."""
    for tp in pool:
        _, st = lgsr.lgsr_forward(ctx, tp["surfels"], torch.from_numpy(tp["pose"]), tp["rows"], tp["cols"])
        tp["pairs"] = int(lgsr.lgsr_query(ctx, st)["pairs"])
        st.free()


Request = collections.namedtuple("Request", "id t template grad")


def poisson_stream(pool, n, rate, grad_fraction=0.3, seed=45):
    """n requests with exponential inter-arrival times (mean 1 / rate seconds), a uniformly
    random template each, and a gradient with probability grad_fraction."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    tpl = rng.integers(len(pool), size=n)
    grad = rng.uniform(size=n) < grad_fraction
    return [Request(i, float(t[i]), int(tpl[i]), bool(grad[i])) for i in range(n)]


# (surfel, tile) pairs per surfel assumed for a template whose forward has not been
# measured: above what the street-block maps reach at every beam model of the service
PAIRS_PER_SURFEL_BOUND = 3


def working_bytes(tpl, grad):
    """Device bytes a request holds beyond its resident map: the library's own account of its
    state and (with a gradient) its loss and backward scratch (lgsr_request_bytes), at the
    template's measured pair count or PAIRS_PER_SURFEL_BOUND per surfel, plus the frame
    outputs (21 B per ray) and, with a gradient, the per-ray loss gradient (20 B) and the
    parameter gradients (40 B per surfel)."""
    n, rays = tpl["n"], tpl["rays"]
    pairs = tpl.get("pairs")
    if pairs is None:
        pairs = PAIRS_PER_SURFEL_BOUND * n
    b = lgsr.lgsr_request_bytes(n, tpl["H"], tpl["W"], pairs, grad) + 21 * rays
    if grad:
        b += 20 * rays + 40 * n
    return b


# ------------------------------------------------------------------------------------------
# the service loop
# ------------------------------------------------------------------------------------------


class Service:
    def __init__(self, ctx: lgsr.Context, pool, mode="batched", max_batch=16, hbm_budget=32 << 30):
        """mode: "batched" (lgsr_render_batch, each request on one of four streams),
        "fused" (lgsr_render_batch with one launch per compositing stage for the whole batch)
        or "single" (one request per call).  hbm_budget: device bytes the service may use for
        requests in flight; what the context already retains (workspace and earlier batch
        states) is taken off it."""
        if mode not in ("batched", "fused", "single"):
            raise ValueError("mode must be 'batched', 'fused' or 'single'")
        self.ctx, self.pool, self.mode = ctx, pool, mode
        self.max_batch = max(1, int(max_batch)) if mode != "single" else 1
        self.opts = lgsr.default_opts(flags=lgsr.LGSR_FLAG_BATCH_FUSED if mode == "fused" else 0) \
            if ctx is not None else None
        retained = lgsr.lgsr_state_bytes(ctx, None) if ctx is not None else 0
        self.hbm_budget = max(0, int(hbm_budget) - retained)

    def _admit(self, pending):
        """Requests from the head of the queue while the batch fits (at least one)."""
        batch, total = [], 0
        while pending and len(batch) < self.max_batch:
            r = pending[0]
            b = working_bytes(self.pool[r.template], r.grad)
            if batch and total + b > self.hbm_budget:
                break
            batch.append(pending.popleft())
            total += b
        return batch

    def _execute(self, batch, t0):
        """Runs a batch; returns each request's completion time (seconds since t0), taken
        when the host sees that request's results ready."""
        if self.mode != "single" and len(batch) > 1:
            reqs = []
            for r in batch:
                tp = self.pool[r.template]
                q = dict(surfels=tp["surfels"], pose=tp["pose"], row_sincos=tp["rows"], col_sincos=tp["cols"])
                if r.grad:
                    q["target_depth"], q["target_normal"] = tp["td"], tp["tn"]
                reqs.append(q)
            lgsr.lgsr_render_batch(self.ctx, reqs, opts=self.opts)
            n = len(batch)
            done_at = [None] * n
            left = n
            while left:
                ready = lgsr.lgsr_batch_poll(self.ctx, n)
                now = time.perf_counter() - t0
                for k in range(n):
                    if ready[k] and done_at[k] is None:
                        done_at[k] = now
                        left -= 1
            torch.cuda.synchronize()
            return done_at
        # one request per call (and a batch of one in batched mode: the batch path's stream
        # joins and per-request events only pay off when requests overlap)
        done_at = []
        for r in batch:
            tp = self.pool[r.template]
            fr, st = lgsr.lgsr_forward(self.ctx, tp["surfels"], torch.from_numpy(tp["pose"]), tp["rows"],
                                       tp["cols"], want_state=r.grad)
            if r.grad:
                _, g = lgsr.lgsr_loss(self.ctx, fr, tp["td"], tp["tn"])
                lgsr.lgsr_backward(self.ctx, st, g)
                st.free()
            torch.cuda.synchronize()
            done_at.append(time.perf_counter() - t0)
        return done_at

    def run(self, stream):
        """Serve a stream in real time; returns latency percentiles and throughput."""
        pending = collections.deque()
        lat, ids, sizes = [], [], []
        rays = 0
        i, n = 0, len(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while len(ids) < n:
            now = time.perf_counter() - t0
            while i < n and stream[i].t <= now:
                pending.append(stream[i])
                i += 1
            if not pending:
                wait = stream[i].t - now
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
                continue
            batch = self._admit(pending)
            for r, done in zip(batch, self._execute(batch, t0)):
                lat.append(done - r.t)
                ids.append(r.id)
                rays += self.pool[r.template]["rays"]
            sizes.append(len(batch))
        span = time.perf_counter() - t0
        lat_ms = np.asarray(lat) * 1e3
        return dict(mode=self.mode, served=len(ids), ids=ids, p50_ms=float(np.percentile(lat_ms, 50)),
                    p99_ms=float(np.percentile(lat_ms, 99)), mean_ms=float(lat_ms.mean()),
                    rays_per_s=float(rays / span), requests_per_s=float(n / span), batches=len(sizes),
                    mean_batch=float(np.mean(sizes)), span_s=span)


def capacity(ctx, pool, n=200, seed=46):
    """Requests per second that one-request-per-call service sustains back to back."""
    stream = [Request(r.id, 0.0, r.template, r.grad) for r in poisson_stream(pool, n, 1.0, seed=seed)]
    Service(ctx, pool, "single").run(stream[: min(20, n)])  # warm the buffers
    rep = Service(ctx, pool, "single").run(stream)
    return n / rep["span_s"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=10_000)
    ap.add_argument("--sizes", default="100000,400000,1000000,2000000")
    ap.add_argument("--fractions", default="0.25,0.5,0.9")
    ap.add_argument("--fixed-rate", type=float, default=2000.0, help="requests per second")
    ap.add_argument("--max-batch", type=int, default=16)
    ap.add_argument("--poses", type=int, default=2)
    args = ap.parse_args()
    t = time.perf_counter()
    maps = make_maps([int(x) for x in args.sizes.split(",")])
    pool = make_pool(maps, poses_per=args.poses)
    print(f"# {len(maps)} maps, {len(pool)} templates ({time.perf_counter() - t:.1f} s)", file=sys.stderr, flush=True)
    ctx = lgsr.Context(0)
    measure_pairs(ctx, pool)
    cap = capacity(ctx, pool)
    print(f"# single-request capacity {cap:.1f} requests/s", file=sys.stderr, flush=True)
    runs = []
    rates = [(f"{f}x capacity", float(f) * cap) for f in args.fractions.split(",")] + [("fixed", args.fixed_rate)]
    for label, rate in rates:
        stream = poisson_stream(pool, args.requests, rate)
        for mode in ("batched", "single"):
            rep = Service(ctx, pool, mode, max_batch=args.max_batch).run(stream)
            rep.pop("ids")
            rep.update(rate_label=label, rate=rate)
            runs.append(rep)
            print(f"# {label} ({rate:.0f}/s) {mode}: p50 {rep['p50_ms']:.2f} ms p99 {rep['p99_ms']:.2f} ms "
                  f"{rep['rays_per_s'] / 1e6:.1f} Mrays/s, mean batch {rep['mean_batch']:.1f}",
                  file=sys.stderr, flush=True)
    print(json.dumps(dict(maps=[m["n"] for m in maps], templates=len(pool), capacity_rps=cap,
                          requests=args.requests, runs=runs)), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
