"""Sliding-window map and pose refinement through the differentiable renderer.

    python -m paper_2607_04127_amd.window [--iters 10] [--surfels N] [--keep auto|store|recompute]

Runs the map optimisation of Sec. 3.4 over a window of keyframes: every iteration renders
the map from each keyframe pose, takes the loss against that keyframe's range image and
normals, back-propagates through the library's backward to every surfel parameter and
to every pose, and takes one Adam step (fused kernel for the map, tangent Adam with
retraction for the poses).  The default workload is 64 x 2048 beams (-24.9..+2.0 deg),
1,000,000 surfels and 8 keyframes 1.5 m apart with yaw noise; the initial poses are
perturbed by N(0, 5 cm) and N(0, 0.5 deg) and the surfel centres by N(0, 2 cm) with a
fixed seed.  Prints one JSON line: seconds per iteration, the loss curve and the pose
errors before and after.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import autograd as AG
from . import lgsr

DEFAULT_LR = dict(means=2e-3, quats=1e-3, log_scales=5e-3, opacity_logits=2e-2)


def perturb(w: dict, seed: int = 300):
    """(perturbed poses, perturbed means): N(0, 5 cm) translation and N(0, 0.5 deg) rotation
    per pose (right perturbation), N(0, 2 cm) per surfel centre."""
    rng = np.random.Generator(np.random.PCG64(seed))
    poses = []
    for T in w["poses"]:
        xi = np.concatenate([rng.normal(0.0, 0.05, 3), rng.normal(0.0, math.radians(0.5), 3)])
        poses.append(AG.compose(T, xi))
    means = (w["means"].astype(np.float64) + rng.normal(0.0, 0.02, w["means"].shape)).astype(np.float32)
    return poses, means


def pose_errors(poses, truth):
    """(translation error m, rotation error rad) per pose."""
    out = []
    for T, G in zip(poses, truth):
        T, G = np.asarray(T, np.float64), np.asarray(G, np.float64)
        dR = G[:, :3].T @ T[:, :3]
        ang = math.acos(max(-1.0, min(1.0, (np.trace(dR) - 1.0) / 2.0)))
        out.append((float(np.linalg.norm(T[:, 3] - G[:, 3])), ang))
    return out


class Window:
    """Device-resident map parameters, per-keyframe targets and both optimisers."""

    def __init__(self, ctx: lgsr.Context, w: dict, poses, means=None, keep_lists="auto", lr=None,
                 pose_lr=(1e-3, 2e-4), hbm_budget=16 << 30, objective="basic", ns_start=0, s_max=1.0):
        """objective: "basic" (depth L1 + G-ICP normal term) or "full" (Eq. 13: also the
        opacity BCE, the rendered-surface normal term from iteration ns_start on, and the
        scale regulariser with threshold s_max)."""
        if objective not in ("basic", "full"):
            raise ValueError("objective must be 'basic' or 'full'")
        self.objective, self.ns_start, self.s_max, self.iter = objective, int(ns_start), float(s_max), 0
        dev = ctx.device
        self.ctx = ctx
        self.rows = torch.from_numpy(w["row_sincos"]).to(dev)
        self.cols = torch.from_numpy(w["col_sincos"]).to(dev)
        src = dict(means=w["means"] if means is None else means, quats=w["quats"], log_scales=w["log_scales"],
                   opacity_logits=w["opacity_logits"])
        self.params = {k: torch.from_numpy(np.ascontiguousarray(src[k])).to(dev).requires_grad_(True)
                       for k in AG.SURF_KEYS}
        self.targets = [(torch.from_numpy(td).to(dev), torch.from_numpy(tn).to(dev)) for td, tn in w["targets"]]
        self.renderer = AG.Renderer(ctx, self.rows, self.cols, keep_lists=keep_lists, hbm_budget=hbm_budget)
        self.map_opt = AG.MapAdam(ctx, self.params, lr or DEFAULT_LR)
        self.pose_opt = AG.PoseAdam(poses, *pose_lr)

    def loss_and_backward(self):
        """Sum over keyframes of the loss, then one backward (every keyframe's forward state is
        alive until then, kept or dropped for recomputation against the HBM budget);
        gradients land in .grad of the map parameters and of the pose tangents."""
        losses = []
        if self.objective == "full":
            wts = lgsr.default_objective_weights()
            if self.iter < self.ns_start:
                wts.lambda_ns = 0.0
        for k, (td, tn) in enumerate(self.targets):
            fr = AG.render(self.renderer, self.params, self.pose_opt.T0[k], self.pose_opt.xi[k])
            if self.objective == "full":
                losses.append(AG.objective(self.renderer, fr, td, tn, wts)[0])
            else:
                losses.append(AG.loss(self.renderer, fr, td, tn)[0])
        if self.objective == "full":
            losses.append(AG.scale_reg(self.ctx, self.params["log_scales"], 10.0, self.s_max))
        total = torch.stack(losses).sum()
        total.backward()
        return float(total.detach())

    def step(self):
        self.map_opt.zero_grad()
        self.pose_opt.zero_grad()
        total = self.loss_and_backward()
        self.map_opt.step()
        self.pose_opt.step()
        self.iter += 1
        return total


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--surfels", type=int, default=None)
    ap.add_argument("--keep", default="auto", choices=("auto", "store", "recompute"))
    ap.add_argument("--objective", default="basic", choices=("basic", "full"))
    ap.add_argument("--ns-start", type=int, default=5, help="iteration that enables the surface-normal term")
    args = ap.parse_args()
    import scenegen

    t0 = time.perf_counter()
    w = scenegen.make_workload("window64x2048_1m", n=args.surfels)
    print(f"# workload: N={w['means'].shape[0]} {w['H']}x{w['W']} {len(w['poses'])} poses "
          f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    poses, means = perturb(w)
    ctx = lgsr.Context(0)
    win = Window(ctx, w, poses, means=means, keep_lists=args.keep, objective=args.objective, ns_start=args.ns_start)
    err0 = pose_errors(win.pose_opt.T0, w["poses"])
    curve, times = [], []
    for it in range(args.iters):
        torch.cuda.synchronize()
        a = time.perf_counter()
        curve.append(win.step())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - a)
        print(f"# iter {it}: loss {curve[-1]:.6f} ({times[-1] * 1e3:.1f} ms)", file=sys.stderr, flush=True)
    err1 = pose_errors(win.pose_opt.T0, w["poses"])
    rays = w["H"] * w["W"] * len(w["poses"])
    out = dict(workload="window64x2048_1m", surfels=int(w["means"].shape[0]), poses=len(w["poses"]),
               iters=args.iters, keep_lists=args.keep, objective=args.objective, s_per_iter=float(np.median(times)),
               rays_per_s=float(rays / np.median(times)), loss=curve,
               recomputed_backwards=win.renderer.recomputed,
               pose_err_before=dict(t_m=float(np.mean([e[0] for e in err0])),
                                    r_deg=float(np.degrees(np.mean([e[1] for e in err0])))),
               pose_err_after=dict(t_m=float(np.mean([e[0] for e in err1])),
                                   r_deg=float(np.degrees(np.mean([e[1] for e in err1])))))
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    if os.environ.get("WORLD_SIZE", "1") != "1":
        sys.exit("one GPU only")
    main()
