"""Differentiable rendering on top of the C ABI (torch.autograd), for map and pose refinement.

``render(renderer, surfels, T0, xi)`` renders the surfel map (Sec. 3.1) under the pose
T0 * Exp(xi) and returns depth, opacity, normal (differentiable) and the ray-drop mask.
Its backward is the library's hand-written backward; the pose gradient, which the library
gives in the tangent of the right perturbation at T, is mapped to xi with the right
Jacobian of SE(3), so xi may be any tangent vector (an optimiser that retracts xi into T0
after every step keeps it at zero, where the Jacobian is the identity).

Between forward and backward the renderer either keeps the forward's state (records,
sorted per-tile lists, per-ray compositing state) or drops it and runs the forward again
in the backward (the forward is deterministic, so both give identical gradients).  With
``keep_lists="auto"`` a state is kept while the states held stay within ``hbm_budget``
bytes.

``loss(renderer, frame, target_depth, target_normal)`` is the loss of Sec. 3.4 (masked
depth L1, Eq. 10 left, plus the G-ICP normal cosine term, Eq. 11 first term) as a
differentiable scalar.  ``MapAdam`` and ``PoseAdam`` are optimisers for the map (the
library's fused Adam kernel) and for poses (Adam in the tangent, retracted every step).
"""
from __future__ import annotations

import math
import weakref

import numpy as np
import torch

from . import lgsr

SURF_KEYS = ("means", "quats", "log_scales", "opacity_logits")

# ------------------------------------------------------------------------------------------
# SE(3) in float64 on the host: xi = (rho, omega), Exp(xi) = [[R(omega), V(omega) rho], [0, 1]]
# ------------------------------------------------------------------------------------------


def hat(w) -> np.ndarray:
    w = np.asarray(w, np.float64)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def _coeffs(th: float):
    """sin(th)/th, (1 - cos th)/th^2, (th - sin th)/th^3 with series near 0."""
    if th < 1e-4:
        t2 = th * th
        return 1.0 - t2 / 6.0, 0.5 - t2 / 24.0, 1.0 / 6.0 - t2 / 120.0
    return math.sin(th) / th, (1.0 - math.cos(th)) / (th * th), (th - math.sin(th)) / (th ** 3)


def se3_exp(xi) -> np.ndarray:
    """3 x 4 [R | t] of Exp(xi), xi = (rho, omega)."""
    xi = np.asarray(xi, np.float64).reshape(6)
    rho, om = xi[:3], xi[3:]
    th = float(np.linalg.norm(om))
    a, b, c = _coeffs(th)
    W = hat(om)
    W2 = W @ W
    R = np.eye(3) + a * W + b * W2
    V = np.eye(3) + b * W + c * W2
    return np.hstack([R, (V @ rho)[:, None]])


def compose(T0, xi) -> np.ndarray:
    """T0 * Exp(xi) as 3 x 4 float64."""
    T0 = np.asarray(T0, np.float64).reshape(3, 4)
    E = se3_exp(xi)
    return np.hstack([T0[:, :3] @ E[:, :3], (T0[:, :3] @ E[:, 3] + T0[:, 3])[:, None]])


def se3_ad(xi) -> np.ndarray:
    """ad_xi = [[omega^, rho^], [0, omega^]] (6 x 6, blocks ordered (rho, omega))."""
    xi = np.asarray(xi, np.float64).reshape(6)
    out = np.zeros((6, 6))
    W = hat(xi[3:])
    out[:3, :3] = W
    out[3:, 3:] = W
    out[:3, 3:] = hat(xi[:3])
    return out


def se3_right_jacobian(xi) -> np.ndarray:
    """J_r(xi) = sum_n (-ad_xi)^n / (n + 1)!, so that Exp(xi + d) = Exp(xi) Exp(J_r d) to first
    order in d.  The series is entire; it is summed until its terms fall below 1e-18."""
    A = -se3_ad(xi)
    out = np.eye(6)
    term = np.eye(6)
    for n in range(1, 200):
        term = term @ A / (n + 1)
        out += term
        if np.abs(term).max() < 1e-18:
            break
    return out


# ------------------------------------------------------------------------------------------
# renderer and autograd functions
# ------------------------------------------------------------------------------------------


class Renderer:
    """A context, a beam model and render options, plus the store/recompute policy."""

    def __init__(self, ctx: lgsr.Context, row_sincos: torch.Tensor, col_sincos: torch.Tensor,
                 opts: lgsr.RasterOpts | None = None, keep_lists: str = "auto", hbm_budget: int = 16 << 30,
                 weights: lgsr.LossWeights | None = None):
        if keep_lists not in ("auto", "store", "recompute"):
            raise ValueError("keep_lists must be 'auto', 'store' or 'recompute'")
        self.ctx, self.rows, self.cols = ctx, row_sincos, col_sincos
        self.opts = opts if opts is not None else lgsr.default_opts()
        self.weights = weights if weights is not None else lgsr.default_loss_weights()
        self.keep_lists, self.hbm_budget = keep_lists, int(hbm_budget)
        self.held = 0        # bytes of states kept for pending backwards
        self.recomputed = 0  # backwards that ran the forward again

    @property
    def shape(self):
        return self.rows.shape[0], self.cols.shape[0]

    def _keep(self, nbytes: int) -> bool:
        if self.keep_lists == "store":
            return True
        if self.keep_lists == "recompute":
            return False
        return self.held + nbytes <= self.hbm_budget


def _pose32(T: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32))


def _release(renderer: Renderer, state: lgsr.State, nbytes: int):
    renderer.held -= nbytes
    state.free()


class _Held:
    """A state kept for a pending backward.  Its bytes return to the renderer's budget and the
    state is freed once the backward has used it, or when the autograd graph that holds it is
    dropped without a backward."""

    def __init__(self, renderer: Renderer, state: lgsr.State, nbytes: int):
        renderer.held += nbytes
        self.state = state
        self.release = weakref.finalize(self, _release, renderer, state, nbytes)


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(fctx, renderer: Renderer, T0: np.ndarray, xi: torch.Tensor, means, quats, log_scales, logits):
        xi64 = xi.detach().to("cpu", torch.float64).numpy().reshape(6)
        pose = _pose32(compose(T0, xi64))
        S = dict(means=means.detach(), quats=quats.detach(), log_scales=log_scales.detach(),
                 opacity_logits=logits.detach())
        # a backward can only follow when some input asks for a gradient
        wants_grad = any(fctx.needs_input_grad[2:])
        frame, st = lgsr.lgsr_forward(renderer.ctx, S, pose, renderer.rows, renderer.cols, opts=renderer.opts,
                                      want_state=wants_grad)
        fctx.held = None
        if wants_grad:
            nbytes = lgsr.lgsr_state_bytes(renderer.ctx, st)
            if renderer._keep(nbytes):
                fctx.held = _Held(renderer, st, nbytes)
            else:
                st.free()
        fctx.renderer, fctx.pose, fctx.xi64 = renderer, pose, xi64
        fctx.xi_meta = (xi.device, xi.dtype)
        fctx.save_for_backward(means, quats, log_scales, logits)
        fctx.mark_non_differentiable(frame["drop"])
        return frame["depth"], frame["opacity"], frame["normal"], frame["drop"]

    @staticmethod
    def backward(fctx, g_depth, g_opacity, g_normal, _g_drop):
        r: Renderer = fctx.renderer
        means, quats, log_scales, logits = fctx.saved_tensors
        H, W = r.shape
        dev = r.ctx.device
        held, fctx.held = fctx.held, None
        if held is None:
            S = dict(means=means.detach(), quats=quats.detach(), log_scales=log_scales.detach(),
                     opacity_logits=logits.detach())
            _, st = lgsr.lgsr_forward(r.ctx, S, fctx.pose, r.rows, r.cols, opts=r.opts, want_state=True)
            r.recomputed += 1
        else:
            st = held.state

        def full(g, shape):
            return torch.zeros(shape, device=dev) if g is None else g.contiguous().to(torch.float32)

        grad = dict(depth=full(g_depth, (H, W)), opacity=full(g_opacity, (H, W)), normal=full(g_normal, (H, W, 3)))
        out, gp = lgsr.lgsr_backward(r.ctx, st, grad)
        if held is None:
            st.free()
        else:
            held.release()
        Jr = torch.from_numpy(se3_right_jacobian(fctx.xi64).T.astype(np.float32)).to(dev)
        g_xi = (Jr @ gp).to(device=fctx.xi_meta[0], dtype=fctx.xi_meta[1])
        return (None, None, g_xi, out["means"], out["quats"], out["log_scales"], out["opacity_logits"])


def render(renderer: Renderer, surfels: dict, T0, xi: torch.Tensor | None = None):
    """Differentiable render under T0 * Exp(xi).  T0: 3 x 4 (array-like, sensor to world);
    xi: 6-vector tensor (rho, omega) or None (identity perturbation, no pose gradient).
    Returns dict(depth, opacity, normal, drop)."""
    if xi is None:
        xi = torch.zeros(6, dtype=torch.float64)
    T0 = np.asarray(T0, np.float64).reshape(3, 4)
    d, a, n, drop = _Render.apply(renderer, T0, xi, *(surfels[k] for k in SURF_KEYS))
    return dict(depth=d, opacity=a, normal=n, drop=drop)


class _Loss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, renderer: Renderer, depth, opacity, normal, target_depth, target_normal):
        frame = dict(depth=depth.detach().contiguous(), opacity=opacity.detach().contiguous(),
                     normal=normal.detach().contiguous())
        L, g = lgsr.lgsr_loss(renderer.ctx, frame, target_depth, target_normal, weights=renderer.weights)
        fctx.grads = g
        terms = L[1:].clone()
        fctx.mark_non_differentiable(terms)
        return L[0].clone(), terms

    @staticmethod
    def backward(fctx, gL, _gterms):
        g = fctx.grads
        return None, g["depth"] * gL, g["opacity"] * gL, g["normal"] * gL, None, None


def loss(renderer: Renderer, frame: dict, target_depth: torch.Tensor, target_normal: torch.Tensor):
    """(total loss, tensor([depth term, normal term, |Omega_D|, |Omega_N|])); the total is
    differentiable with respect to the rendered depth, opacity and normal."""
    return _Loss.apply(renderer, frame["depth"], frame["opacity"], frame["normal"], target_depth, target_normal)


class _Objective(torch.autograd.Function):
    @staticmethod
    def forward(fctx, renderer: Renderer, weights, depth, opacity, normal, target_depth, target_normal):
        frame = dict(depth=depth.detach().contiguous(), opacity=opacity.detach().contiguous(),
                     normal=normal.detach().contiguous())
        L, g = lgsr.lgsr_objective(renderer.ctx, frame, renderer.rows, renderer.cols, target_depth, target_normal,
                                   weights)
        fctx.grads = g
        terms = L[1:].clone()
        fctx.mark_non_differentiable(terms)
        return L[0].clone(), terms

    @staticmethod
    def backward(fctx, gL, _gterms):
        g = fctx.grads
        return None, None, g["depth"] * gL, g["opacity"] * gL, g["normal"] * gL, None, None


def objective(renderer: Renderer, frame: dict, target_depth: torch.Tensor, target_normal: torch.Tensor,
              weights: lgsr.ObjectiveWeights | None = None):
    """Frame terms of the full objective (Eq. 10-11 weighted as in Eq. 13): (total, tensor(
    [depth, opacity, G-ICP normal, surface normal terms, |Omega_D|, |Omega_N|, |Omega_S|]));
    the total is differentiable with respect to the rendered depth, opacity and normal."""
    w = weights if weights is not None else lgsr.default_objective_weights()
    return _Objective.apply(renderer, w, frame["depth"], frame["opacity"], frame["normal"], target_depth,
                            target_normal)


class _ScaleReg(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx: lgsr.Context, lambda_s: float, s_max: float, log_scales):
        g = torch.zeros_like(log_scales)
        L = lgsr.lgsr_scale_reg(ctx, log_scales.detach().contiguous(), lambda_s, s_max, grad_log_scales=g)
        fctx.g = g
        return L[0].clone()

    @staticmethod
    def backward(fctx, gL):
        return None, None, None, fctx.g * gL


def scale_reg(ctx: lgsr.Context, log_scales: torch.Tensor, lambda_s: float = 10.0, s_max: float = 1.0):
    """lambda_s sum_i max(0, max(s_i) - s_max) (Eq. 12), differentiable in log_scales."""
    return _ScaleReg.apply(ctx, float(lambda_s), float(s_max), log_scales)


# ------------------------------------------------------------------------------------------
# optimisers
# ------------------------------------------------------------------------------------------


class MapAdam:
    """Adam over the surfel parameters with the library's fused kernel (one launch per step)."""

    def __init__(self, ctx: lgsr.Context, surfels: dict, lr: dict, betas=(0.9, 0.999), eps=1e-15):
        self.ctx, self.params, self.lr = ctx, surfels, dict(lr)
        self.betas, self.eps, self.t = betas, eps, 0
        self.m = {k: torch.zeros_like(surfels[k]) for k in SURF_KEYS}
        self.v = {k: torch.zeros_like(surfels[k]) for k in SURF_KEYS}

    @torch.no_grad()
    def step(self):
        self.t += 1
        groups = []
        for k in SURF_KEYS:
            p = self.params[k]
            if p.grad is None or self.lr.get(k, 0.0) == 0.0:
                continue
            groups.append((p.data, p.grad.contiguous(), self.m[k], self.v[k], self.lr[k]))
        if groups:
            lgsr.lgsr_adam_step(self.ctx, groups, self.t, self.betas[0], self.betas[1], self.eps)

    def zero_grad(self):
        for k in SURF_KEYS:
            self.params[k].grad = None


class PoseAdam:
    """Adam on pose tangents xi (K x 6, float64 on the host), retracted into the base poses
    after every step: T0_k <- T0_k Exp(xi_k), xi_k <- 0 (moments stay in the tangent)."""

    def __init__(self, poses, lr_rho: float, lr_omega: float, betas=(0.9, 0.999), eps=1e-12):
        self.T0 = [np.asarray(T, np.float64).reshape(3, 4).copy() for T in poses]
        K = len(self.T0)
        self.xi = torch.zeros((K, 6), dtype=torch.float64, requires_grad=True)
        self.lr = np.array([lr_rho] * 3 + [lr_omega] * 3)
        self.betas, self.eps, self.t = betas, eps, 0
        self.m = np.zeros((K, 6))
        self.v = np.zeros((K, 6))

    @torch.no_grad()
    def step(self):
        if self.xi.grad is None:
            return
        self.t += 1
        g = self.xi.grad.numpy()
        b1, b2 = self.betas
        self.m = b1 * self.m + (1 - b1) * g
        self.v = b2 * self.v + (1 - b2) * g * g
        mh = self.m / (1 - b1 ** self.t)
        vh = self.v / (1 - b2 ** self.t)
        step = -self.lr * mh / (np.sqrt(vh) + self.eps)
        xi = self.xi.detach().numpy()
        for k in range(len(self.T0)):
            self.T0[k] = compose(self.T0[k], xi[k] + step[k])
        self.xi.zero_()

    def zero_grad(self):
        self.xi.grad = None
