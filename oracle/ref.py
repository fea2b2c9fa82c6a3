"""numpy front end of the FP64 oracle library (test infrastructure; see lgsr_ref.h).

Inputs may be float32 or float64; they are promoted exactly to float64.  Threshold
parameters are rounded to float32 first so that the oracle tests exactly the threshold
values the float32 renderer receives.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

DEFAULT_PARAMS = dict(cutoff_sigma=3.0, alpha_thr=1.0 / 255.0, alpha_max=0.99, T_min=1e-4,
                      near=0.2, den_eps=1e-6, drop_tau=0.5)
DEFAULT_WEIGHTS = dict(w_depth=1.0, lambda_n=1.0, lambda_ng=0.05)
# Eq. 13 weights of Sec. 4.1; eps (Eq. 10) and s_max (Eq. 12) are not given numerically
DEFAULT_OBJECTIVE = dict(w_depth=1.0, lambda_alpha=0.1, eps=1e-6, lambda_n=1.0, lambda_ng=0.05, lambda_ns=0.01)
DEFAULT_SCALE_REG = dict(lambda_s=10.0, s_max=1.0)


class _Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("cutoff_sigma", "alpha_thr", "alpha_max", "T_min", "near", "den_eps", "drop_tau")]


class _Map(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("log_scales", ctypes.c_void_p), ("opacity_logits", ctypes.c_void_p)]


class _Beams(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("row_sincos", ctypes.c_void_p),
                ("col_sincos", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        # LGSR_REF_LIB names another build of the oracle (the mutation tests use it)
        path = os.environ.get("LGSR_REF_LIB") or _build.LIB
        src = os.path.join(_build.HERE, "lgsr_ref.c")
        if path == _build.LIB and (not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src)):
            _build.build()
        L = ctypes.CDLL(path)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        L.lgsr_ref_forward.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.lgsr_ref_forward.restype = ctypes.c_int
        L.lgsr_ref_loss.argtypes = [i64, vp, vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, vp, vp, vp, vp]
        L.lgsr_ref_loss.restype = ctypes.c_int
        L.lgsr_ref_backward.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.lgsr_ref_backward.restype = ctypes.c_int
        L.lgsr_ref_threads.restype = ctypes.c_int
        L.lgsr_ref_surf_normal.argtypes = [vp, vp, vp, vp, vp]
        L.lgsr_ref_surf_normal.restype = ctypes.c_int
        d = ctypes.c_double
        L.lgsr_ref_objective.argtypes = [vp, vp, vp, vp, vp, vp, d, d, d, d, d, d, vp, vp, vp, vp]
        L.lgsr_ref_objective.restype = ctypes.c_int
        L.lgsr_ref_scale_reg.argtypes = [i64, vp, d, d, vp, vp, vp]
        L.lgsr_ref_scale_reg.restype = ctypes.c_int
        L.lgsr_ref_scan_to_range.argtypes = [i64, vp, vp, ctypes.c_int32, ctypes.c_int32, d, d, d, d, vp, vp, vp, vp]
        L.lgsr_ref_scan_to_range.restype = ctypes.c_int
        L.lgsr_ref_target_cov.argtypes = [i64, vp, vp, d, vp]
        L.lgsr_ref_target_cov.restype = ctypes.c_int
        L.lgsr_ref_set_threads.argtypes = [ctypes.c_int]
        L.lgsr_ref_set_threads.restype = None
        L.lgsr_ref_order.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lgsr_ref_order.restype = ctypes.c_int
        L.lgsr_ref_contributors.argtypes = [vp, vp, vp, vp, i64, vp, vp, i64, vp]
        L.lgsr_ref_contributors.restype = ctypes.c_int
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().lgsr_ref_threads())


def set_threads(n: int) -> None:
    """Threads of later oracle calls (OpenMP)."""
    lib().lgsr_ref_set_threads(int(n))


def params(**kw) -> dict:
    p = dict(DEFAULT_PARAMS)
    p.update(kw)
    return {k: float(np.float32(v)) for k, v in p.items()}


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _Inputs:
    """Keeps the float64 copies alive for the duration of a call."""

    def __init__(self, surfels, pose, row_sincos, col_sincos, prm):
        self.means = _f64(surfels["means"]).reshape(-1, 3)
        self.quats = _f64(surfels["quats"]).reshape(-1, 4)
        self.log_scales = _f64(surfels["log_scales"]).reshape(-1, 2)
        self.logits = _f64(surfels["opacity_logits"]).reshape(-1)
        n = self.means.shape[0]
        assert self.quats.shape[0] == n and self.log_scales.shape[0] == n and self.logits.shape[0] == n
        self.pose = _f64(pose).reshape(12)
        self.rows = _f64(row_sincos).reshape(-1, 2)
        self.cols = _f64(col_sincos).reshape(-1, 2)
        self.H, self.W = self.rows.shape[0], self.cols.shape[0]
        self.map = _Map(n, _ptr(self.means), _ptr(self.quats), _ptr(self.log_scales), _ptr(self.logits))
        self.beams = _Beams(self.H, self.W, _ptr(self.rows), _ptr(self.cols))
        self.prm = _Params(**params(**(prm or {})))
        self.n = n


def _rays(inp, ray_ids):
    if ray_ids is None:
        return inp.H * inp.W, None
    ids = np.ascontiguousarray(np.asarray(ray_ids, dtype=np.int64).reshape(-1))
    return ids.shape[0], ids


def forward(surfels, pose, row_sincos, col_sincos, prm=None, ray_ids=None, extra=False):
    """Render (all rays, or ``ray_ids`` = k * W + j).  Returns float64 arrays: depth, opacity,
    normal (n,3), drop (uint8), t_final, K; with ``extra`` also margin, order_gap, n_hits and
    den_min."""
    inp = _Inputs(surfels, pose, row_sincos, col_sincos, prm)
    n_rays, ids = _rays(inp, ray_ids)
    out = dict(depth=np.zeros(n_rays), opacity=np.zeros(n_rays), normal=np.zeros((n_rays, 3)),
               drop=np.zeros(n_rays, np.uint8), t_final=np.zeros(n_rays), K=np.zeros(n_rays, np.int32))
    if extra:
        out["margin"] = np.zeros(n_rays)
        out["order_gap"] = np.zeros(n_rays)
        out["n_hits"] = np.zeros(n_rays, np.int32)
        out["den_min"] = np.zeros(n_rays)
    rc = lib().lgsr_ref_forward(ctypes.byref(inp.map), _ptr(inp.pose), ctypes.byref(inp.beams),
                                ctypes.byref(inp.prm), n_rays, _ptr(ids), _ptr(out["depth"]),
                                _ptr(out["opacity"]), _ptr(out["normal"]), _ptr(out["drop"]),
                                _ptr(out["t_final"]), _ptr(out["K"]), _ptr(out.get("margin")),
                                _ptr(out.get("order_gap")), _ptr(out.get("n_hits")), _ptr(out.get("den_min")))
    if rc != 0:
        raise ValueError("lgsr_ref_forward rejected its arguments")
    return out


def order(surfels, pose, prm=None):
    """(order, range): the rendering surfels in compositing order and their FP64 centre
    ranges."""
    row = np.zeros((1, 2))
    inp = _Inputs(surfels, pose, row, row, prm)
    o = np.zeros(max(1, inp.n), np.int64)
    r = np.zeros(max(1, inp.n))
    m = ctypes.c_int64(0)
    rc = lib().lgsr_ref_order(ctypes.byref(inp.map), _ptr(inp.pose), ctypes.byref(inp.prm), _ptr(o), _ptr(r),
                              ctypes.byref(m))
    if rc != 0:
        raise ValueError("lgsr_ref_order rejected its arguments")
    return o[:m.value], r[:m.value]


def contributors(surfels, pose, row_sincos, col_sincos, ray_ids, prm=None, cap=256):
    """Per ray of ray_ids: the composited surfel ids front to back (list of int64 arrays)."""
    inp = _Inputs(surfels, pose, row_sincos, col_sincos, prm)
    n_rays, ids = _rays(inp, ray_ids)
    out = np.zeros((max(1, n_rays), cap), np.int64)
    cnt = np.zeros(max(1, n_rays), np.int32)
    rc = lib().lgsr_ref_contributors(ctypes.byref(inp.map), _ptr(inp.pose), ctypes.byref(inp.beams),
                                     ctypes.byref(inp.prm), n_rays, _ptr(ids), _ptr(out), cap, _ptr(cnt))
    if rc != 0:
        raise ValueError("lgsr_ref_contributors rejected its arguments")
    if np.any(cnt[:n_rays] > cap):
        raise ValueError("more contributors than cap")
    return [out[i, :cnt[i]].copy() for i in range(n_rays)]


def loss(pred, target_depth, target_normal, weights=None, ray_weight=None):
    """Loss and its gradient w.r.t. the rendered (depth, opacity, normal).  Returns
    (loss[5] = total, depth term, normal term, |Omega_D|, |Omega_N|; g_depth, g_opacity, g_normal)."""
    w = dict(DEFAULT_WEIGHTS)
    w.update(weights or {})
    w = {k: float(np.float32(v)) for k, v in w.items()}
    depth = _f64(pred["depth"]).reshape(-1)
    n = depth.shape[0]
    opacity = _f64(pred["opacity"]).reshape(-1)
    normal = _f64(pred["normal"]).reshape(-1, 3)
    td = _f64(target_depth).reshape(-1)
    tn = _f64(target_normal).reshape(-1, 3)
    rw = None if ray_weight is None else _f64(ray_weight).reshape(-1)
    out = np.zeros(5)
    gd, go, gn = np.zeros(n), np.zeros(n), np.zeros((n, 3))
    rc = lib().lgsr_ref_loss(n, _ptr(depth), _ptr(opacity), _ptr(normal), _ptr(td), _ptr(tn), _ptr(rw),
                             w["w_depth"], w["lambda_n"], w["lambda_ng"], _ptr(out), _ptr(gd), _ptr(go),
                             _ptr(gn))
    if rc != 0:
        raise ValueError("lgsr_ref_loss rejected its arguments")
    return out, gd, go, gn


def backward(surfels, pose, row_sincos, col_sincos, g_depth, g_opacity, g_normal, prm=None,
             ray_ids=None, with_mass=False):
    """Gradients of sum(g . rendered) w.r.t. means, quats, log_scales, opacity_logits and the
    pose tangent (rho, omega) of the right perturbation.  With ``with_mass`` also ``mass``
    (n, 4): per surfel the sum over rays of the norm of each ray's contribution to the
    means / quats / log_scales / opacity_logit gradient, and ``pose_mass`` (6,)."""
    inp = _Inputs(surfels, pose, row_sincos, col_sincos, prm)
    n_rays, ids = _rays(inp, ray_ids)
    gd = _f64(g_depth).reshape(-1)
    go = _f64(g_opacity).reshape(-1)
    gn = _f64(g_normal).reshape(-1, 3)
    assert gd.shape[0] == n_rays and go.shape[0] == n_rays and gn.shape[0] == n_rays
    n = inp.n
    out = dict(means=np.zeros((n, 3)), quats=np.zeros((n, 4)), log_scales=np.zeros((n, 2)),
               opacity_logits=np.zeros(n), pose=np.zeros(6))
    if with_mass:
        out["mass"] = np.zeros((n, 4))
        out["pose_mass"] = np.zeros(6)
    rc = lib().lgsr_ref_backward(ctypes.byref(inp.map), _ptr(inp.pose), ctypes.byref(inp.beams),
                                 ctypes.byref(inp.prm), n_rays, _ptr(ids), _ptr(gd), _ptr(go), _ptr(gn),
                                 _ptr(out["means"]), _ptr(out["quats"]), _ptr(out["log_scales"]),
                                 _ptr(out["opacity_logits"]), _ptr(out["pose"]), _ptr(out.get("mass")),
                                 _ptr(out.get("pose_mass")))
    if rc != 0:
        raise ValueError("lgsr_ref_backward rejected its arguments")
    return out


def loss_and_grad(surfels, pose, row_sincos, col_sincos, target_depth, target_normal, prm=None,
                  weights=None, ray_ids=None, ray_weight=None):
    """Forward + loss + backward in one call (float64 throughout)."""
    fw = forward(surfels, pose, row_sincos, col_sincos, prm, ray_ids)
    td = np.asarray(target_depth).reshape(-1)
    tn = np.asarray(target_normal).reshape(-1, 3)
    if ray_ids is not None:
        td, tn = td[np.asarray(ray_ids)], tn[np.asarray(ray_ids)]
    L, gd, go, gn = loss(fw, td, tn, weights, ray_weight)
    g = backward(surfels, pose, row_sincos, col_sincos, gd, go, gn, prm, ray_ids)
    return L, fw, g


def _beams(row_sincos, col_sincos):
    rows = _f64(row_sincos).reshape(-1, 2)
    cols = _f64(col_sincos).reshape(-1, 2)
    return rows, cols, _Beams(rows.shape[0], cols.shape[0], _ptr(rows), _ptr(cols))


def surf_normal(row_sincos, col_sincos, depth):
    """N_surf of a rendered H x W range image: (normals (H*W, 3), defined (H*W,) uint8,
    flip_margin (H*W,))."""
    rows, cols, B = _beams(row_sincos, col_sincos)
    n = rows.shape[0] * cols.shape[0]
    d = _f64(depth).reshape(-1)
    assert d.shape[0] == n
    ns, ok, fm = np.zeros((n, 3)), np.zeros(n, np.uint8), np.zeros(n)
    if lib().lgsr_ref_surf_normal(ctypes.byref(B), _ptr(d), _ptr(ns), _ptr(ok), _ptr(fm)) != 0:
        raise ValueError("lgsr_ref_surf_normal rejected its arguments")
    return ns, ok, fm


def objective(row_sincos, col_sincos, pred, target_depth, target_normal, weights=None, grad=True):
    """Frame terms of the full objective over the H x W image.  Returns (loss[8] = total,
    depth, opacity, G-ICP normal and surface normal terms, |Omega_D|, |Omega_N|, |Omega_S|;
    g_depth, g_opacity, g_normal) (gradients None when grad is False).  Weights are rounded
    to float32 like the ones the renderer receives."""
    w = dict(DEFAULT_OBJECTIVE)
    w.update(weights or {})
    w = {k: float(np.float32(v)) for k, v in w.items()}
    rows, cols, B = _beams(row_sincos, col_sincos)
    n = rows.shape[0] * cols.shape[0]
    depth = _f64(pred["depth"]).reshape(-1)
    opacity = _f64(pred["opacity"]).reshape(-1)
    normal = _f64(pred["normal"]).reshape(-1, 3)
    td = _f64(target_depth).reshape(-1)
    tn = _f64(target_normal).reshape(-1, 3)
    assert depth.shape[0] == n and opacity.shape[0] == n and normal.shape[0] == n and td.shape[0] == n
    out = np.zeros(8)
    g = (np.zeros(n), np.zeros(n), np.zeros((n, 3))) if grad else (None, None, None)
    rc = lib().lgsr_ref_objective(ctypes.byref(B), _ptr(depth), _ptr(opacity), _ptr(normal), _ptr(td), _ptr(tn),
                                  w["w_depth"], w["lambda_alpha"], w["eps"], w["lambda_n"], w["lambda_ng"],
                                  w["lambda_ns"], _ptr(out), *(_ptr(x) for x in g))
    if rc != 0:
        raise ValueError("lgsr_ref_objective rejected its arguments")
    return (out,) + g


def scale_reg(log_scales, lambda_s=None, s_max=None):
    """Scale regulariser: (loss, g_log_scales (n, 2), margin (n,))."""
    ls = _f64(log_scales).reshape(-1, 2)
    lam = float(np.float32(DEFAULT_SCALE_REG["lambda_s"] if lambda_s is None else lambda_s))
    smax = float(np.float32(DEFAULT_SCALE_REG["s_max"] if s_max is None else s_max))
    n = ls.shape[0]
    loss = np.zeros(1)
    g, m = np.zeros((n, 2)), np.zeros(n)
    if lib().lgsr_ref_scale_reg(n, _ptr(ls), lam, smax, _ptr(loss), _ptr(g), _ptr(m)) != 0:
        raise ValueError("lgsr_ref_scale_reg rejected its arguments")
    return float(loss[0]), g, m


def scan_to_range(points, H, W, el_min, el_max, r_min=0.0, r_max=float("inf"), normals=None):
    """Spherical range image of a scan (angles in radians): dict(depth (H*W,), normal (H*W,3),
    index (H*W,) int64, bin_margin (n,)).  Grid parameters are rounded to float32 like the
    ones the GPU receives."""
    pts = _f64(points).reshape(-1, 3)
    n = pts.shape[0]
    nrm = None if normals is None else _f64(normals).reshape(-1, 3)
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    out = dict(depth=np.zeros(H * W), normal=np.zeros((H * W, 3)), index=np.zeros(H * W, np.int64),
               bin_margin=np.zeros(n))
    rc = lib().lgsr_ref_scan_to_range(n, _ptr(pts), _ptr(nrm), H, W, f32(el_min), f32(el_max), f32(r_min),
                                      f32(r_max), _ptr(out["depth"]), _ptr(out["normal"]), _ptr(out["index"]),
                                      _ptr(out["bin_margin"]))
    if rc != 0:
        raise ValueError("lgsr_ref_scan_to_range rejected its arguments")
    return out


def target_cov(quats, log_scales, eps=0.01):
    """Surfel target covariances (n, 6): xx, xy, xz, yy, yz, zz."""
    q = _f64(quats).reshape(-1, 4)
    ls = _f64(log_scales).reshape(-1, 2)
    cov = np.zeros((q.shape[0], 6))
    if lib().lgsr_ref_target_cov(q.shape[0], _ptr(q), _ptr(ls), float(np.float32(eps)), _ptr(cov)) != 0:
        raise ValueError("lgsr_ref_target_cov rejected its arguments")
    return cov
