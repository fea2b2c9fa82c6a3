"""ctypes binding of the gfx950 renderer library (include/lgsr.h), same entry-point names.

Argument marshalling only: tensors are checked (device, dtype, shape, contiguity), their
device pointers and torch's current HIP stream are handed to the C ABI, and outputs are
allocated with torch.  Every step of the rendering path runs in the library's kernels;
there is no fallback.  If the library is not built, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# LGSR_LIB names another build of the library (the sanitizer test loads a host-sanitized one)
LIB_PATH = os.environ.get("LGSR_LIB") or os.path.join(HERE, "liblgsr.so")

LGSR_FLAG_BATCH_FUSED = 1
LGSR_OK, LGSR_EINVAL, LGSR_ENOMEM, LGSR_EDEVICE, LGSR_ECAPACITY, LGSR_ESTATE, LGSR_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ECAPACITY", -5: "ESTATE", -6: "EINTERNAL"}

EXPORTS = ("lgsr_default_opts", "lgsr_default_loss_weights", "lgsr_create", "lgsr_destroy", "lgsr_set_stream",
           "lgsr_last_error", "lgsr_forward", "lgsr_loss", "lgsr_backward", "lgsr_state_free", "lgsr_query",
           "lgsr_profile", "lgsr_profile_read", "lgsr_sync", "lgsr_state_bytes", "lgsr_adam_step",
           "lgsr_render_batch", "lgsr_default_objective_weights", "lgsr_objective", "lgsr_scale_reg",
           "lgsr_scan_to_range", "lgsr_target_cov", "lgsr_tile_list", "lgsr_loss_noalloc",
           "lgsr_stream_probe", "lgsr_count_hits", "lgsr_batch_poll", "lgsr_request_bytes")
STAGES = ("project", "scan", "readback", "emit", "tile_sort", "raster_fwd", "loss", "bwd_prep", "raster_bwd",
          "chain")


class LgsrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


vp = ctypes.c_void_p


class Surfels(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means", vp), ("quats", vp), ("log_scales", vp), ("opacity_logits", vp)]


class Beams(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("row_sincos", vp), ("col_sincos", vp)]


class RasterOpts(ctypes.Structure):
    _fields_ = [("cutoff_sigma", ctypes.c_float), ("alpha_thr", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("T_min", ctypes.c_float), ("near", ctypes.c_float), ("den_eps", ctypes.c_float),
                ("drop_tau", ctypes.c_float), ("chunk", ctypes.c_int32), ("flags", ctypes.c_int32)]


class Frame(ctypes.Structure):
    _fields_ = [("depth", vp), ("opacity", vp), ("normal", vp), ("drop", vp)]


class LossWeights(ctypes.Structure):
    _fields_ = [("w_depth", ctypes.c_float), ("lambda_n", ctypes.c_float), ("lambda_ng", ctypes.c_float)]


class ObjectiveWeights(ctypes.Structure):
    _fields_ = [(k, ctypes.c_float) for k in ("w_depth", "lambda_alpha", "eps", "lambda_n", "lambda_ng", "lambda_ns")]


class ScanGrid(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("el_min", ctypes.c_float), ("el_max", ctypes.c_float),
                ("r_min", ctypes.c_float), ("r_max", ctypes.c_float)]


class FrameGrad(ctypes.Structure):
    _fields_ = [("d_depth", vp), ("d_opacity", vp), ("d_normal", vp)]


class SurfelGrads(ctypes.Structure):
    _fields_ = [("means", vp), ("quats", vp), ("log_scales", vp), ("opacity_logits", vp)]


class Request(ctypes.Structure):
    _fields_ = [("surfels", Surfels), ("pose_ws", ctypes.c_float * 12), ("beams", Beams), ("out", Frame),
                ("target_depth", vp), ("target_normal", vp), ("loss_out", vp), ("frame_grad", FrameGrad),
                ("grads", SurfelGrads), ("grad_pose", vp)]


class AdamGroup(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("param", vp), ("grad", vp), ("m", vp), ("v", vp), ("lr", ctypes.c_float)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2607_04127_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.lgsr_default_opts.argtypes = [P(RasterOpts)]
        L.lgsr_default_opts.restype = None
        L.lgsr_default_loss_weights.argtypes = [P(LossWeights)]
        L.lgsr_default_loss_weights.restype = None
        L.lgsr_create.argtypes = [P(vp), ctypes.c_int, vp]
        L.lgsr_destroy.argtypes = [vp]
        L.lgsr_destroy.restype = None
        L.lgsr_set_stream.argtypes = [vp, vp]
        L.lgsr_last_error.argtypes = [vp]
        L.lgsr_last_error.restype = ctypes.c_char_p
        L.lgsr_forward.argtypes = [vp, P(Surfels), vp, ctypes.c_int32, P(Beams), P(RasterOpts), P(Frame), P(vp)]
        L.lgsr_loss.argtypes = [vp, ctypes.c_int64, P(Frame), vp, vp, P(LossWeights), vp, P(FrameGrad)]
        L.lgsr_loss_noalloc.argtypes = [vp, ctypes.c_int64, P(Frame), vp, vp, P(LossWeights), vp, P(FrameGrad)]
        L.lgsr_stream_probe.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.c_int64, ctypes.c_int32]
        L.lgsr_count_hits.argtypes = [vp, vp, P(ctypes.c_int64)]
        L.lgsr_batch_poll.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int32)]
        L.lgsr_request_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                         ctypes.c_int32, P(ctypes.c_int64)]
        L.lgsr_backward.argtypes = [vp, vp, P(FrameGrad), P(SurfelGrads), vp]
        L.lgsr_state_free.argtypes = [vp]
        L.lgsr_state_free.restype = None
        L.lgsr_query.argtypes = [vp, vp, P(ctypes.c_int64)]
        L.lgsr_sync.argtypes = [vp]
        L.lgsr_profile.argtypes = [vp, ctypes.c_int32]
        L.lgsr_profile_read.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_int64)]
        L.lgsr_state_bytes.argtypes = [vp, vp, P(ctypes.c_int64)]
        L.lgsr_render_batch.argtypes = [vp, ctypes.c_int32, P(Request), P(RasterOpts), P(LossWeights)]
        L.lgsr_adam_step.argtypes = [vp, ctypes.c_int32, P(AdamGroup), ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_int32]
        L.lgsr_default_objective_weights.argtypes = [P(ObjectiveWeights)]
        L.lgsr_default_objective_weights.restype = None
        L.lgsr_objective.argtypes = [vp, P(Beams), P(Frame), vp, vp, P(ObjectiveWeights), vp, P(FrameGrad)]
        L.lgsr_scale_reg.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_float, ctypes.c_float, vp, vp]
        L.lgsr_scan_to_range.argtypes = [vp, ctypes.c_int64, vp, vp, P(ScanGrid), vp, vp, vp]
        L.lgsr_target_cov.argtypes = [vp, ctypes.c_int64, vp, vp, ctypes.c_float, vp]
        L.lgsr_tile_list.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int64,
                                     P(ctypes.c_int64)]
        for name in ("lgsr_create", "lgsr_set_stream", "lgsr_forward", "lgsr_loss", "lgsr_backward", "lgsr_query",
                     "lgsr_profile", "lgsr_profile_read", "lgsr_sync", "lgsr_state_bytes", "lgsr_adam_step",
                     "lgsr_render_batch", "lgsr_objective", "lgsr_scale_reg", "lgsr_scan_to_range",
                     "lgsr_target_cov", "lgsr_tile_list", "lgsr_loss_noalloc", "lgsr_stream_probe",
                     "lgsr_count_hits", "lgsr_batch_poll", "lgsr_request_bytes"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def default_opts(**kw) -> RasterOpts:
    o = RasterOpts()
    lib().lgsr_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_loss_weights(**kw) -> LossWeights:
    w = LossWeights()
    lib().lgsr_default_loss_weights(ctypes.byref(w))
    for k, v in kw.items():
        setattr(w, k, v)
    return w


def default_objective_weights(**kw) -> ObjectiveWeights:
    w = ObjectiveWeights()
    lib().lgsr_default_objective_weights(ctypes.byref(w))
    for k, v in kw.items():
        setattr(w, k, v)
    return w


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, name: str, shape, device, dtype=torch.float32):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    """Owns an lgsr_ctx on one device; calls follow torch's current stream."""

    def __init__(self, device: int | torch.device = 0):
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.device = dev
        h = vp()
        with torch.cuda.device(dev):
            st = lib().lgsr_create(ctypes.byref(h), dev.index or 0, vp(torch.cuda.current_stream(dev).cuda_stream))
        if st != LGSR_OK:
            raise LgsrError(st, "lgsr_create failed")
        self.handle = h
        self._states = weakref.WeakSet()

    def _check(self, st: int):
        if st != LGSR_OK:
            raise LgsrError(st, lib().lgsr_last_error(self.handle).decode())

    def _stream(self):
        self._check(lib().lgsr_set_stream(self.handle, vp(torch.cuda.current_stream(self.device).cuda_stream)))

    def close(self):
        if getattr(self, "handle", None):
            for st in list(self._states):  # destroying the context invalidates its states
                st.handle = None
            lib().lgsr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class State:
    def __init__(self, ctx: Context, handle, keep):
        self.ctx, self.handle, self._keep = ctx, handle, keep
        ctx._states.add(self)

    def free(self):
        if self.handle and self.ctx.handle:
            lib().lgsr_state_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _surfels(ctx, S):
    n = S["means"].shape[0]
    d = ctx.device
    m = _dev(S["means"], "means", (n, 3), d)
    q = _dev(S["quats"], "quats", (n, 4), d)
    ls = _dev(S["log_scales"], "log_scales", (n, 2), d)
    lo = _dev(S["opacity_logits"], "opacity_logits", (n,), d)
    return Surfels(n, _ptr(m), _ptr(q), _ptr(ls), _ptr(lo)), (m, q, ls, lo)


def lgsr_forward(ctx: Context, surfels: dict, pose: torch.Tensor, row_sincos: torch.Tensor, col_sincos: torch.Tensor,
                 opts: RasterOpts | None = None, want_state: bool = True, out: dict | None = None):
    """Render.  ``pose`` is a float32 (3, 4) tensor on the CPU (host) or on the context's device.
    Returns (frame dict: depth (H,W), opacity (H,W), normal (H,W,3), drop (H,W) uint8; State or None)."""
    d = ctx.device
    H, W = row_sincos.shape[0], col_sincos.shape[0]
    _dev(row_sincos, "row_sincos", (H, 2), d)
    _dev(col_sincos, "col_sincos", (W, 2), d)
    if pose.dtype != torch.float32 or tuple(pose.shape) != (3, 4) or not pose.is_contiguous():
        raise ValueError("pose must be a contiguous float32 (3, 4) tensor")
    if pose.device.type == "cpu":
        on_dev = 0
    elif pose.device == d:
        on_dev = 1
    else:
        raise ValueError(f"pose must be on the CPU or on {d}")
    s, keep = _surfels(ctx, surfels)
    if out is None:
        out = dict(depth=torch.empty((H, W), device=d), opacity=torch.empty((H, W), device=d),
                   normal=torch.empty((H, W, 3), device=d), drop=torch.empty((H, W), device=d, dtype=torch.uint8))
    else:
        _dev(out["depth"], "depth", (H, W), d)
        _dev(out["opacity"], "opacity", (H, W), d)
        _dev(out["normal"], "normal", (H, W, 3), d)
        _dev(out["drop"], "drop", (H, W), d, torch.uint8)
    fr = Frame(_ptr(out["depth"]), _ptr(out["opacity"]), _ptr(out["normal"]), _ptr(out["drop"]))
    bm = Beams(H, W, _ptr(row_sincos), _ptr(col_sincos))
    o = opts if opts is not None else default_opts()
    h = vp()
    ctx._stream()
    ctx._check(lib().lgsr_forward(ctx.handle, ctypes.byref(s), _ptr(pose), on_dev, ctypes.byref(bm), ctypes.byref(o),
                                  ctypes.byref(fr), ctypes.byref(h) if want_state else None))
    state = State(ctx, h, (keep, row_sincos, col_sincos, pose)) if want_state else None
    return out, state


def lgsr_loss(ctx: Context, frame: dict, target_depth: torch.Tensor, target_normal: torch.Tensor,
              weights: LossWeights | None = None, loss_out: torch.Tensor | None = None, grad_out: dict | None = None):
    """Loss (float32[5] on the device: total, depth term, normal term, |Omega_D|, |Omega_N|)
    and dL/d(depth, opacity, normal)."""
    d = ctx.device
    H, W = frame["depth"].shape
    n = H * W
    _dev(frame["depth"], "depth", (H, W), d)
    _dev(frame["normal"], "normal", (H, W, 3), d)
    _dev(target_depth, "target_depth", (H, W), d)
    _dev(target_normal, "target_normal", (H, W, 3), d)
    if loss_out is None:
        loss_out = torch.empty(5, device=d)
    _dev(loss_out, "loss_out", (5,), d)
    if grad_out is None:
        grad_out = dict(depth=torch.empty((H, W), device=d), opacity=torch.empty((H, W), device=d),
                        normal=torch.empty((H, W, 3), device=d))
    fr = Frame(_ptr(frame["depth"]), _ptr(frame.get("opacity")), _ptr(frame["normal"]), None)
    fg = FrameGrad(_ptr(grad_out["depth"]), _ptr(grad_out["opacity"]), _ptr(grad_out["normal"]))
    w = weights if weights is not None else default_loss_weights()
    ctx._stream()
    ctx._check(lib().lgsr_loss(ctx.handle, n, ctypes.byref(fr), _ptr(target_depth), _ptr(target_normal),
                               ctypes.byref(w), _ptr(loss_out), ctypes.byref(fg)))
    return loss_out, grad_out


def lgsr_loss_noalloc(ctx: Context, frame: dict, target_depth: torch.Tensor, target_normal: torch.Tensor,
                      loss_out: torch.Tensor, grad_out: dict, weights: LossWeights | None = None):
    """lgsr_loss into caller-provided outputs, with no device allocation by the library (its
    partial sums use a static device array shared by every call on the device)."""
    d = ctx.device
    H, W = frame["depth"].shape
    _dev(frame["depth"], "depth", (H, W), d)
    _dev(frame["normal"], "normal", (H, W, 3), d)
    _dev(target_depth, "target_depth", (H, W), d)
    _dev(target_normal, "target_normal", (H, W, 3), d)
    _dev(loss_out, "loss_out", (5,), d)
    fr = Frame(_ptr(frame["depth"]), _ptr(frame.get("opacity")), _ptr(frame["normal"]), None)
    fg = FrameGrad(_ptr(grad_out["depth"]), _ptr(grad_out["opacity"]), _ptr(grad_out["normal"]))
    w = weights if weights is not None else default_loss_weights()
    ctx._stream()
    ctx._check(lib().lgsr_loss_noalloc(ctx.handle, H * W, ctypes.byref(fr), _ptr(target_depth), _ptr(target_normal),
                                       ctypes.byref(w), _ptr(loss_out), ctypes.byref(fg)))
    return loss_out, grad_out


def lgsr_objective(ctx: Context, frame: dict, row_sincos: torch.Tensor, col_sincos: torch.Tensor,
                   target_depth: torch.Tensor, target_normal: torch.Tensor, weights: ObjectiveWeights | None = None,
                   loss_out: torch.Tensor | None = None, grad_out: dict | None = None, want_grad: bool = True):
    """Frame terms of the full objective (float32[8] on the device: total, depth, opacity,
    G-ICP normal and surface normal terms, |Omega_D|, |Omega_N|, |Omega_S|) and, when
    want_grad, dL/d(depth, opacity, normal) (else None)."""
    d = ctx.device
    H, W = row_sincos.shape[0], col_sincos.shape[0]
    _dev(row_sincos, "row_sincos", (H, 2), d)
    _dev(col_sincos, "col_sincos", (W, 2), d)
    _dev(frame["depth"], "depth", (H, W), d)
    _dev(frame["opacity"], "opacity", (H, W), d)
    _dev(frame["normal"], "normal", (H, W, 3), d)
    _dev(target_depth, "target_depth", (H, W), d)
    _dev(target_normal, "target_normal", (H, W, 3), d)
    if loss_out is None:
        loss_out = torch.empty(8, device=d)
    _dev(loss_out, "loss_out", (8,), d)
    fg = None
    if want_grad:
        if grad_out is None:
            grad_out = dict(depth=torch.empty((H, W), device=d), opacity=torch.empty((H, W), device=d),
                            normal=torch.empty((H, W, 3), device=d))
        _dev(grad_out["depth"], "grad depth", (H, W), d)
        _dev(grad_out["opacity"], "grad opacity", (H, W), d)
        _dev(grad_out["normal"], "grad normal", (H, W, 3), d)
        fg = FrameGrad(_ptr(grad_out["depth"]), _ptr(grad_out["opacity"]), _ptr(grad_out["normal"]))
    else:
        grad_out = None
    bm = Beams(H, W, _ptr(row_sincos), _ptr(col_sincos))
    fr = Frame(_ptr(frame["depth"]), _ptr(frame["opacity"]), _ptr(frame["normal"]), None)
    w = weights if weights is not None else default_objective_weights()
    ctx._stream()
    ctx._check(lib().lgsr_objective(ctx.handle, ctypes.byref(bm), ctypes.byref(fr), _ptr(target_depth),
                                    _ptr(target_normal), ctypes.byref(w), _ptr(loss_out),
                                    ctypes.byref(fg) if fg is not None else None))
    return loss_out, grad_out


def lgsr_scale_reg(ctx: Context, log_scales: torch.Tensor, lambda_s: float = 10.0, s_max: float = 1.0,
                   loss_out: torch.Tensor | None = None, grad_log_scales: torch.Tensor | None = None):
    """Scale regulariser lambda_s sum max(0, max(s) - s_max) (float32[1] on the device); its
    gradient is ADDED into grad_log_scales (n, 2) when given."""
    d = ctx.device
    n = log_scales.shape[0]
    _dev(log_scales, "log_scales", (n, 2), d)
    if loss_out is None:
        loss_out = torch.empty(1, device=d)
    _dev(loss_out, "loss_out", (1,), d)
    if grad_log_scales is not None:
        _dev(grad_log_scales, "grad_log_scales", (n, 2), d)
    ctx._stream()
    ctx._check(lib().lgsr_scale_reg(ctx.handle, n, _ptr(log_scales), float(lambda_s), float(s_max), _ptr(loss_out),
                                    _ptr(grad_log_scales)))
    return loss_out


def lgsr_scan_to_range(ctx: Context, points: torch.Tensor, H: int, W: int, el_min: float, el_max: float,
                       r_min: float = 0.0, r_max: float = float("inf"), normals: torch.Tensor | None = None,
                       out: dict | None = None):
    """Spherical range image of a scan (angles in radians): dict(depth (H,W), normal (H,W,3),
    index (H,W) int32: the winning point or -1)."""
    d = ctx.device
    n = points.shape[0]
    _dev(points, "points", (n, 3), d)
    if normals is not None:
        _dev(normals, "normals", (n, 3), d)
    if out is None:
        out = dict(depth=torch.empty((H, W), device=d), normal=torch.empty((H, W, 3), device=d),
                   index=torch.empty((H, W), device=d, dtype=torch.int32))
    _dev(out["depth"], "depth", (H, W), d)
    _dev(out["normal"], "normal", (H, W, 3), d)
    _dev(out["index"], "index", (H, W), d, torch.int32)
    g = ScanGrid(H, W, el_min, el_max, r_min, r_max)
    ctx._stream()
    ctx._check(lib().lgsr_scan_to_range(ctx.handle, n, _ptr(points), _ptr(normals), ctypes.byref(g),
                                        _ptr(out["depth"]), _ptr(out["normal"]), _ptr(out["index"])))
    return out


def lgsr_target_cov(ctx: Context, quats: torch.Tensor, log_scales: torch.Tensor, eps: float = 0.01,
                    out: torch.Tensor | None = None):
    """Surfel target covariances (n, 6): xx, xy, xz, yy, yz, zz."""
    d = ctx.device
    n = quats.shape[0]
    _dev(quats, "quats", (n, 4), d)
    _dev(log_scales, "log_scales", (n, 2), d)
    if out is None:
        out = torch.empty((n, 6), device=d)
    _dev(out, "cov", (n, 6), d)
    ctx._stream()
    ctx._check(lib().lgsr_target_cov(ctx.handle, n, _ptr(quats), _ptr(log_scales), float(eps), _ptr(out)))
    return out


def lgsr_backward(ctx: Context, state: State, grad: dict, out: dict | None = None,
                  grad_pose: torch.Tensor | None = None):
    """Gradients w.r.t. means (n,3), quats (n,4), log_scales (n,2), opacity_logits (n,) and the
    pose tangent (rho, omega) (6,) of the right perturbation."""
    d = ctx.device
    if state is None or not state.handle:
        raise ValueError("a live State from lgsr_forward is required")
    H, W = grad["depth"].shape
    _dev(grad["depth"], "d_depth", (H, W), d)
    _dev(grad["opacity"], "d_opacity", (H, W), d)
    _dev(grad["normal"], "d_normal", (H, W, 3), d)
    n = state._keep[0][0].shape[0]
    if out is None:
        out = dict(means=torch.empty((n, 3), device=d), quats=torch.empty((n, 4), device=d),
                   log_scales=torch.empty((n, 2), device=d), opacity_logits=torch.empty((n,), device=d))
    if grad_pose is None:
        grad_pose = torch.empty(6, device=d)
    fg = FrameGrad(_ptr(grad["depth"]), _ptr(grad["opacity"]), _ptr(grad["normal"]))
    sg = SurfelGrads(_ptr(out["means"]), _ptr(out["quats"]), _ptr(out["log_scales"]), _ptr(out["opacity_logits"]))
    ctx._stream()
    ctx._check(lib().lgsr_backward(ctx.handle, state.handle, ctypes.byref(fg), ctypes.byref(sg), _ptr(grad_pose)))
    return out, grad_pose


def lgsr_state_free(state: State):
    state.free()


def lgsr_query(ctx: Context, state: State) -> dict:
    o = (ctypes.c_int64 * 8)()
    ctx._stream()
    ctx._check(lib().lgsr_query(ctx.handle, state.handle, o))
    return dict(pairs=o[0], visible=o[1], workspace_bytes=o[2], max_list=o[3], ray_tests=o[4], composites=o[5],
                rays_hit=o[6], ray_tests_needed=o[7])


def lgsr_count_hits(ctx: Context, state: State) -> dict:
    """Hits passing every per-hit test summed over rays, ignoring early termination, and the
    rays with one; waits."""
    o = (ctypes.c_int64 * 2)()
    ctx._stream()
    ctx._check(lib().lgsr_count_hits(ctx.handle, state.handle, o))
    return dict(hits_all=o[0], rays_with_hits=o[1])


def lgsr_tile_list(ctx: Context, state: State, tile_row: int, tile_col: int):
    """The sorted surfel ids (numpy uint32) of one 16 x 16-ray tile's list; waits."""
    import numpy as np
    n = ctypes.c_int64(0)
    ctx._stream()
    ctx._check(lib().lgsr_tile_list(ctx.handle, state.handle, tile_row, tile_col, None, 0, ctypes.byref(n)))
    out = np.zeros(max(1, n.value), np.uint32)
    ctx._check(lib().lgsr_tile_list(ctx.handle, state.handle, tile_row, tile_col,
                                    out.ctypes.data_as(ctypes.c_void_p), n.value, ctypes.byref(n)))
    return out[:n.value]


def lgsr_stream_probe(ctx: Context, kind: str, a: torch.Tensor, b: torch.Tensor, c: torch.Tensor | None = None,
                      plain: bool = False, blocks: int = 0):
    """Streaming probe (not part of the path): kind "copy" a = b, "triad" a = b + 3 c;
    non-temporal 4-vector accesses, or plain one-vector ones; blocks 0 = 4096."""
    for t in (a, b) + ((c,) if c is not None else ()):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device != ctx.device:
            raise ValueError("probe arrays must be contiguous float32 on the context's device")
    ctx._stream()
    k = (0 if kind == "copy" else 1) + (2 if plain else 0)
    ctx._check(lib().lgsr_stream_probe(ctx.handle, k, _ptr(b), _ptr(c), _ptr(a), a.numel(), int(blocks)))


def lgsr_request_bytes(n: int, H: int, W: int, pairs: int, with_grad: bool) -> int:
    """Device bytes a request holds beyond its inputs and outputs (no device needed)."""
    b = ctypes.c_int64(0)
    rc = lib().lgsr_request_bytes(n, H, W, pairs, 1 if with_grad else 0, ctypes.byref(b))
    if rc != LGSR_OK:
        raise ValueError(f"lgsr_request_bytes: {_STATUS.get(rc, rc)}")
    return b.value


def lgsr_batch_poll(ctx: Context, n: int):
    """Per request of the latest batch, whether its kernels have finished (list of bool)."""
    d = (ctypes.c_int32 * max(1, n))()
    ctx._check(lib().lgsr_batch_poll(ctx.handle, n, d))
    return [bool(d[i]) for i in range(n)]


def lgsr_render_batch(ctx: Context, requests, opts: RasterOpts | None = None, weights: LossWeights | None = None):
    """Render a batch of requests in one call (mixed maps, poses and resolutions).

    Each request is a dict with ``surfels`` (dict of device tensors), ``pose`` (3 x 4, host
    array-like), ``row_sincos`` and ``col_sincos`` (device tensors) and optionally
    ``target_depth`` / ``target_normal`` (device tensors: render + gradient) and ``out``
    (preallocated frame dict).  Returns one dict per request: the frame (depth, opacity,
    normal, drop) and, for gradient requests, ``loss`` (5,), ``grads`` (means, quats,
    log_scales, opacity_logits) and ``grad_pose`` (6,).  Asynchronous on torch's current
    stream."""
    d = ctx.device
    arr = (Request * max(1, len(requests)))()
    results, keep = [], []
    for k, q in enumerate(requests):
        rows, cols = q["row_sincos"], q["col_sincos"]
        H, W = rows.shape[0], cols.shape[0]
        _dev(rows, "row_sincos", (H, 2), d)
        _dev(cols, "col_sincos", (W, 2), d)
        s_, tens = _surfels(ctx, q["surfels"])
        out = q.get("out") or dict(depth=torch.empty((H, W), device=d), opacity=torch.empty((H, W), device=d),
                                   normal=torch.empty((H, W, 3), device=d),
                                   drop=torch.empty((H, W), device=d, dtype=torch.uint8))
        _dev(out["depth"], "depth", (H, W), d)
        _dev(out["opacity"], "opacity", (H, W), d)
        _dev(out["normal"], "normal", (H, W, 3), d)
        _dev(out["drop"], "drop", (H, W), d, torch.uint8)
        pose = torch.as_tensor(q["pose"], dtype=torch.float32).reshape(12)
        r = arr[k]
        r.surfels = s_
        for c in range(12):
            r.pose_ws[c] = float(pose[c])
        r.beams = Beams(H, W, _ptr(rows), _ptr(cols))
        r.out = Frame(_ptr(out["depth"]), _ptr(out["opacity"]), _ptr(out["normal"]), _ptr(out["drop"]))
        res = dict(frame=out)
        if q.get("target_depth") is not None:
            td, tn = q["target_depth"], q["target_normal"]
            _dev(td, "target_depth", (H, W), d)
            _dev(tn, "target_normal", (H, W, 3), d)
            n = s_.n
            fg = dict(depth=torch.empty((H, W), device=d), opacity=torch.empty((H, W), device=d),
                      normal=torch.empty((H, W, 3), device=d))
            gr = dict(means=torch.empty((n, 3), device=d), quats=torch.empty((n, 4), device=d),
                      log_scales=torch.empty((n, 2), device=d), opacity_logits=torch.empty((n,), device=d))
            res.update(loss=torch.empty(5, device=d), grads=gr, grad_pose=torch.empty(6, device=d), frame_grad=fg)
            r.target_depth, r.target_normal = _ptr(td), _ptr(tn)
            r.loss_out = _ptr(res["loss"])
            r.frame_grad = FrameGrad(_ptr(fg["depth"]), _ptr(fg["opacity"]), _ptr(fg["normal"]))
            r.grads = SurfelGrads(_ptr(gr["means"]), _ptr(gr["quats"]), _ptr(gr["log_scales"]),
                                  _ptr(gr["opacity_logits"]))
            r.grad_pose = _ptr(res["grad_pose"])
            keep.append((td, tn))
        keep.append((tens, rows, cols))
        results.append(res)
    o = opts if opts is not None else default_opts()
    w = weights if weights is not None else default_loss_weights()
    ctx._stream()
    ctx._check(lib().lgsr_render_batch(ctx.handle, len(requests), arr, ctypes.byref(o), ctypes.byref(w)))
    return results


def lgsr_state_bytes(ctx: Context, state: State | None) -> int:
    """Device bytes held by a state, or by the context itself when state is None (host-side
    bookkeeping, no GPU work)."""
    b = ctypes.c_int64()
    ctx._check(lib().lgsr_state_bytes(ctx.handle, state.handle if state is not None else None, ctypes.byref(b)))
    return int(b.value)


def lgsr_adam_step(ctx: Context, groups, step: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One fused Adam step.  groups: iterable of (param, grad, m, v, lr) with float32
    contiguous tensors of equal shape on the context's device (param, m, v updated in place)."""
    d = ctx.device
    arr = (AdamGroup * 8)()
    k = 0
    for param, grad, m, v, lr in groups:
        if k == 8:
            raise ValueError("at most 8 groups per step")
        for name, t in (("param", param), ("grad", grad), ("m", m), ("v", v)):
            _dev(t, name, tuple(param.shape), d)
        arr[k] = AdamGroup(param.numel(), _ptr(param), _ptr(grad), _ptr(m), _ptr(v), float(lr))
        k += 1
    ctx._stream()
    ctx._check(lib().lgsr_adam_step(ctx.handle, k, arr, beta1, beta2, eps, int(step)))


def lgsr_profile(ctx: Context, stages=True):
    """Enable stage timers: True = all stages, False = off, or an iterable of stage names."""
    if stages is True:
        mask = -1
    elif not stages:
        mask = 0
    else:
        mask = 0
        for name in stages:
            mask |= 1 << STAGES.index(name)
    ctx._check(lib().lgsr_profile(ctx.handle, mask))


def lgsr_profile_read(ctx: Context) -> dict:
    """{stage: (milliseconds, calls)} accumulated since the last read (waits for the stream)."""
    ms = (ctypes.c_double * len(STAGES))()
    calls = (ctypes.c_int64 * len(STAGES))()
    ctx._stream()
    ctx._check(lib().lgsr_profile_read(ctx.handle, ms, calls))
    return {name: (ms[i], calls[i]) for i, name in enumerate(STAGES)}


def lgsr_sync(ctx: Context):
    ctx._check(lib().lgsr_sync(ctx.handle))
