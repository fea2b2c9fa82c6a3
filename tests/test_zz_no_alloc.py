"""The allocation-free loss entry point (lgsr_loss_noalloc), called through the C ABI,
against lgsr_loss on the same inputs: two calls in a row, the second with a smaller frame,
so that the second call reads partial sums the first left in the shared static scratch
only where it wrote them itself.  Both evaluate the same kernels with the same launch
shape, so the results agree bit for bit."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _frame(H, W, seed, dev):
    rng = np.random.default_rng(seed)
    depth = rng.uniform(2, 40, (H, W)) * (rng.random((H, W)) > 0.2)
    nrm = rng.normal(size=(H, W, 3))
    nrm[rng.random((H, W)) < 0.05] = 0.0
    td = np.where(rng.random((H, W)) > 0.1, depth + rng.normal(scale=0.3, size=(H, W)), 0.0)
    tn = rng.normal(size=(H, W, 3))
    tn /= np.linalg.norm(tn, axis=2, keepdims=True)
    tn[td <= 0] = 0.0
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)  # noqa: E731
    return dict(depth=f(depth), opacity=f(np.ones((H, W))), normal=f(nrm)), f(td), f(tn)


def _outs(H, W, dev):
    return torch.full((5,), float("nan"), device=dev), dict(
        depth=torch.full((H, W), float("nan"), device=dev), opacity=torch.full((H, W), float("nan"), device=dev),
        normal=torch.full((H, W, 3), float("nan"), device=dev))


def test_loss_noalloc_matches_loss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_04127_amd import lgsr
    dev = torch.device("cuda:0")
    ctx = lgsr.Context(0)
    L = lgsr.lib()
    try:
        # the largest frame first: 128 x 2048 rays use the most workgroups (the scratch's
        # limit), then 32 x 1024 and a ragged 7 x 33
        for k, (H, W) in enumerate([(128, 2048), (32, 1024), (7, 33)]):
            frame, td, tn = _frame(H, W, 100 + k, dev)
            lo_ref, g_ref = _outs(H, W, dev)
            lgsr.lgsr_loss(ctx, frame, td, tn, loss_out=lo_ref, grad_out=g_ref)
            lo, g = _outs(H, W, dev)
            # straight through the C ABI
            fr = lgsr.Frame(lgsr._ptr(frame["depth"]), lgsr._ptr(frame["opacity"]), lgsr._ptr(frame["normal"]), None)
            fg = lgsr.FrameGrad(lgsr._ptr(g["depth"]), lgsr._ptr(g["opacity"]), lgsr._ptr(g["normal"]))
            w = lgsr.default_loss_weights()
            ctx._stream()
            rc = L.lgsr_loss_noalloc(ctx.handle, H * W, ctypes.byref(fr), lgsr._ptr(td), lgsr._ptr(tn),
                                     ctypes.byref(w), lgsr._ptr(lo), ctypes.byref(fg))
            assert rc == lgsr.LGSR_OK, L.lgsr_last_error(ctx.handle)
            torch.cuda.synchronize()
            print(f"\n[loss noalloc {H}x{W}] loss={lo.cpu().numpy()} ref={lo_ref.cpu().numpy()}", flush=True)
            assert torch.equal(lo, lo_ref)
            for key in ("depth", "opacity", "normal"):
                assert torch.equal(g[key], g_ref[key]), key
            # the binding's wrapper gives the same
            lo2, g2 = _outs(H, W, dev)
            lgsr.lgsr_loss_noalloc(ctx, frame, td, tn, lo2, g2)
            torch.cuda.synchronize()
            assert torch.equal(lo2, lo_ref) and torch.equal(g2["normal"], g_ref["normal"])
        # arguments are checked before anything is launched
        assert L.lgsr_loss_noalloc(ctx.handle, -1, None, None, None, None, None, None) == lgsr.LGSR_EINVAL
        assert L.lgsr_loss_noalloc(None, 0, None, None, None, None, None, None) == lgsr.LGSR_EINVAL
    finally:
        ctx.close()
