"""GPU parity of the full mapping objective (lgsr_objective: Eq. 10-11 weighted as in Eq. 13,
with the rendered-surface normal term) and of the scale regulariser (lgsr_scale_reg, Eq. 12)
against the FP64 oracle, on seeded renderer-shaped frames (exact raycasts of the street-block
scene with range noise, holes and opacity-scaled noisy normals) and edge shapes.

Tolerances: counts exact; the loss terms 1e-5 relative (1e-4 for the two normal terms);
gradients 1e-3 relative per element plus 1e-5 of the largest magnitude of that output
(float32 stencil differences of nearly equal points lose a few digits).  Pixels whose
N_surf orientation is a near tie (|v.d| / |v| < 1e-3) are left out with everything their
stencil reaches."""
import numpy as np
import pytest

import scenegen
from oracle import ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_04127_amd import lgsr
    c = lgsr.Context(0)
    yield c
    c.close()


def _case(H, W, seed, el=(-22.5, 22.5)):
    sc = scenegen.make_scene("block", 2, 400)
    rows, cols = scenegen.beam_tables(H, W, *el)
    rng = np.random.default_rng(seed)
    pose = scenegen.make_pose(rng.uniform(0, 6.28), *rng.uniform(-5, 5, 2))
    depth, op, nrm = scenegen.synthetic_frame(sc, pose, rows, cols, seed)
    pose2 = pose.copy()
    pose2[:, 3] += rng.normal(0, 0.05, 3).astype(np.float32)
    td, tn = scenegen.targets_for_pose(sc, pose2, rows, cols, 0.1, seed + 1)
    return rows, cols, dict(depth=depth, opacity=op, normal=nrm), td, tn


def _tie_mask(rows, cols, depth):
    """Pixels within reach (radius 2) of an N_surf orientation near-tie."""
    H, W = rows.shape[0], cols.shape[0]
    _, ok, fm = ref.surf_normal(rows, cols, depth)
    tie = (fm.reshape(H, W) < 1e-3) & ok.reshape(H, W).astype(bool)
    pad = np.zeros((H + 4, W), bool)
    pad[2:H + 2] = tie
    out = np.zeros((H, W), bool)
    for dk, dj in [(a, b) for a in range(-2, 3) for b in range(-2, 3) if abs(a) + abs(b) <= 2]:
        out |= np.roll(pad, dj, axis=1)[2 + dk:H + 2 + dk]
    return out.reshape(-1), int(tie.sum())


def _run(ctx, rows, cols, pred, td, tn, w):
    from paper_2607_04127_amd import lgsr
    d = torch.device("cuda", 0)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(d)  # noqa: E731
    L, g = lgsr.lgsr_objective(ctx, {k: dv(v) for k, v in pred.items()}, dv(rows), dv(cols), dv(td), dv(tn),
                               lgsr.default_objective_weights(**w))
    torch.cuda.synchronize()
    return L.cpu().numpy(), {k: v.cpu().numpy() for k, v in g.items()}


def _compare(tag, L, g, Lr, gd, go, gn, skip):
    assert tuple(L[5:8]) == tuple(Lr[5:8]), (tag, L[5:8], Lr[5:8])
    for i, rel in ((0, 1e-5), (1, 1e-5), (2, 1e-5), (3, 1e-4), (4, 1e-4)):
        assert abs(L[i] - Lr[i]) <= rel * abs(Lr[i]) + 1e-7, (tag, i, L[i], Lr[i])
    keep = ~skip
    stats = {}
    for name, a, b in (("depth", g["depth"].reshape(-1), gd), ("opacity", g["opacity"].reshape(-1), go),
                       ("normal", g["normal"].reshape(-1, 3), gn)):
        a, b = a[keep].astype(np.float64), b[keep]
        scale = np.abs(b).max() if b.size else 0.0
        err = np.abs(a - b)
        bad = err > 1e-3 * np.abs(b) + 1e-5 * scale + 1e-30
        stats[name] = (int(bad.sum()), float((err / (np.abs(b) + 1e-5 * scale + 1e-30)).max(initial=0.0)))
        assert not bad.any(), (tag, name, stats[name])
    return stats


@pytest.mark.parametrize("H,W,lam_ns", [(64, 1024, 0.01), (64, 1024, 0.5), (32, 256, 0.3), (17, 33, 0.3),
                                        (3, 5, 1.0), (2, 9, 1.0), (1, 7, 1.0), (9, 1, 1.0)])
def test_objective_matches_oracle(ctx, H, W, lam_ns):
    rows, cols, pred, td, tn = _case(H, W, seed=H * 1000 + W)
    w = dict(lambda_ns=lam_ns)
    Lr, gd, go, gn = ref.objective(rows, cols, pred, td, tn, w)
    skip, ties = _tie_mask(rows, cols, pred["depth"])
    L, g = _run(ctx, rows, cols, pred, td, tn, w)
    stats = _compare((H, W), L, g, Lr, gd, go, gn, skip)
    print(f"\n[objective {H}x{W} lambda_ns={lam_ns}] loss={L[0]:.6g} ref={Lr[0]:.6g} |Omega_S|={int(Lr[7])} "
          f"ties={ties} " + " ".join(f"{k}: bad={v[0]} worst={v[1]:.2e}" for k, v in stats.items()), flush=True)
    if H * W >= 1024:
        assert Lr[7] > 0.2 * Lr[5]


def test_objective_empty_and_zero_weights(ctx):
    """No valid target: every term and gradient zero; lambda_ns = 0 skips the stencil."""
    rows, cols, pred, td, tn = _case(16, 64, seed=9)
    L, g = _run(ctx, rows, cols, pred, np.zeros_like(td), np.zeros_like(tn), {})
    assert not L[:7].any() and all(not v.any() for v in g.values())
    Lr, gd, go, gn = ref.objective(rows, cols, pred, td, tn, dict(lambda_ns=0.0, lambda_alpha=0.0))
    L, g = _run(ctx, rows, cols, pred, td, tn, dict(lambda_ns=0.0, lambda_alpha=0.0))
    _compare("zero weights", L, g, Lr, gd, go, gn, np.zeros(16 * 64, bool))
    assert L[2] == 0.0 and L[4] == 0.0 and not g["opacity"].any()


@pytest.mark.parametrize("n,s_max", [(300_000, 1.0), (300_000, 0.3), (1, 0.5), (0, 1.0), (1000, 1e6)])
def test_scale_regulariser_matches_oracle(ctx, n, s_max):
    from paper_2607_04127_amd import lgsr
    rng = np.random.default_rng(n + 7)
    ls = np.log(rng.uniform(0.05, 2.0, size=(n, 2))).astype(np.float32)
    if n >= 10:
        ls[: n // 10, 1] = ls[: n // 10, 0]  # exact ties: the first scale takes the gradient
    base = rng.normal(size=(n, 2)).astype(np.float32)
    Lr, gr, m = ref.scale_reg(ls, 10.0, s_max)
    d = torch.device("cuda", 0)
    g = torch.from_numpy(base).to(d)
    L = lgsr.lgsr_scale_reg(ctx, torch.from_numpy(ls).to(d), 10.0, s_max, grad_log_scales=g)
    torch.cuda.synchronize()
    L, g = float(L.cpu()[0]), g.cpu().numpy().astype(np.float64)
    keep = m >= 1e-5
    assert abs(L - Lr) <= 1e-5 * abs(Lr) + 1e-5 * (~keep).sum() * 10.0 * s_max + 1e-7, (L, Lr)
    want = base.astype(np.float64) + gr
    err = np.abs(g - want)[keep]
    assert (err <= 1e-6 * np.abs(want[keep]) + 1e-6).all(), err.max(initial=0.0)
    print(f"\n[scale reg n={n} s_max={s_max}] loss={L:.6g} ref={Lr:.6g} active={(gr != 0).any(1).sum()}", flush=True)


def test_autograd_full_objective_equals_direct_calls(ctx):
    """Eq. 13 through torch.autograd (render -> objective + scale regulariser) gives the
    gradients of the direct C-ABI sequence lgsr_forward -> lgsr_objective -> lgsr_backward ->
    lgsr_scale_reg (up to float32 summation order of the backward's atomics)."""
    from paper_2607_04127_amd import autograd as AG
    from paper_2607_04127_amd import lgsr
    from tests import _gpu as G
    w = scenegen.make_workload("room32x256_1k")
    w = dict(w, log_scales=(w["log_scales"] + np.float32(1.2)).astype(np.float32))  # some surfels above s_max
    dw = G.to_dev(w)
    weights = lgsr.default_objective_weights(lambda_ns=0.2)
    fr, st = G.gpu_forward(ctx, dw)
    L, g = lgsr.lgsr_objective(ctx, fr, dw["row_sincos"], dw["col_sincos"], dw["target_depth"], dw["target_normal"],
                               weights)
    out, gp = lgsr.lgsr_backward(ctx, st, g)
    Ls = lgsr.lgsr_scale_reg(ctx, dw["log_scales"], 10.0, 0.3, grad_log_scales=out["log_scales"])
    torch.cuda.synchronize()
    st.free()
    direct = {k: v.cpu().numpy() for k, v in out.items()}
    r = AG.Renderer(ctx, dw["row_sincos"], dw["col_sincos"])
    P = {k: dw[k].clone().requires_grad_(True) for k in G.SURF_KEYS}
    xi = torch.zeros(6, dtype=torch.float64, requires_grad=True)
    fr2 = AG.render(r, P, w["pose"], xi)
    La, terms = AG.objective(r, fr2, dw["target_depth"], dw["target_normal"], weights)
    total = La + AG.scale_reg(ctx, P["log_scales"], 10.0, 0.3)
    total.backward()
    torch.cuda.synchronize()
    assert float(La) == float(L[0]) and float(Ls[0]) > 0
    assert float(total) == pytest.approx(float(L[0]) + float(Ls[0]), rel=1e-6)
    for k in G.SURF_KEYS:
        a, b = P[k].grad.cpu().numpy().astype(np.float64), direct[k].astype(np.float64)
        assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max() + 1e-30, k
    assert (direct["log_scales"] != 0).any() and terms[3].item() > 0
