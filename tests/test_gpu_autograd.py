"""GPU tests of the differentiable-rendering layer (torch.autograd over the C ABI): the
autograd path equals the direct calls, keeping and recomputing the forward's lists give
identical gradients, the pose-tangent gradient at a nonzero xi matches the oracle (analytic
and finite differences), the fused Adam kernel matches a float64 Adam, and a window of
keyframes (1M surfels, 8 poses) matches the oracle at iteration 0 and, refined with both
optimisers, reduces its loss."""
import numpy as np
import pytest

import scenegen
from oracle import ref
from tests import _gpu as G

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


@pytest.fixture(scope="module")
def room_off():
    """The room with targets moved 5-30 cm off the rendered surfaces (smooth L1)."""
    w = scenegen.make_workload("room32x256_1k")
    rng = np.random.default_rng(12)
    td = w["target_depth"]
    td = np.where(td > 0, td + rng.choice([-1, 1], td.shape) * rng.uniform(0.05, 0.3, td.shape), 0)
    return dict(w, target_depth=td.astype(np.float32))


def _renderer(ctx, w, **kw):
    from paper_2607_04127_amd import autograd as AG
    rows = torch.from_numpy(w["row_sincos"]).cuda()
    cols = torch.from_numpy(w["col_sincos"]).cuda()
    return AG.Renderer(ctx, rows, cols, **kw)


def _leaf(w):
    return {k: torch.from_numpy(np.ascontiguousarray(w[k])).cuda().requires_grad_(True) for k in G.SURF_KEYS}


def _autograd_grads(ctx, w, keep, xi=None):
    from paper_2607_04127_amd import autograd as AG
    r = _renderer(ctx, w, keep_lists=keep)
    P = _leaf(w)
    xi_t = torch.zeros(6, dtype=torch.float64, requires_grad=True) if xi is None else \
        torch.tensor(xi, dtype=torch.float64, requires_grad=True)
    fr = AG.render(r, P, w["pose"], xi_t)
    L, _ = AG.loss(r, fr, torch.from_numpy(w["target_depth"]).cuda(), torch.from_numpy(w["target_normal"]).cuda())
    L.backward()
    torch.cuda.synchronize()
    return float(L), {k: P[k].grad.cpu().numpy() for k in G.SURF_KEYS}, xi_t.grad.numpy(), r


def _close(a, b, what):
    """Equal up to float32 summation order: the backward adds record gradients with atomics,
    so two runs may round differently (the forward itself is bitwise reproducible)."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    scale = np.abs(b).max() if b.size else 0.0
    assert np.abs(a - b).max(initial=0.0) <= 1e-5 * scale + 1e-30, what


def test_autograd_equals_direct_calls_and_keep_modes(ctx, room_off):
    from paper_2607_04127_amd import lgsr
    w = room_off
    dw = G.to_dev(w)
    fr, st = G.gpu_forward(ctx, dw)
    L, g = lgsr.lgsr_loss(ctx, fr, dw["target_depth"], dw["target_normal"])
    out, gp = lgsr.lgsr_backward(ctx, st, g)
    torch.cuda.synchronize()
    st.free()
    direct = {k: v.cpu().numpy() for k, v in out.items()}
    for keep in ("store", "recompute"):
        La, ga, gxi, r = _autograd_grads(ctx, w, keep)
        assert La == float(L[0])
        for k in G.SURF_KEYS:
            _close(ga[k], direct[k], (keep, k))
        _close(gxi, gp.cpu().numpy(), (keep, "pose"))
        assert r.recomputed == (1 if keep == "recompute" else 0) and r.held == 0
    # a budget too small for one state recomputes
    _, gb, _, r = _autograd_grads(ctx, w, "auto")
    assert r.recomputed == 0
    from paper_2607_04127_amd import autograd as AG
    r2 = _renderer(ctx, w, keep_lists="auto", hbm_budget=1)
    P = _leaf(w)
    fr = AG.render(r2, P, w["pose"])
    AG.loss(r2, fr, torch.from_numpy(w["target_depth"]).cuda(), torch.from_numpy(w["target_normal"]).cuda())[0].backward()
    assert r2.recomputed == 1
    _close(P["means"].grad.cpu().numpy(), direct["means"], "auto, recomputed")


def test_kept_states_return_their_budget(ctx, room_off):
    """A render that no backward can follow keeps no state, and a kept state whose graph is
    dropped without a backward gives its bytes back to the renderer's budget."""
    import gc

    from paper_2607_04127_amd import autograd as AG
    w = room_off
    r = _renderer(ctx, w, keep_lists="store")
    P = _leaf(w)
    with torch.no_grad():
        AG.render(r, P, w["pose"])
    assert r.held == 0
    frozen = {k: v.detach() for k, v in P.items()}
    AG.render(r, frozen, w["pose"])  # no input asks for a gradient
    assert r.held == 0
    fr = AG.render(r, P, w["pose"])
    assert r.held > 0
    del fr
    gc.collect()
    assert r.held == 0
    fr = AG.render(r, P, w["pose"])
    AG.loss(r, fr, torch.from_numpy(w["target_depth"]).cuda(), torch.from_numpy(w["target_normal"]).cuda())[0].backward()
    assert r.held == 0 and r.recomputed == 0


def test_pose_tangent_gradient_at_nonzero_xi(ctx, room_off):
    """d loss / d xi at T0 Exp(xi), xi != 0: against J_r(xi)^T applied to the oracle's
    right-perturbation gradient at T (tolerance of the gradient parity), and against central
    differences of the oracle's loss in xi.  For the differences the loss keeps only rays
    whose threshold decisions and compositing order are at least 1e-3 (relative) from
    flipping (the others get target depth 0, which drops them from both losses), so the
    loss is smooth over the step."""
    from paper_2607_04127_amd import autograd as AG
    w = room_off
    xi = np.array([0.05, -0.03, 0.02, 0.01, -0.02, 0.015])
    T = AG.compose(w["pose"], xi)
    Tf = T.astype(np.float32).astype(np.float64)  # the pose the renderer receives
    of = ref.forward(w, Tf, w["row_sincos"], w["col_sincos"], extra=True)
    smooth = (of["margin"] > 1e-3) & (of["order_gap"] > 1e-3)
    td = np.where(smooth.reshape(w["target_depth"].shape), w["target_depth"], 0).astype(np.float32)
    ws = dict(w, target_depth=td)
    assert (td > 0).sum() > 1000
    _, _, gxi, _ = _autograd_grads(ctx, ws, "store", xi=xi)
    _, _, g = ref.loss_and_grad(ws, Tf, w["row_sincos"], w["col_sincos"], td, w["target_normal"])
    expect = AG.se3_right_jacobian(xi).T @ g["pose"]
    assert np.abs(gxi - expect).max() <= 1e-3 * np.linalg.norm(expect), (gxi, expect)

    def L_of(x):
        Lx, _, _ = ref.loss_and_grad(ws, AG.compose(w["pose"], x), w["row_sincos"], w["col_sincos"], td,
                                     w["target_normal"])
        return Lx[0]

    h = 1e-6
    fd = np.array([(L_of(xi + h * e) - L_of(xi - h * e)) / (2 * h) for e in np.eye(6)])
    assert np.abs(gxi - fd).max() <= 2e-3 * np.linalg.norm(fd), (gxi, fd)


def test_loss_function_backward(ctx, room_off):
    from paper_2607_04127_amd import autograd as AG, lgsr
    w = room_off
    dw = G.to_dev(w)
    fr, _ = G.gpu_forward(ctx, dw, want_state=False)
    frame = {k: fr[k].clone().requires_grad_(True) for k in ("depth", "opacity", "normal")}
    r = _renderer(ctx, w)
    L, terms = AG.loss(r, frame, dw["target_depth"], dw["target_normal"])
    (2.0 * L).backward()
    L2, g = lgsr.lgsr_loss(ctx, {k: fr[k] for k in ("depth", "opacity", "normal")}, dw["target_depth"],
                           dw["target_normal"])
    torch.cuda.synchronize()
    assert float(L) == float(L2[0]) and torch.equal(terms, L2[1:])
    for k in ("depth", "opacity", "normal"):
        assert torch.equal(frame[k].grad, 2.0 * g[k]), k


def _adam64(p, g, m, v, lr, b1, b2, eps, t):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    return p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps), m, v


def test_adam_kernel_matches_float64_adam(ctx):
    from paper_2607_04127_amd import lgsr
    rng = np.random.default_rng(9)
    sizes = [1, 3, 4096, 16387, 70001]
    lrs = [1e-2, 3e-3, 1e-3, 5e-4, 2e-2]
    base = [torch.from_numpy(rng.normal(size=n + 1).astype(np.float32)).cuda() for n in sizes]
    # group 3 works on a slice at an odd offset (the kernel's scalar path)
    P = [b[:-1] if k != 3 else b[1:] for k, b in enumerate(base)]
    outside = [float(b[-1]) if k != 3 else float(b[0]) for k, b in enumerate(base)]
    M = [torch.zeros_like(p) for p in P]
    V = [torch.zeros_like(p) for p in P]
    ref_state = [(p.cpu().numpy().astype(np.float64), np.zeros(p.numel()), np.zeros(p.numel())) for p in P]
    for t in range(1, 4):
        Gs = [torch.from_numpy(rng.normal(size=p.numel()).astype(np.float32)).cuda() for p in P]
        lgsr.lgsr_adam_step(ctx, [(P[k], Gs[k], M[k], V[k], lrs[k]) for k in range(len(P))], t, 0.9, 0.999, 1e-8)
        ref_state = [_adam64(ps, Gs[k].cpu().numpy().astype(np.float64), ms, vs, lrs[k], 0.9, 0.999, 1e-8, t)
                     for k, (ps, ms, vs) in enumerate(ref_state)]
    torch.cuda.synchronize()
    for k, p in enumerate(P):
        np.testing.assert_allclose(p.cpu().numpy(), ref_state[k][0], rtol=2e-6, atol=2e-6 * lrs[k])
    # the element just outside each group's slice is untouched
    assert [float(b[-1]) if k != 3 else float(b[0]) for k, b in enumerate(base)] == outside


@pytest.fixture(scope="module")
def window_1m(ctx):
    """The sliding window at its stated size: 64 x 2048 beams (-24.9 to +2 degrees), 1,000,000
    surfels, 8 keyframe poses 1.5 m apart with yaw noise, pose estimates and centres
    perturbed, lists recomputed in the backward."""
    from paper_2607_04127_amd import window as WN
    w = scenegen.make_workload("window64x2048_1m")
    poses, means = WN.perturb(w)
    return dict(w=w, poses=poses, means=means,
                win=WN.Window(ctx, w, poses, means=means, keep_lists="recompute"))


@pytest.mark.parametrize("k", range(8))
def test_window_1m_iteration0_parity(window_1m, k):
    """Iteration 0, keyframe k, on 4,096 seeded rays of the 131,072: the frame through the
    autograd path against the oracle's forward on those rays (tie rays aside, bars widened
    with 1 / den_min at grazing incidence), and the gradient of the keyframe's loss on those
    rays (upstream from the oracle's loss, tie rays zeroed) against the oracle's backward,
    for every surfel parameter and the keyframe's pose tangent.  The oracle takes the map
    as the window holds it on the device."""
    from paper_2607_04127_amd import autograd as AG
    w, win = window_1m["w"], window_1m["win"]
    H, W = w["H"], w["W"]
    assert win.iter == 0 and not win.pose_opt.xi.detach().numpy().any()
    ids = np.sort(np.random.default_rng(500 + k).choice(H * W, size=4096, replace=False))
    Pk = np.asarray(win.pose_opt.T0[k], np.float32).astype(np.float64)  # the pose the renderer receives
    wp = dict(w, pose=Pk, **{key: win.params[key].detach().cpu().numpy() for key in G.SURF_KEYS})
    of = G.oracle_forward(wp, ray_ids=ids)
    for key in G.SURF_KEYS:
        win.params[key].grad = None
    win.pose_opt.xi.grad = None
    fr = AG.render(win.renderer, win.params, win.pose_opt.T0[k], win.pose_opt.xi[k])
    st = G.compare_forward(fr, of, ray_ids=ids, conditioned=True)
    mask = (~G.tie_mask(of)).astype(np.float64)
    td, tn = w["targets"][k]
    _, gd, _, gn = ref.loss(of, np.asarray(td).reshape(-1)[ids], np.asarray(tn).reshape(-1, 3)[ids])
    gd, gn = (gd * mask).astype(np.float32), (gn * mask[:, None]).astype(np.float32)
    up_d = np.zeros(H * W, np.float32)
    up_n = np.zeros((H * W, 3), np.float32)
    up_d[ids], up_n[ids] = gd, gn
    lin = (fr["depth"] * torch.from_numpy(up_d.reshape(H, W)).cuda()).sum() + \
          (fr["normal"] * torch.from_numpy(up_n.reshape(H, W, 3)).cuda()).sum()
    lin.backward()
    torch.cuda.synchronize()
    g_ref = ref.backward(wp, Pk, w["row_sincos"], w["col_sincos"], gd, np.zeros_like(gd), gn, ray_ids=ids,
                         with_mass=True)
    worst = {}
    for j, key in enumerate(G.SURF_KEYS):
        r = G.grad_report(win.params[key].grad.cpu().numpy(), g_ref[key], mass=g_ref["mass"][:, j])
        worst[key] = round(r["worst"], 3)
        if r["bad"] or r["cos"] <= 0.99999:
            raise AssertionError(f"{key}: {r}; rays of the worst surfel: "
                                 f"{_rays_of(wp, ids, of, r['worst_row']['row'])}")
    gxi = win.pose_opt.xi.grad[k].numpy()
    nbad, cos, wp_ = G.grad_check(gxi, g_ref["pose"], mass=g_ref["pose_mass"], per_row=False)
    assert nbad == 0 and cos > 0.99999, ("pose", nbad, cos, wp_)
    assert not np.delete(win.pose_opt.xi.grad.numpy(), k, axis=0).any(), "other keyframes got a gradient"
    print(f"\n[window 1M keyframe {k}] {st}; worst gradient / bound {worst}, pose {wp_:.3f}", flush=True)


def _rays_of(wp, ids, of, sid):
    """Diagnostics: the sampled rays that composite surfel sid, with their tie figures."""
    lists = ref.contributors(wp, wp["pose"], wp["row_sincos"], wp["col_sincos"], ray_ids=ids, cap=4096)
    out = []
    for i, row in enumerate(lists):
        if sid in row:
            out.append(dict(ray=int(ids[i]), pos=int(np.flatnonzero(row == sid)[0]), K=len(row),
                            margin=float(of["margin"][i]), order_gap=float(of["order_gap"][i]),
                            den_min=float(of["den_min"][i])))
    return out


def test_window_1m_descent(window_1m):
    """Ten iterations of map + pose refinement on the full window (recompute mode): the
    summed loss decreases."""
    win = window_1m["win"]
    for key in G.SURF_KEYS:
        win.params[key].grad = None
    win.pose_opt.xi.grad = None
    curve = [win.step() for _ in range(10)]
    print(f"\n[window 1M x 8] loss {curve[0]:.5f} -> {curve[-1]:.5f}", flush=True)
    assert curve[-1] < 0.9 * curve[0], curve
