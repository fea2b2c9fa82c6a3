"""GPU parity: the gfx950 renderer, called through its C ABI, against the FP64 oracle on the
same seeded inputs (tolerances and the tie-ray rule in tests/_gpu.py)."""
import math

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
def room():
    return scenegen.make_workload("room32x256_1k")


@pytest.fixture(scope="module")
def block():
    return scenegen.make_workload("block64x1024_300k")


def _print(name, stats):
    print(f"\n[{name}] " + " ".join(f"{k}={v}" for k, v in stats.items()), flush=True)


def _loss_upstream(w, of, ray_ids=None, mask=None):
    """Oracle loss gradients of the oracle frame, float32-rounded, zero on masked-out rays."""
    td = np.asarray(w["target_depth"]).reshape(-1)
    tn = np.asarray(w["target_normal"]).reshape(-1, 3)
    if ray_ids is not None:
        td, tn = td[ray_ids], tn[ray_ids]
    _, gd, go, gn = ref.loss(of, td, tn)
    if mask is not None:
        gd, go, gn = gd * mask, go * mask, gn * mask[:, None]
    return gd.astype(np.float32), go.astype(np.float32), gn.astype(np.float32)


def _gpu_backward(ctx, dw, state, H, W, gd, go, gn, ray_ids=None):
    from paper_2607_04127_amd import lgsr
    full = np.zeros(H * W, np.float32), np.zeros(H * W, np.float32), np.zeros((H * W, 3), np.float32)
    if ray_ids is None:
        full = (gd, go, gn)
    else:
        full[0][ray_ids], full[1][ray_ids], full[2][ray_ids] = gd, go, gn
    grad = dict(depth=torch.from_numpy(full[0].reshape(H, W)).cuda(),
                opacity=torch.from_numpy(full[1].reshape(H, W)).cuda(),
                normal=torch.from_numpy(full[2].reshape(H, W, 3)).cuda())
    out, gp = lgsr.lgsr_backward(ctx, state, grad)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, gp.cpu().numpy()


def _check_grads(name, g_gpu, gp_gpu, g_ref):
    """Per parameter kind: (failures, cosine, worst error / bound); the diagnostics line
    gives, per kind, the rows that pass only through the mass floor and the elements that
    miss the plain element-wise rule (all of them / those in rows passing without the floor)."""
    report, diag = {}, {}
    for k, key in enumerate(G.SURF_KEYS):
        r = G.grad_report(g_gpu[key], g_ref[key], mass=g_ref["mass"][:, k])
        report[key] = (r["bad"], round(r["cos"], 9), round(r["worst"], 3))
        diag[key] = f"floor_only={r['floor_only']}/{r['rows']} elem={r['elem_bad']}/{r['elems']} " \
                    f"elem_nonfloor={r['elem_bad_nonfloor']}"
    r = G.grad_report(gp_gpu, g_ref["pose"], mass=g_ref["pose_mass"], per_row=False)
    report["pose"] = (r["bad"], round(r["cos"], 9), round(r["worst"], 3))
    diag["pose"] = f"floor_only={r['floor_only']}/6 elem={r['elem_bad']}/6"
    _print(name, report)
    _print(name + " diagnostics", diag)
    for key, (nbad, cos, _) in report.items():
        assert nbad == 0, (key, report[key])
        assert cos > 0.99999, (key, report[key])


# ------------------------------------------------------------------------------------------
# 32 x 256 beams, 1,000 surfels (full image)
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("chunk", [0, 16, 4096])
def test_forward_room(ctx, room, chunk):
    """Full image; chunk 16 splits every tile list into many parallel chunks (merge and
    fix-up paths), 4096 keeps each list in one chunk."""
    dw = G.to_dev(room)
    fr, st = G.gpu_forward(ctx, dw, chunk=chunk)
    torch.cuda.synchronize()
    of = G.oracle_forward(room)
    stats = G.compare_forward(fr, of)
    from paper_2607_04127_amd import lgsr
    q = lgsr.lgsr_query(ctx, st)
    stats.update(pairs=q["pairs"], visible=q["visible"], max_list=q["max_list"])
    _print(f"forward room32x256_1k chunk={chunk}", stats)
    assert stats["tie"] < 0.01 * stats["rays"]
    st.free()


def test_forward_is_deterministic(ctx, room):
    dw = G.to_dev(room)
    a, _ = G.gpu_forward(ctx, dw, want_state=False)
    a = {k: v.clone() for k, v in a.items()}
    b, _ = G.gpu_forward(ctx, dw, want_state=False)
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_loss_kernel(ctx, room):
    """The loss kernel on the renderer's own frame against the oracle loss of that frame."""
    from paper_2607_04127_amd import lgsr
    dw = G.to_dev(room)
    fr, _ = G.gpu_forward(ctx, dw, want_state=False)
    L, g = lgsr.lgsr_loss(ctx, fr, dw["target_depth"], dw["target_normal"])
    torch.cuda.synchronize()
    pred = {k: fr[k].cpu().numpy().astype(np.float64).reshape(-1, *(fr[k].shape[2:])) for k in ("depth", "opacity",
                                                                                                "normal")}
    L_ref, gd, go, gn = ref.loss(pred, room["target_depth"], room["target_normal"])
    L = L.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(L[:3], L_ref[:3], rtol=1e-5)
    assert tuple(L[3:]) == tuple(L_ref[3:])
    np.testing.assert_allclose(g["depth"].cpu().numpy().reshape(-1), gd, rtol=1e-6, atol=0)
    assert np.all(g["opacity"].cpu().numpy() == 0)
    np.testing.assert_allclose(g["normal"].cpu().numpy().reshape(-1, 3), gn, rtol=1e-4, atol=1e-9)


@pytest.mark.parametrize("chunk", [0, 16, 4096])
def test_backward_room(ctx, room, chunk):
    H, W = room["H"], room["W"]
    dw = G.to_dev(room)
    _, st = G.gpu_forward(ctx, dw, chunk=chunk)
    of = G.oracle_forward(room)
    mask = (~G.tie_mask(of)).astype(np.float64)
    gd, go, gn = _loss_upstream(room, of, mask=mask)
    # an opacity upstream as well, so the g_A path (used by the opacity BCE) is covered
    rng = np.random.default_rng(4)
    go = (rng.normal(size=go.shape) * 1e-4 * mask).astype(np.float32)
    g_gpu, gp = _gpu_backward(ctx, dw, st, H, W, gd, go, gn)
    g_ref = ref.backward(room, room["pose"], room["row_sincos"], room["col_sincos"], gd, go, gn, with_mass=True)
    _check_grads(f"backward room32x256_1k chunk={chunk}", g_gpu, gp, g_ref)
    st.free()


def _moved(w0, rotvec, tv):
    """The workload's surfels and pose moved by one rigid transform (M, tv): the image, and
    so the sensor-frame targets, stay the same in exact arithmetic."""
    from scipy.spatial.transform import Rotation
    from tests import _util as U
    M = Rotation.from_rotvec(rotvec).as_matrix()
    tv = np.asarray(tv, np.float64)
    P = np.asarray(w0["pose"], np.float64)
    w = dict(w0)
    w["means"] = (np.asarray(w0["means"], np.float64) @ M.T + tv).astype(np.float32)
    w["quats"] = U.quat_wxyz(M[None] @ U.rot_of_wxyz(np.asarray(w0["quats"], np.float64))).astype(np.float32)
    w["pose"] = U.pose_from(M @ P[:, :3], M @ P[:, 3] + tv).astype(np.float32)
    return w


def test_forward_room_general_rotation(ctx, room):
    """Forward parity at a general rigid pose: every entry of the pose rotation is far from
    zero, and the float32 pose is not exactly orthonormal.  Rays that meet the ground at
    grazing incidence are sensitive to the plane normal in proportion to 1/(n.d), which the
    sensor frame formed in float pairs keeps within the 1e-5 bar."""
    w = _moved(room, [0.4, -0.9, 0.6], [2.0, -5.0, 0.75])
    assert np.abs(w["pose"][:, :3]).min() > 0.05
    fr, st = G.gpu_forward(ctx, G.to_dev(w))
    torch.cuda.synchronize()
    of = G.oracle_forward(w)
    stats = G.compare_forward(fr, of)
    _print("forward room32x256_1k general rotation", stats)
    assert stats["tie"] < 0.01 * stats["rays"]
    st.free()


def test_backward_room_general_rotation(ctx, room):
    """The room and its pose moved by one rigid transform about a general axis: the image
    (and so the sensor-frame targets) stays the same, while every entry of the pose rotation
    is far from zero, so a mixed-up row or column of it in the chain cannot hide."""
    w = _moved(room, [0.4, -0.9, 0.6], [2.0, -5.0, 0.75])
    assert np.abs(w["pose"][:, :3]).min() > 0.05
    H, W = w["H"], w["W"]
    dw = G.to_dev(w)
    _, st = G.gpu_forward(ctx, dw)
    of = G.oracle_forward(w)
    mask = (~G.tie_mask(of)).astype(np.float64)
    gd, go, gn = _loss_upstream(w, of, mask=mask)
    rng = np.random.default_rng(4)
    go = (rng.normal(size=go.shape) * 1e-4 * mask).astype(np.float32)
    g_gpu, gp = _gpu_backward(ctx, dw, st, H, W, gd, go, gn)
    g_ref = ref.backward(w, w["pose"], w["row_sincos"], w["col_sincos"], gd, go, gn, with_mass=True)
    _check_grads("backward room32x256_1k general rotation", g_gpu, gp, g_ref)
    st.free()


def test_end_to_end_loss_and_grad(ctx, room):
    """forward -> loss -> backward entirely on the GPU vs the oracle's loss_and_grad.  The
    surfels sit on the raycast surfaces, so many rendered depths equal their targets
    exactly, at the corner of |x| where the sign is arbitrary; targets are moved off it."""
    from paper_2607_04127_amd import lgsr
    rng = np.random.default_rng(12)
    td = room["target_depth"]
    td = np.where(td > 0, td + rng.choice([-1, 1], td.shape) * rng.uniform(0.05, 0.3, td.shape), 0).astype(np.float32)
    w = dict(room, target_depth=td)
    dw = G.to_dev(w)
    fr, st = G.gpu_forward(ctx, dw)
    L, g = lgsr.lgsr_loss(ctx, fr, dw["target_depth"], dw["target_normal"])
    out, gp = lgsr.lgsr_backward(ctx, st, g)
    torch.cuda.synchronize()
    L_ref, of, g_ref = ref.loss_and_grad(w, w["pose"], w["row_sincos"], w["col_sincos"], w["target_depth"],
                                         w["target_normal"])
    np.testing.assert_allclose(L.cpu().numpy()[:3], L_ref[:3], rtol=1e-4)
    for key in G.SURF_KEYS:
        _, cos, _ = G.grad_check(out[key].cpu().numpy(), g_ref[key])
        assert cos > 0.999, (key, cos)
    _, cos, _ = G.grad_check(gp.cpu().numpy(), g_ref["pose"])
    assert cos > 0.999
    st.free()


# ------------------------------------------------------------------------------------------
# 64 x 1024 beams, 300,000 surfels: the benchmark configuration, sampled rays
# ------------------------------------------------------------------------------------------

def test_forward_block_full_image(ctx, block):
    """The benchmark configuration, every one of its 65,536 rays, in the launch
    configuration the benchmark times (automatic chunk length)."""
    dw = G.to_dev(block)
    fr, st = G.gpu_forward(ctx, dw)
    torch.cuda.synchronize()
    of = G.oracle_forward(block)
    stats = G.compare_forward(fr, of)
    from paper_2607_04127_amd import lgsr
    q = lgsr.lgsr_query(ctx, st)
    stats.update(pairs=q["pairs"], visible=q["visible"], max_list=q["max_list"], mean_K=float(of["K"].mean()),
                 composites=q["composites"], composites_oracle=int(of["K"].sum()))
    _print("forward block64x1024_300k (full image)", stats)
    assert stats["tie"] < 0.02 * stats["rays"]
    st.free()


@pytest.mark.parametrize("chunk", [64])
def test_forward_block_sampled(ctx, block, chunk):
    H, W = block["H"], block["W"]
    dw = G.to_dev(block)
    fr, st = G.gpu_forward(ctx, dw, chunk=chunk)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2024)
    ids = np.sort(rng.choice(H * W, size=4096, replace=False))
    of = G.oracle_forward(block, ray_ids=ids)
    stats = G.compare_forward(fr, of, ray_ids=ids)
    from paper_2607_04127_amd import lgsr
    q = lgsr.lgsr_query(ctx, st)
    stats.update(pairs=q["pairs"], visible=q["visible"], max_list=q["max_list"], mean_K=float(of["K"].mean()))
    _print(f"forward block64x1024_300k (4096 sampled rays) chunk={chunk}", stats)
    assert stats["tie"] < 0.02 * stats["rays"]
    st.free()


def _roll_pitch(w0, roll_deg=3.0, pitch_deg=-2.0):
    """The workload's pose turned by a few degrees of roll and pitch about the sensor (the
    kind of pose the pose optimiser produces); the targets are not used."""
    from scipy.spatial.transform import Rotation
    from tests import _util as U
    P = np.asarray(w0["pose"], np.float64)
    Rl = Rotation.from_euler("xy", [roll_deg, pitch_deg], degrees=True).as_matrix()
    w = dict(w0)
    w["pose"] = U.pose_from(P[:, :3] @ Rl, P[:, 3]).astype(np.float32)
    return w


def test_forward_block_roll_pitch(ctx, block):
    w = _roll_pitch(block)
    H, W = w["H"], w["W"]
    fr, st = G.gpu_forward(ctx, G.to_dev(w))
    torch.cuda.synchronize()
    rng = np.random.default_rng(2025)
    ids = np.sort(rng.choice(H * W, size=4096, replace=False))
    of = G.oracle_forward(w, ray_ids=ids)
    stats = G.compare_forward(fr, of, ray_ids=ids)
    _print("forward block64x1024_300k roll 3, pitch -2 degrees (4096 sampled rays)", stats)
    assert stats["tie"] < 0.02 * stats["rays"] and stats["hit"] > 1000
    st.free()


@pytest.mark.parametrize("chunk", [0, 64])
def test_backward_block_sampled(ctx, block, chunk):
    """Upstream gradient nonzero on 8192 sampled rays only: the renderer's full backward
    then equals the oracle's backward restricted to those rays, for every surfel."""
    H, W = block["H"], block["W"]
    dw = G.to_dev(block)
    _, st = G.gpu_forward(ctx, dw, chunk=chunk)
    rng = np.random.default_rng(77)
    ids = np.sort(rng.choice(H * W, size=8192 if chunk == 0 else 2048, replace=False))
    of = G.oracle_forward(block, ray_ids=ids)
    mask = (~G.tie_mask(of)).astype(np.float64)
    gd, go, gn = _loss_upstream(block, of, ray_ids=ids, mask=mask)
    g_gpu, gp = _gpu_backward(ctx, dw, st, H, W, gd, go, gn, ray_ids=ids)
    g_ref = ref.backward(block, block["pose"], block["row_sincos"], block["col_sincos"], gd, go, gn, ray_ids=ids,
                         with_mass=True)
    _check_grads(f"backward block64x1024_300k ({len(ids)} sampled rays) chunk={chunk}", g_gpu, gp, g_ref)
    st.free()


# ------------------------------------------------------------------------------------------
# edge cases
# ------------------------------------------------------------------------------------------

def _small_map(n, seed=0, scale=1.0):
    w = scenegen.make_workload("room32x256_1k")
    idx = np.random.default_rng(seed).choice(1000, size=n, replace=False)
    S = {k: np.ascontiguousarray(w[k][idx]) for k in G.SURF_KEYS}
    S["log_scales"] = (S["log_scales"] + np.float32(math.log(scale))).astype(np.float32)
    return S, w


def test_empty_map(ctx):
    row, col = scenegen.beam_tables(32, 256, -15, 15)
    w = dict(means=np.zeros((0, 3), np.float32), quats=np.zeros((0, 4), np.float32),
             log_scales=np.zeros((0, 2), np.float32), opacity_logits=np.zeros(0, np.float32),
             row_sincos=row, col_sincos=col, pose=np.hstack([np.eye(3), np.zeros((3, 1))]).astype(np.float32))
    fr, st = G.gpu_forward(ctx, G.to_dev(w))
    torch.cuda.synchronize()
    assert torch.all(fr["depth"] == 0) and torch.all(fr["drop"] == 1)
    g = dict(depth=torch.ones_like(fr["depth"]), opacity=torch.ones_like(fr["depth"]),
             normal=torch.ones_like(fr["normal"]))
    from paper_2607_04127_amd import lgsr
    out, gp = lgsr.lgsr_backward(ctx, st, g)
    torch.cuda.synchronize()
    assert torch.all(gp == 0)
    st.free()


@pytest.mark.parametrize("H,W", [(37, 250), (1, 64), (16, 17), (70, 1030)])
def test_ragged_grids(ctx, H, W):
    """Image sizes that are not multiples of the 16 x 16 tile or the 8 x 8 wave sub-tile."""
    S, w = _small_map(200, seed=H * 1000 + W, scale=3.0)
    row, col = scenegen.beam_tables(H, W, -15, 15)
    wl = dict(S, row_sincos=row, col_sincos=col, pose=w["pose"])
    fr, st = G.gpu_forward(ctx, G.to_dev(wl))
    torch.cuda.synchronize()
    of = G.oracle_forward(wl)
    stats = G.compare_forward(fr, of)
    assert stats["hit"] > 0
    st.free()


def test_wrap_and_near_surfels(ctx):
    """Surfels straddling azimuth 0, one near the sensor whose footprint covers every tile,
    one nearer than `near` (dropped), a zero quaternion (dropped), an edge-on surfel, and one
    whose centre lies beyond `near` while its plane is met nearer than `near` by the ray it
    faces (that hit is skipped; rays meeting it farther out hit it)."""
    from tests import _util as U
    row, col = scenegen.beam_tables(32, 256, -15, 15)
    D = scenegen.ray_dirs_f64(row, col).reshape(-1, 3)
    cen, frames, sc, al = [], [], [], []
    rng = np.random.default_rng(8)
    for k in range(40):  # around azimuth 0 at various ranges and sizes
        d = D[(k % 32) * 256 + (0 if k % 2 else 255)]
        r = rng.uniform(3, 30)
        cen.append(r * d)
        frames.append(U.frame_facing(-d + rng.normal(scale=0.2, size=3), spin=rng.uniform(0, 6.28)))
        sc.append(rng.uniform(0.02, 0.1, 2) * r)
        al.append(rng.uniform(0.3, 0.95))
    cen.append([0.0, 0.0, -1.0])  # 1 m below the sensor, 2 m wide: every ray in the lower half
    frames.append(U.frame_facing([0.0, 0.0, 1.0]))
    sc.append([2.0, 2.0])
    al.append(0.6)
    cen.append(0.1 * D[5000])  # nearer than 0.2 m
    frames.append(U.frame_facing(-D[5000]))
    sc.append([1.0, 1.0])
    al.append(0.9)
    cen.append(10 * D[3000])  # edge-on
    frames.append(U.frame_facing(np.cross(D[3000], [0.0, 0.0, 1.0])))
    sc.append([1.0, 1.0])
    al.append(0.9)
    i_near = 5 * 256 + 100  # upper half, away from the surfels above
    e = np.cross(D[i_near], [0.0, 0.0, 1.0])
    e /= np.linalg.norm(e)
    cen.append(0.15 * D[i_near] + 0.25 * e)  # centre 0.29 m away; met at t = 0.15 m, 1.25 sigma off centre
    frames.append(U.frame_facing(-D[i_near]))
    sc.append([0.2, 0.2])
    al.append(0.9)
    S = {k: v.astype(np.float32) for k, v in U.surfels(cen, frames, sc, al).items()}
    S["quats"][3] = 0.0  # zero quaternion: renders nothing
    wl = dict(S, row_sincos=row, col_sincos=col, pose=np.hstack([np.eye(3), np.zeros((3, 1))]).astype(np.float32))
    fr, st = G.gpu_forward(ctx, G.to_dev(wl))
    torch.cuda.synchronize()
    of = G.oracle_forward(wl)
    stats = G.compare_forward(fr, of)
    _print("wrap/near", stats)
    seam = of["K"].reshape(32, 256)
    assert seam[:, 0].sum() > 0 and seam[:, 255].sum() > 0
    assert of["K"][i_near] == 0 and float(fr["opacity"].reshape(-1)[i_near]) == 0.0
    st.free()
