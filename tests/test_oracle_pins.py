"""Pins of the FP64 oracle against facts fixed by the paper's definitions and by mathematics,
not by the oracle's own formulas: closed forms, invariants, symmetries, independent library
routines (scipy rotations, numpy linear solves) and central finite differences.

Paper: arXiv 2607.04127 -- Sec. 3.1 (map of 2D Gaussian primitives rendered under the
spherical projection into depth/opacity/normals), Sec. 3.4 (masked depth L1 and cosine
normal loss, Eq. 10 left and Eq. 11 first term), Sec. 4.1 (loss weights).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenegen
from tests import _util as U

PRM = dict(cutoff_sigma=3.0, alpha_thr=1 / 255, alpha_max=0.99, T_min=1e-4, near=0.2, den_eps=1e-6,
           drop_tau=0.5)


@pytest.fixture(scope="module")
def ref(oracle_lib):
    return oracle_lib


@pytest.fixture(scope="module")
def beams():
    return scenegen.beam_tables(32, 256, -15.0, 15.0)


def _dirs(rows, cols):
    return scenegen.ray_dirs_f64(rows, cols).reshape(-1, 3)


# ------------------------------------------------------------------------------------------
# P1: one surfel seen head-on (closed form on its axis ray, linear-solve route elsewhere)
# ------------------------------------------------------------------------------------------

def test_head_on_surfel_closed_form(ref, beams):
    rows, cols = beams
    D = _dirs(rows, cols)
    k0, j0 = 13, 40
    d0 = D[k0 * 256 + j0]
    r, alpha, s = 12.5, 0.7, (0.9, 0.5)
    F = U.frame_facing(-d0, spin=0.4)
    S = U.surfels(r * d0, F[None], [s], [alpha])
    out = ref.forward(S, U.identity_pose(), rows, cols, PRM)
    i0 = k0 * 256 + j0
    assert out["K"][i0] == 1
    assert out["depth"][i0] == pytest.approx(r, rel=1e-14)
    assert out["opacity"][i0] == pytest.approx(alpha, rel=1e-14)
    np.testing.assert_allclose(out["normal"][i0], -d0, atol=1e-14)

    # every other ray: intersection from an independent 3x3 solve d t - a (s0 u) - b (s1 v) = mu
    a, b = F[:, 0], F[:, 1]
    exp_op = np.zeros(D.shape[0])
    exp_depth = np.zeros(D.shape[0])
    for i, d in enumerate(D):
        M = np.stack([d, -a, -b], axis=1)
        t, su, sv = np.linalg.solve(M, r * d0)
        u, v = su / s[0], sv / s[1]
        q2 = u * u + v * v
        if t < 0.2 or q2 > 9:
            continue
        ah = min(0.99, alpha * math.exp(-q2 / 2))
        if ah < 1 / 255:
            continue
        exp_op[i], exp_depth[i] = ah, t
    hit = exp_op > 0
    assert hit.sum() > 20  # the footprint spans many rays
    np.testing.assert_allclose(out["opacity"], exp_op, rtol=1e-10, atol=1e-300)
    np.testing.assert_allclose(out["depth"], exp_depth, rtol=1e-10, atol=1e-300)
    np.testing.assert_array_equal(out["K"], hit.astype(np.int32))
    np.testing.assert_allclose(out["normal"][hit], np.broadcast_to(-d0, (hit.sum(), 3)), atol=1e-14)
    np.testing.assert_array_equal(out["drop"], (exp_op < 0.5).astype(np.uint8))


# ------------------------------------------------------------------------------------------
# P2: two stacked surfels -> two-layer compositing, order by range not index
# ------------------------------------------------------------------------------------------

def test_two_stacked_surfels(ref, beams):
    rows, cols = beams
    D = _dirs(rows, cols)
    i0 = 7 * 256 + 100
    d0 = D[i0]
    r1, r2, a1, a2 = 8.0, 9.5, 0.6, 0.8
    F = U.frame_facing(-d0)
    # the far surfel first in index order: compositing must still go near to far
    S = U.surfels([r2 * d0, r1 * d0], [F, F], [(1.0, 1.0), (1.0, 1.0)], [a2, a1])
    out = ref.forward(S, U.identity_pose(), rows, cols, PRM, ray_ids=[i0])
    A = 1 - (1 - a1) * (1 - a2)
    assert out["opacity"][0] == pytest.approx(A, rel=1e-14)
    assert out["depth"][0] == pytest.approx((a1 * r1 + (1 - a1) * a2 * r2) / A, rel=1e-14)
    assert out["t_final"][0] == pytest.approx((1 - a1) * (1 - a2), rel=1e-13)
    S2 = {k: v[::-1].copy() for k, v in S.items()}
    out2 = ref.forward(S2, U.identity_pose(), rows, cols, PRM, ray_ids=[i0])
    assert out2["depth"][0] == out["depth"][0] and out2["opacity"][0] == out["opacity"][0]


# ------------------------------------------------------------------------------------------
# P3: weights and the final transmittance telescope to 1
# ------------------------------------------------------------------------------------------

def test_telescoping(ref):
    w = scenegen.make_workload("room32x256_1k")
    out = ref.forward(w, w["pose"], w["row_sincos"], w["col_sincos"], PRM)
    assert (out["K"] > 0).mean() > 0.5
    np.testing.assert_allclose(out["opacity"] + out["t_final"], 1.0, atol=1e-13)
    assert np.all(out["opacity"][out["K"] == 0] == 0)


# ------------------------------------------------------------------------------------------
# P4: early termination after the hit that takes T below T_min
# ------------------------------------------------------------------------------------------

def test_termination(ref, beams):
    rows, cols = beams
    D = _dirs(rows, cols)
    i0 = 20 * 256 + 3
    d0 = D[i0]
    F = U.frame_facing(-d0)
    n = 10
    S = U.surfels([(10.0 + k) * d0 for k in range(n)], [F] * n, [(1.0, 1.0)] * n, [0.8] * n)
    out = ref.forward(S, U.identity_pose(), rows, cols, PRM, ray_ids=[i0])
    # T = 0.2^k: 0.2^5 = 3.2e-4 >= 1e-4 > 0.2^6 = 6.4e-5 -> exactly six hits
    assert out["K"][0] == 6
    assert out["opacity"][0] == pytest.approx(1 - 0.2 ** 6, rel=1e-14)
    expect_d = sum(0.8 * 0.2 ** k * (10.0 + k) for k in range(6)) / (1 - 0.2 ** 6)
    assert out["depth"][0] == pytest.approx(expect_d, rel=1e-14)


# ------------------------------------------------------------------------------------------
# P5/P6: opacity clamp and the alpha threshold
# ------------------------------------------------------------------------------------------

def test_clamp_and_alpha_threshold(ref, beams):
    rows, cols = beams
    D = _dirs(rows, cols)
    i0 = 16 * 256 + 64
    d0 = D[i0]
    F = U.frame_facing(-d0)
    S = U.surfels([10 * d0], [F], [(1.0, 1.0)], [0.5])
    S["opacity_logits"][:] = 20.0
    out = ref.forward(S, U.identity_pose(), rows, cols, PRM, ray_ids=[i0])
    assert out["opacity"][0] == float(np.float32(0.99))  # the float32 clamp value

    # alpha G just below / above 1/255 on the axis ray: G = 1 so alpha decides
    thr = float(np.float32(1 / 255))
    for alpha, k in ((thr * (1 - 1e-6), 0), (thr * (1 + 1e-6), 1)):
        S = U.surfels([10 * d0], [F], [(1.0, 1.0)], [alpha])
        out = ref.forward(S, U.identity_pose(), rows, cols, PRM, ray_ids=[i0])
        assert out["K"][0] == k
        assert out["drop"][0] == 1


# ------------------------------------------------------------------------------------------
# P7: 360 degree wrap -- a yaw of the sensor rolls the range image
# ------------------------------------------------------------------------------------------

def _yaw(theta):
    return Rotation.from_euler("z", theta).as_matrix()


def test_wrap_quarter_turn_rolls_image(ref):
    w = scenegen.make_workload("room32x256_1k")
    H, W = w["H"], w["W"]
    base = ref.forward(w, U.identity_pose(), w["row_sincos"], w["col_sincos"], PRM)
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])  # exact quarter turn
    rot = ref.forward(w, U.pose_from(Rz, np.zeros(3)), w["row_sincos"], w["col_sincos"], PRM)
    q = W // 4
    for key in ("depth", "opacity", "t_final"):
        exp = np.roll(base[key].reshape(H, W), -q, axis=1)
        np.testing.assert_allclose(rot[key].reshape(H, W), exp, rtol=1e-12, atol=1e-300)
    n_exp = np.roll(base["normal"].reshape(H, W, 3), -q, axis=1) @ Rz  # R^T n, row form
    np.testing.assert_allclose(rot["normal"].reshape(H, W, 3), n_exp, atol=1e-12)
    assert (base["K"] > 0).sum() > 1000


def test_wrap_one_column(ref):
    """Yaw by one column (2 pi / W): the image rolls by one column, including rays whose
    footprint straddles azimuth 0 (tolerance covers the float32 rounding of the tables)."""
    w = scenegen.make_workload("room32x256_1k")
    H, W = w["H"], w["W"]
    base = ref.forward(w, U.identity_pose(), w["row_sincos"], w["col_sincos"], PRM, extra=True)
    rot = ref.forward(w, U.pose_from(_yaw(2 * np.pi / W), np.zeros(3)), w["row_sincos"],
                      w["col_sincos"], PRM, extra=True)
    bd = np.roll(base["opacity"].reshape(H, W), -1, axis=1)
    bm = np.roll(base["margin"].reshape(H, W), -1, axis=1)
    ok = (bm > 1e-3) & (rot["margin"].reshape(H, W) > 1e-3)
    assert ok.mean() > 0.95
    np.testing.assert_allclose(rot["opacity"].reshape(H, W)[ok], bd[ok], rtol=1e-4, atol=1e-9)
    # the seam columns are part of the comparison
    assert ok[:, 0].any() and ok[:, -1].any()


# ------------------------------------------------------------------------------------------
# P8: symmetries of the primitive; P9: rigid equivariance of map + pose
# ------------------------------------------------------------------------------------------

def _compose_local(S, R_local, swap_scales=False):
    Rm = U.rot_of_wxyz(S["quats"]) @ R_local
    out = dict(S)
    out["quats"] = U.quat_wxyz(Rm) * np.linalg.norm(S["quats"], axis=1, keepdims=True)
    if swap_scales:
        out["log_scales"] = S["log_scales"][:, ::-1].copy()
    return out


def test_flip_about_tangent_axis_is_invisible(ref):
    w = scenegen.make_workload("room32x256_1k")
    S = {k: np.asarray(w[k], np.float64) for k in ("means", "quats", "log_scales", "opacity_logits")}
    base = ref.forward(S, w["pose"], w["row_sincos"], w["col_sincos"], PRM)
    flip = np.diag([1.0, -1.0, -1.0])  # pi about a: n -> -n, b -> -b
    out = ref.forward(_compose_local(S, flip), w["pose"], w["row_sincos"], w["col_sincos"], PRM)
    for key in ("depth", "opacity", "normal"):
        np.testing.assert_allclose(out[key], base[key], rtol=1e-9, atol=1e-12)


def test_swap_tangent_axes_with_scales_is_invisible(ref):
    w = scenegen.make_workload("room32x256_1k")
    S = {k: np.asarray(w[k], np.float64) for k in ("means", "quats", "log_scales", "opacity_logits")}
    base = ref.forward(S, w["pose"], w["row_sincos"], w["col_sincos"], PRM)
    swap = np.array([[0.0, 1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, -1.0]])  # [b a -n]
    out = ref.forward(_compose_local(S, swap, swap_scales=True), w["pose"], w["row_sincos"],
                      w["col_sincos"], PRM)
    for key in ("depth", "opacity", "normal"):
        np.testing.assert_allclose(out[key], base[key], rtol=1e-9, atol=1e-12)


def test_rigid_equivariance(ref):
    w = scenegen.make_workload("room32x256_1k")
    S = {k: np.asarray(w[k], np.float64) for k in ("means", "quats", "log_scales", "opacity_logits")}
    base = ref.forward(S, w["pose"], w["row_sincos"], w["col_sincos"], PRM)
    M = Rotation.from_rotvec([0.3, -1.1, 0.7]).as_matrix()
    tv = np.array([3.0, -7.5, 1.25])
    S2 = dict(S)
    S2["means"] = S["means"] @ M.T + tv
    S2["quats"] = U.quat_wxyz(M[None] @ U.rot_of_wxyz(S["quats"]))
    P = np.asarray(w["pose"], np.float64)
    P2 = U.pose_from(M @ P[:, :3], M @ P[:, 3] + tv)
    out = ref.forward(S2, P2, w["row_sincos"], w["col_sincos"], PRM)
    for key in ("depth", "opacity", "normal"):
        np.testing.assert_allclose(out[key], base[key], rtol=1e-9, atol=1e-11)


# ------------------------------------------------------------------------------------------
# Coplanar surfels: depth equals the analytic plane hit and the normal the plane normal
# ------------------------------------------------------------------------------------------

def test_coplanar_surfels_render_the_plane(ref, beams):
    rows, cols = beams
    rng = np.random.default_rng(7)
    n = 300
    xy = rng.uniform(-15, 15, size=(n, 2))
    centers = np.column_stack([xy, np.full(n, -1.7)])
    frames = [U.frame_facing([0.0, 0.0, 1.0], spin=s) for s in rng.uniform(0, 2 * np.pi, n)]
    S = U.surfels(centers, frames, rng.uniform(0.3, 1.5, size=(n, 2)), rng.uniform(0.3, 0.95, n))
    out = ref.forward(S, U.identity_pose(), rows, cols, PRM)
    D = _dirs(rows, cols)
    hit = out["K"] > 0
    assert hit.sum() > 200
    t_plane = -1.7 / D[hit, 2]
    np.testing.assert_allclose(out["depth"][hit], t_plane, rtol=1e-12)
    np.testing.assert_allclose(out["normal"][hit], np.broadcast_to([0.0, 0.0, 1.0], (hit.sum(), 3)),
                               atol=1e-13)


# ------------------------------------------------------------------------------------------
# P15: empty map, near surfel, edge-on surfel
# ------------------------------------------------------------------------------------------

def test_edge_cases(ref, beams):
    rows, cols = beams
    empty = dict(means=np.zeros((0, 3)), quats=np.zeros((0, 4)), log_scales=np.zeros((0, 2)),
                 opacity_logits=np.zeros(0))
    out = ref.forward(empty, U.identity_pose(), rows, cols, PRM)
    assert np.all(out["K"] == 0) and np.all(out["drop"] == 1) and np.all(out["depth"] == 0)
    D = _dirs(rows, cols)
    i0 = 10 * 256 + 10
    d0 = D[i0]
    # nearer than 0.2 m: dropped even though its footprint covers the ray
    S = U.surfels([0.15 * d0], [U.frame_facing(-d0)], [(1.0, 1.0)], [0.9])
    assert ref.forward(S, U.identity_pose(), rows, cols, PRM, ray_ids=[i0])["K"][0] == 0
    # the near rule applies per hit: a surfel facing the ray with its centre 0.29 m away
    # (beyond 0.2 m) but its plane met by the ray at t = 0.15 m gives no hit; moved back so
    # the ray meets it at 0.30 m, it gives one hit at exactly that depth
    e = np.cross(d0, [0.0, 0.0, 1.0])
    e /= np.linalg.norm(e)
    for t_hit, want_k in ((0.15, 0), (0.30, 1)):
        S = U.surfels([t_hit * d0 + 0.25 * e], [U.frame_facing(-d0)], [(1.0, 1.0)], [0.9])
        out = ref.forward(S, U.identity_pose(), rows, cols, PRM, ray_ids=[i0])
        assert out["K"][0] == want_k, t_hit
        if want_k:
            assert out["depth"][0] == pytest.approx(t_hit, rel=1e-12)
    # edge-on: normal orthogonal to the ray through its centre
    F = U.frame_facing(np.cross(d0, [0.0, 0.0, 1.0]))
    S = U.surfels([10 * d0], [F], [(1.0, 1.0)], [0.9])
    assert ref.forward(S, U.identity_pose(), rows, cols, PRM, ray_ids=[i0])["K"][0] == 0


# ------------------------------------------------------------------------------------------
# Loss (Eq. 10 left, Eq. 11 first term) on hand-checked numbers
# ------------------------------------------------------------------------------------------

def test_loss_hand_values(ref):
    depth = np.array([10.0, 5.0, 0.0, 7.0])
    normal = np.array([[0.0, 0.0, 2.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 3.0, 4.0]])
    td = np.array([9.0, 0.0, 3.0, 7.5])
    tn = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 0.0]])
    pred = dict(depth=depth, opacity=np.ones(4), normal=normal)
    L, gd, go, gn = ref.loss(pred, td, tn)
    # Omega_D = {0, 2, 3}; Omega_N = {0, 2}
    exp_d = (1.0 + 3.0 + 0.5) / 3
    lng = float(np.float32(0.05))  # weights reach the renderer as float32
    exp_n = lng * ((1 - 1.0) + 1.0) / 2  # ray 2 renders no normal: cost 1
    assert L[1] == pytest.approx(exp_d, rel=1e-15)
    assert L[2] == pytest.approx(exp_n, rel=1e-15)
    assert L[0] == pytest.approx(exp_d + exp_n, rel=1e-15)
    assert (L[3], L[4]) == (3.0, 2.0)
    np.testing.assert_allclose(gd, [1 / 3, 0.0, -1 / 3, -1 / 3], rtol=1e-15)
    assert np.all(go == 0)
    # ray 0: N_hat = (0,0,2) parallel to N -> the cosine is stationary
    np.testing.assert_allclose(gn[0], 0.0, atol=1e-17)
    assert np.all(gn[1:] == 0)
    # a tilted normal: gradient against a numerical derivative of 1 - cos
    pred2 = dict(depth=depth, opacity=np.ones(4), normal=np.array([[0.3, -0.2, 0.9]] + normal[1:].tolist()))
    _, _, _, gn2 = ref.loss(pred2, td, tn)
    f = lambda v: lng * (1 - v @ tn[0] / np.linalg.norm(v)) / 2  # noqa: E731
    v0 = pred2["normal"][0]
    num = np.array([(f(v0 + e) - f(v0 - e)) / 2e-7 for e in np.eye(3) * 1e-7])
    np.testing.assert_allclose(gn2[0], num, rtol=1e-6)


# ------------------------------------------------------------------------------------------
# P10: every gradient against central finite differences of the oracle's own loss
# ------------------------------------------------------------------------------------------

def _fd_scene():
    """A 12x48 window of the 32x256 beam model looking at ~60 surfels of the room scene."""
    w = scenegen.make_workload("room32x256_1k")
    rows = w["row_sincos"][10:22]
    cols = w["col_sincos"][20:68]
    S = {k: np.asarray(w[k], np.float64) for k in ("means", "quats", "log_scales", "opacity_logits")}
    pose = np.asarray(w["pose"], np.float64)
    # keep surfels whose azimuth falls near the window
    az = np.arctan2(S["means"][:, 1], S["means"][:, 0])
    th0, th1 = 2 * np.pi * 20 / 256, 2 * np.pi * 68 / 256
    keep = (az > th0 - 0.3) & (az < th1 + 0.3)
    S = {k: v[keep].copy() for k, v in S.items()}
    tg_d, tg_n = scenegen.targets_for_pose(w["scene"], pose, rows.astype(np.float32),
                                           cols.astype(np.float32))
    return S, pose, rows, cols, tg_d, tg_n


def _fd_check(S, pose, g, func, n_surf=10, hs=(1e-6, 1e-7, 1e-7, 1e-7), seed=11):
    """Central differences of ``func(S, pose)`` against the analytic gradient ``g`` for every
    parameter of ``n_surf`` touched surfels and the six pose directions."""
    rng = np.random.default_rng(seed)
    touched = np.nonzero(np.abs(g["opacity_logits"]) > 0)[0]
    assert touched.size > 10
    checks = []
    for i in rng.choice(touched, size=min(n_surf, touched.size), replace=False):
        for (key, width), h in zip((("means", 3), ("quats", 4), ("log_scales", 2), ("opacity_logits", 1)), hs):
            for c in range(width):
                Sp = {k: v.copy() for k, v in S.items()}
                Sm = {k: v.copy() for k, v in S.items()}
                idx = (i,) if width == 1 else (i, c)
                Sp[key][idx] += h
                Sm[key][idx] -= h
                fd = (func(Sp, pose) - func(Sm, pose)) / (2 * h)
                checks.append((key, int(i), c, float(g[key][idx]), fd))
    for c in range(6):
        h = 1e-7
        xi = np.zeros(6)
        xi[c] = h
        fd = (func(S, U.right_perturb(pose, xi)) - func(S, U.right_perturb(pose, -xi))) / (2 * h)
        checks.append(("pose", -1, c, float(g["pose"][c]), fd))
    ana = np.array([x[3] for x in checks])
    fd = np.array([x[4] for x in checks])
    scale = np.abs(fd).max()
    assert scale > 0
    bad = np.abs(ana - fd) > 1e-5 * np.maximum(np.abs(fd), 1e-3 * scale)
    # a central difference straddling a threshold event is not a derivative: allow at most
    # one such straddle among the ~106 checks
    assert bad.sum() <= 1, [checks[i] for i in np.nonzero(bad)[0]]


def test_render_backward_matches_finite_differences(ref):
    """Backward of the renderer: gradient of a fixed random linear functional of the
    rendered depth, opacity and normal (all three paths at once)."""
    S, pose, rows, cols, _, _ = _fd_scene()
    n = rows.shape[0] * cols.shape[0]
    rng = np.random.default_rng(5)
    gD, gA, gN = rng.normal(size=n), rng.normal(size=n), rng.normal(size=(n, 3))
    # a third of the surfels nearly opaque, so that alpha G > alpha_max clamps near their centres
    opaque = rng.uniform(size=S["opacity_logits"].shape[0]) < 0.35
    S["opacity_logits"] = np.where(opaque, rng.uniform(5.0, 8.0, opaque.shape), S["opacity_logits"])

    def func(S_, P_):
        f = ref.forward(S_, P_, rows, cols, PRM)
        return (gD * f["depth"]).sum() + (gA * f["opacity"]).sum() + (gN * f["normal"]).sum()

    g = ref.backward(S, pose, rows, cols, gD, gA, gN, PRM)
    _fd_check(S, pose, g, func)


def test_render_backward_finite_differences_under_a_rotated_pose(ref):
    """The same check after moving the scene and the pose by one rigid transform: the image
    does not change, but every surfel and pose gradient now passes through a sensor-to-world
    rotation that is not the identity (the scene's own pose is)."""
    S, pose, rows, cols, _, _ = _fd_scene()
    M = Rotation.from_rotvec([0.4, -0.9, 0.6]).as_matrix()
    tv = np.array([2.0, -5.0, 0.75])
    S2 = dict(S)
    S2["means"] = S["means"] @ M.T + tv
    S2["quats"] = U.quat_wxyz(M[None] @ U.rot_of_wxyz(S["quats"]))
    P2 = U.pose_from(M @ pose[:, :3], M @ pose[:, 3] + tv)
    n = rows.shape[0] * cols.shape[0]
    rng = np.random.default_rng(6)
    gD, gA, gN = rng.normal(size=n), rng.normal(size=n), rng.normal(size=(n, 3))

    def func(S_, P_):
        f = ref.forward(S_, P_, rows, cols, PRM)
        return (gD * f["depth"]).sum() + (gA * f["opacity"]).sum() + (gN * f["normal"]).sum()

    g = ref.backward(S2, P2, rows, cols, gD, gA, gN, PRM)
    _fd_check(S2, P2, g, func)


def test_loss_gradients_match_finite_differences(ref):
    """Forward + loss (Eq. 10 left, Eq. 11 first term) + backward.  Surfels sit on the scanned surfaces, so many
    rendered depths equal their raycast targets exactly, at the corner of |x|; the targets
    are moved off it by a random 5-30 cm so the central differences are derivatives."""
    S, pose, rows, cols, td, tn = _fd_scene()
    rng = np.random.default_rng(9)
    td = np.where(td > 0, td + rng.choice([-1, 1], td.shape) * rng.uniform(0.05, 0.3, td.shape), 0.0)
    L, fw, g = ref.loss_and_grad(S, pose, rows, cols, td, tn, PRM)
    assert (fw["K"] > 0).mean() > 0.3 and L[0] > 0

    def func(S_, P_):
        return ref.loss(ref.forward(S_, P_, rows, cols, PRM), td, tn)[0][0]

    _fd_check(S, pose, g, func)


# ------------------------------------------------------------------------------------------
# P11: the pure-Python restatement agrees with the C oracle on tiny inputs
# ------------------------------------------------------------------------------------------

def test_tiny_restatement_agrees(ref):
    from oracle import tiny
    w = scenegen.make_workload("room32x256_1k")
    rng = np.random.default_rng(3)
    idx = rng.choice(1000, size=16, replace=False)
    S = {k: np.asarray(w[k], np.float64)[idx] for k in ("means", "quats", "log_scales", "opacity_logits")}
    # enlarge so the few surfels cover many rays
    S["log_scales"] = S["log_scales"] + 1.5
    rows, cols = w["row_sincos"][8:16], w["col_sincos"][0:256:4]
    out = ref.forward(S, w["pose"], rows, cols, PRM)
    lit = tiny.render(S["means"], S["quats"], S["log_scales"], S["opacity_logits"], w["pose"], rows, cols,
                      alpha_thr=float(np.float32(1 / 255)), alpha_max=float(np.float32(0.99)),
                      T_min=float(np.float32(1e-4)), near=float(np.float32(0.2)),
                      den_eps=float(np.float32(1e-6)))
    assert sum(x[4] for x in lit) > 20
    np.testing.assert_allclose(out["depth"], [x[0] for x in lit], rtol=1e-12)
    np.testing.assert_allclose(out["opacity"], [x[1] for x in lit], rtol=1e-12)
    np.testing.assert_allclose(out["normal"], [x[2] for x in lit], atol=1e-12)
    np.testing.assert_array_equal(out["K"], [x[4] for x in lit])


# ------------------------------------------------------------------------------------------
# Gradient mass (used by the GPU tolerances): it bounds the gradient (triangle inequality)
# and equals its norm when a single ray contributes
# ------------------------------------------------------------------------------------------

def test_gradient_mass_bounds_gradient(ref):
    S, pose, rows, cols, td, tn = _fd_scene()
    n = rows.shape[0] * cols.shape[0]
    rng = np.random.default_rng(21)
    gD, gA, gN = rng.normal(size=n), rng.normal(size=n), rng.normal(size=(n, 3))
    g = ref.backward(S, pose, rows, cols, gD, gA, gN, PRM, with_mass=True)
    m = g["mass"]
    assert np.all(m >= 0) and m[:, 3].max() > 0
    for k, key in enumerate(("means", "quats", "log_scales")):
        assert np.all(np.linalg.norm(g[key], axis=1) <= m[:, k] * (1 + 1e-12) + 1e-300)
    assert np.all(np.abs(g["opacity_logits"]) <= m[:, 3] * (1 + 1e-12) + 1e-300)
    assert np.all(np.abs(g["pose"]) <= g["pose_mass"] * (1 + 1e-12))
    # where the signed terms do not cancel (one ray, one contributor, depth upstream only),
    # the opacity mass is the gradient's own magnitude
    fw = ref.forward(S, pose, rows, cols, PRM)
    single = np.nonzero(fw["K"] == 1)[0]
    assert single.size > 0
    one = np.zeros(n)
    one[single[0]] = 1.0
    g1 = ref.backward(S, pose, rows, cols, np.zeros(n), one, np.zeros((n, 3)), PRM, with_mass=True)
    np.testing.assert_allclose(np.abs(g1["opacity_logits"]), g1["mass"][:, 3], rtol=1e-12, atol=1e-300)
