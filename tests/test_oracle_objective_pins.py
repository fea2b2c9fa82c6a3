"""Pins of the oracle's full mapping objective (Sec. 3.4): the rendered-surface normal N_surf
(Sec. 3.4 (ii)) against closed forms (a sphere about the sensor, planes), mirror symmetries
that hold only for central differences, and invariance under a turn of the sensor by whole
columns (the azimuth wrap-around); the loss terms of Eq. 10-13 against closed forms; every
gradient against central finite differences of the oracle's own loss."""
import math

import numpy as np
import pytest

import scenegen
from oracle import ref


def _tables(H, W, el_deg, az0=0.0):
    """float64 beam tables: elevations uniform over el_deg (row 0 first), azimuths
    az0 + 2 pi j / W, exact to float64 rounding."""
    el = np.radians(np.linspace(el_deg[0], el_deg[1], H))
    az = az0 + 2.0 * np.pi * np.arange(W) / W
    return np.stack([np.sin(el), np.cos(el)], 1), np.stack([np.sin(az), np.cos(az)], 1)


def _dirs(rows, cols):
    sp, cp = rows[:, 0][:, None], rows[:, 1][:, None]
    st, ct = cols[:, 0][None, :], cols[:, 1][None, :]
    return np.stack([cp * ct, cp * st, sp * np.ones_like(ct)], -1)  # (H, W, 3)


# ------------------------------------------------------------------------------------------
# N_surf
# ------------------------------------------------------------------------------------------

def test_sphere_about_the_sensor_faces_it():
    """Constant range r: with uniform elevation steps the two central differences are exact
    tangents, so N_surf = -d on every row with both row neighbours, all columns."""
    H, W = 9, 24
    rows, cols = _tables(H, W, (-20, 20))
    ns, ok, _ = ref.surf_normal(rows, cols, np.full(H * W, 7.5))
    ok = ok.reshape(H, W).astype(bool)
    assert not ok[0].any() and not ok[-1].any() and ok[1:-1].all()
    d = _dirs(rows, cols).reshape(-1, 3)
    np.testing.assert_allclose(ns[ok.reshape(-1)], -d[ok.reshape(-1)], atol=1e-12)


@pytest.mark.parametrize("nrm,c", [((0.0, 0.0, 1.0), -1.7), ((0.15, -0.1, 1.0), -2.0), ((-0.2, 0.3, 1.0), -1.2)])
def test_planes_give_their_normal(nrm, c):
    """Points of a plane n.P = c (c < 0: the sensor on the side n points to): any two
    non-parallel in-plane differences span it, so N_surf = n / |n| exactly, at every defined
    pixel including both seam columns."""
    H, W = 12, 32
    rows, cols = _tables(H, W, (-55, -25), az0=0.3)
    n = np.asarray(nrm) / np.linalg.norm(nrm)
    d = _dirs(rows, cols)
    nd = d @ n
    assert (nd < 0).all()
    depth = (c / np.linalg.norm(nrm)) / nd
    ns, ok, _ = ref.surf_normal(rows, cols, depth.reshape(-1))
    ok = ok.astype(bool)
    assert ok.sum() == (H - 2) * W
    np.testing.assert_allclose(ns[ok], np.broadcast_to(n, (ok.sum(), 3)), atol=1e-10)


def test_undefined_next_to_missing_ranges():
    """A pixel needs rendered ranges at its four neighbours (not at itself)."""
    H, W = 7, 10
    rows, cols = _tables(H, W, (-10, 10))
    depth = np.full((H, W), 5.0)
    depth[3, 4] = 0.0
    _, ok, _ = ref.surf_normal(rows, cols, depth.reshape(-1))
    ok = ok.reshape(H, W).astype(bool)
    for k, j in [(3, 3), (3, 5), (2, 4), (4, 4)]:
        assert not ok[k, j]
    assert ok[3, 4] and ok[1:-1].sum() == (H - 2) * W - 4


def _orthonormal_basis(rows, cols, k, j):
    el = math.atan2(rows[k, 0], rows[k, 1])
    az = math.atan2(cols[j, 0], cols[j, 1])
    e_az = np.array([-math.sin(az), math.cos(az), 0.0])
    e_el = np.array([-math.sin(el) * math.cos(az), -math.sin(el) * math.sin(az), math.cos(el)])
    return e_az, e_el


def test_mirror_symmetry_needs_central_differences():
    """A range image mirror-symmetric in azimuth about column 0 (through the seam) and in
    elevation about the middle row gives, at those pixels, a normal with no component along
    the mirrored direction.  One-sided differences, or a seam that does not wrap, break it."""
    H, W = 11, 40
    k0 = H // 2
    rows, cols = _tables(H, W, (-15, 15))
    rng = np.random.default_rng(3)
    base = rng.uniform(6.0, 9.0, size=(H, W))
    jm = (-np.arange(W)) % W
    sym = 0.5 * (base + base[:, jm])           # D(k, j) = D(k, -j)
    sym = 0.5 * (sym + sym[::-1])              # D(k0 + m, j) = D(k0 - m, j)
    ns, ok, _ = ref.surf_normal(rows, cols, sym.reshape(-1))
    ns = ns.reshape(H, W, 3)
    for k in range(1, H - 1):
        e_az, _ = _orthonormal_basis(rows, cols, k, 0)
        assert abs(ns[k, 0] @ e_az) < 1e-12, k
        e_az, _ = _orthonormal_basis(rows, cols, k, W // 2)
        assert abs(ns[k, W // 2] @ e_az) < 1e-12, k
    for j in range(W):
        _, e_el = _orthonormal_basis(rows, cols, k0, j)
        assert abs(ns[k0, j] @ e_el) < 1e-12, j
    # and the image is not trivial: elsewhere the normals do lean along both
    e_az, e_el = _orthonormal_basis(rows, cols, 2, 7)
    assert abs(ns[2, 7] @ e_az) > 1e-3 and abs(ns[2, 7] @ e_el) > 1e-3


def test_turning_the_sensor_by_whole_columns():
    """Shifting a range image by s columns (uniform azimuths over the full turn) is the same
    surface seen by a sensor turned by s steps: N_surf shifts by s and turns by the same angle
    about z, also for the pixels whose stencil crosses the seam."""
    H, W, s = 8, 36, 5
    rows, cols = _tables(H, W, (-12, 12))
    rng = np.random.default_rng(8)
    depth = rng.uniform(4.0, 12.0, size=(H, W))
    n0, ok0, _ = ref.surf_normal(rows, cols, depth.reshape(-1))
    n1, ok1, _ = ref.surf_normal(rows, cols, np.roll(depth, s, axis=1).reshape(-1))
    a = 2.0 * np.pi * s / W
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    n0, n1 = n0.reshape(H, W, 3), n1.reshape(H, W, 3)
    np.testing.assert_array_equal(np.roll(ok0.reshape(H, W), s, axis=1), ok1.reshape(H, W))
    np.testing.assert_allclose(np.roll(n0 @ Rz.T, s, axis=1), n1, atol=1e-12)


# ------------------------------------------------------------------------------------------
# loss terms: closed forms
# ------------------------------------------------------------------------------------------

def _sphere_case(H=9, W=24, r=6.0):
    rows, cols = _tables(H, W, (-20, 20))
    d = _dirs(rows, cols).reshape(-1, 3)
    depth = np.full(H * W, r)
    return rows, cols, d, depth


def test_closed_form_terms_and_denominators():
    """Sphere image, target valid on a subset Omega_D, G-ICP normals on a smaller subset:
    depth term = w c for |D^ - D| = c; opacity term = -lambda_alpha log(a + eps) for constant
    opacity a; G-ICP term = lambda_n lambda_ng (1 - cos) for a fixed angle; surface term =
    lambda_n lambda_ns 2 |Omega_S| / |Omega_D| for N^ = -rho N_surf."""
    H, W = 9, 24
    rows, cols, d, depth = _sphere_case(H, W)
    n = H * W
    rng = np.random.default_rng(1)
    valid = rng.uniform(size=n) < 0.7
    has_n = valid & (rng.uniform(size=n) < 0.6)
    c, a, rho, ang = 0.25, 0.4, 0.7, 0.6
    td = np.where(valid, depth + np.where(rng.uniform(size=n) < 0.5, c, -c), 0.0)
    op = np.where(valid, a, 0.9)
    Nh = rho * d                                   # = -rho N_surf (N_surf = -d)
    # G-ICP normal at angle `ang` from N^
    perp = np.cross(d, [0.0, 0.0, 1.0])
    perp /= np.linalg.norm(perp, axis=1, keepdims=True)
    tn = np.where(has_n[:, None], math.cos(ang) * d + math.sin(ang) * perp, 0.0)
    w = dict(w_depth=1.5, lambda_alpha=0.1, eps=0.05, lambda_n=2.0, lambda_ng=0.05, lambda_ns=0.01)
    wf = {k: float(np.float32(v)) for k, v in w.items()}
    L, gd, go, gn = ref.objective(rows, cols, dict(depth=depth, opacity=op, normal=Nh), td, tn, w)
    _, ok, _ = ref.surf_normal(rows, cols, depth)
    nD, nN, nS = valid.sum(), has_n.sum(), (valid & ok.astype(bool)).sum()
    assert (L[5], L[6], L[7]) == (nD, nN, nS)
    assert nD != nS and nN != nD
    assert L[1] == pytest.approx(wf["w_depth"] * c, rel=1e-12)
    assert L[2] == pytest.approx(-wf["lambda_alpha"] * math.log(a + wf["eps"]), rel=1e-12)
    assert L[3] == pytest.approx(wf["lambda_n"] * wf["lambda_ng"] * (1 - math.cos(ang)), rel=1e-12)
    assert L[4] == pytest.approx(wf["lambda_n"] * wf["lambda_ns"] * 2.0 * nS / nD, rel=1e-12)
    assert L[0] == pytest.approx(L[1] + L[2] + L[3] + L[4], rel=1e-14)
    # opacity gradient in closed form; nothing outside Omega_D
    np.testing.assert_allclose(go, np.where(valid, -wf["lambda_alpha"] / (nD * (a + wf["eps"])), 0.0), rtol=1e-12)
    assert not gn[~valid].any()


def test_aligned_normals_cost_nothing():
    H, W = 9, 24
    rows, cols, d, depth = _sphere_case(H, W)
    L, *_ = ref.objective(rows, cols, dict(depth=depth, opacity=np.ones(H * W), normal=-0.8 * d), depth, -d,
                          dict(lambda_alpha=0.0))
    assert abs(L[3]) < 1e-14 and abs(L[4]) < 1e-14 and L[1] == 0.0 and L[0] < 1e-14


def test_empty_masks():
    H, W = 5, 8
    rows, cols, d, depth = _sphere_case(H, W)
    L, gd, go, gn = ref.objective(rows, cols, dict(depth=depth, opacity=np.ones(H * W), normal=d),
                                  np.zeros(H * W), np.zeros((H * W, 3)))
    assert not L[:7].any() and not gd.any() and not go.any() and not gn.any()


# ------------------------------------------------------------------------------------------
# gradients: central finite differences of the oracle's own loss
# ------------------------------------------------------------------------------------------

def _realistic(H=14, W=48, seed=4):
    sc = scenegen.make_scene("block", 2, 400)
    rows, cols = scenegen.beam_tables(H, W, -22.5, 5.0)
    pose = scenegen.make_pose(0.7, 3.0, -2.0)
    depth, op, nrm = scenegen.synthetic_frame(sc, pose, rows, cols, seed)
    td, tn = scenegen.targets_for_pose(sc, scenegen.make_pose(0.71, 3.05, -2.0), rows, cols, 0.1, seed)
    return rows, cols, dict(depth=depth.astype(np.float64), opacity=op.astype(np.float64),
                            normal=nrm.astype(np.float64)), td, tn


def test_gradient_matches_finite_differences():
    rows, cols, pred, td, tn = _realistic()
    H, W = rows.shape[0], cols.shape[0]
    w = dict(lambda_ns=0.3, lambda_alpha=0.1)       # a large surface weight: its stencil dominates
    L, gd, go, gn = ref.objective(rows, cols, pred, td, tn, w)
    assert L[7] > 100 and L[4] > 0
    _, ok, fm = ref.surf_normal(rows, cols, pred["depth"])
    rng = np.random.default_rng(0)
    has = np.flatnonzero(pred["depth"].reshape(-1) > 0)
    # rays whose stencil crosses the seam, next to the first / last rows, and random ones
    seam = [k * W + j for k in range(1, H - 1) for j in (0, W - 1)]
    edge = [1 * W + j for j in range(W)] + [(H - 2) * W + j for j in range(W)]
    pick = np.unique(np.concatenate([rng.choice(has, 40, replace=False),
                                     [i for i in seam + edge if i in set(has)][:40]]))

    def total(p):
        return ref.objective(rows, cols, p, td, tn, w, grad=False)[0][0]

    checked = 0
    for i in pick:
        k, j = divmod(int(i), W)
        # stay away from kinks: |D^ - D| = 0 and orientation ties in the stencil
        near = [(k, j), (k, (j + 1) % W), (k, (j - 1) % W), (min(k + 1, H - 1), j), (max(k - 1, 0), j)]
        if min(fm.reshape(H, W)[a, b] for a, b in near) < 1e-3:
            continue
        for key, g, comps in (("depth", gd, [None]), ("opacity", go, [None]), ("normal", gn, [0, 1, 2])):
            for c in comps:
                x = pred[key].reshape(-1, 3)[i, c] if c is not None else pred[key].reshape(-1)[i]
                h = 1e-6 * max(1.0, abs(x))
                pp = {kk: vv.copy() for kk, vv in pred.items()}
                pm = {kk: vv.copy() for kk, vv in pred.items()}
                if c is None:
                    pp[key].reshape(-1)[i] += h
                    pm[key].reshape(-1)[i] -= h
                    ga = g[i]
                else:
                    pp[key].reshape(-1, 3)[i, c] += h
                    pm[key].reshape(-1, 3)[i, c] -= h
                    ga = g[i, c]
                fd = (total(pp) - total(pm)) / (2 * h)
                assert abs(fd - ga) <= 1e-6 * max(abs(fd), 1e-3) + 1e-9, (key, k, j, c, fd, ga)
                checked += 1
    assert checked > 300


# ------------------------------------------------------------------------------------------
# scale regulariser
# ------------------------------------------------------------------------------------------

def test_scale_regulariser_closed_form():
    s = np.array([[2.0, 0.5], [0.3, 0.2], [0.7, 1.6], [1.2, 1.2], [0.9, 1.0]])
    loss, g, _ = ref.scale_reg(np.log(s), lambda_s=10.0, s_max=1.0)
    assert loss == pytest.approx(10.0 * ((2.0 - 1) + (1.6 - 1) + (1.2 - 1)), rel=1e-12)
    want = np.array([[20.0, 0], [0, 0], [0, 16.0], [12.0, 0], [0, 0]])
    np.testing.assert_allclose(g, want, rtol=1e-12)


def test_scale_regulariser_finite_differences():
    rng = np.random.default_rng(5)
    ls = np.log(rng.uniform(0.2, 2.5, size=(200, 2)))
    loss, g, m = ref.scale_reg(ls, lambda_s=10.0, s_max=1.0)
    assert (g != 0).sum() > 50
    for i in range(200):
        if m[i] < 1e-4 or abs(ls[i, 0] - ls[i, 1]) < 1e-4:
            continue
        for c in range(2):
            p, q = ls.copy(), ls.copy()
            p[i, c] += 1e-7
            q[i, c] -= 1e-7
            fd = (ref.scale_reg(p, 10.0, 1.0)[0] - ref.scale_reg(q, 10.0, 1.0)[0]) / 2e-7
            assert abs(fd - g[i, c]) < 1e-5 * max(1.0, abs(fd)), (i, c, fd, g[i, c])
