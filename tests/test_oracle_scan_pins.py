"""Pins of the oracle's scan projection (Sec. 3.1: a scan becomes a spherical range image on
the grid the map is rendered on) and surfel target covariance (Sec. 3.2): points placed on
beam directions land on their own pixel (row 0 on top, azimuth wrapping over the full
turn), jitter below half a bin keeps them there, the nearest return wins whatever the order,
the field-of-view and range gates, normals turned to face the sensor, a raycast range image
survives the trip to points and back; covariances have the surfel's axes as eigenvectors
with the squared scales and thickness as eigenvalues (axes from scipy's rotation)."""
import math

import numpy as np
import pytest

import scenegen
from oracle import ref

EL = (math.radians(-25.0), math.radians(15.0))


def _dir(el, az):
    return np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], -1)


def _grid(H, W, el=EL):
    step = (el[1] - el[0]) / (H - 1)
    els = el[1] - np.arange(H) * step
    azs = 2 * np.pi * np.arange(W) / W
    return els, azs, step, 2 * np.pi / W


def test_points_on_beam_directions_land_on_their_pixel():
    H, W = 16, 90
    els, azs, _, _ = _grid(H, W)
    rng = np.random.default_rng(0)
    K, J = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    K, J = K.reshape(-1), J.reshape(-1)
    r = rng.uniform(1.0, 50.0, K.size)
    pts = r[:, None] * _dir(els[K], azs[J])
    perm = rng.permutation(K.size)
    out = ref.scan_to_range(pts[perm], H, W, *EL)
    np.testing.assert_array_equal(out["index"], np.argsort(perm))  # pixel k*W+j holds the point made for it
    np.testing.assert_allclose(out["depth"], r, rtol=1e-12)


def test_jitter_below_half_a_bin_keeps_the_pixel():
    H, W = 12, 64
    els, azs, de, da = _grid(H, W)
    rng = np.random.default_rng(1)
    K = rng.integers(0, H, 4000)
    J = rng.integers(0, W, 4000)
    # the seam: azimuths just below 2 pi belong to column 0, just above 0 too
    J[:200] = 0
    el = els[K] + rng.uniform(-0.45, 0.45, K.size) * de
    az = azs[J] + rng.uniform(-0.45, 0.45, J.size) * da
    pts = rng.uniform(2.0, 30.0, K.size)[:, None] * _dir(el, az)
    out = ref.scan_to_range(pts, H, W, *EL)
    hit = np.zeros(H * W, bool)
    hit[K * W + J] = True
    assert (out["index"] >= 0).sum() == hit.sum() and (out["index"][hit] >= 0).all()
    assert ((K * W + J)[out["index"][hit]] == np.flatnonzero(hit)).all()


def test_nearest_return_wins_in_any_order():
    H, W = 6, 20
    els, azs, de, da = _grid(H, W)
    rng = np.random.default_rng(2)
    n = 3000
    K, J = rng.integers(0, H, n), rng.integers(0, W, n)
    dirs = _dir(els[K] + rng.uniform(-0.4, 0.4, n) * de, azs[J] + rng.uniform(-0.4, 0.4, n) * da)
    r = rng.uniform(1.0, 40.0, n)
    r[1::7] = r[0:-1:7]  # repeated ranges in other pixels are harmless
    pts = r[:, None] * dirs
    a = ref.scan_to_range(pts, H, W, *EL)
    for seed in range(3):
        perm = np.random.default_rng(seed).permutation(n)
        b = ref.scan_to_range(pts[perm], H, W, *EL)
        np.testing.assert_array_equal(a["depth"], b["depth"])
        np.testing.assert_array_equal(a["index"], perm[b["index"]])
    pix = K * W + J
    for q in np.unique(pix):
        assert a["depth"][q] == pytest.approx(r[pix == q].min(), rel=1e-14)
        assert r[a["index"][q]] == r[pix == q].min()
    # exact range ties inside one pixel: the lower index
    pts2 = np.concatenate([pts, pts[:50]])
    c = ref.scan_to_range(pts2, H, W, *EL)
    np.testing.assert_array_equal(c["index"], a["index"])


def test_field_of_view_and_range_gates():
    H, W = 5, 8
    els, azs, de, _ = _grid(H, W)
    P = np.array([_dir(els[0] + 0.49 * de, 0.0) * 5,    # just inside the top row
                  _dir(els[0] + 0.51 * de, 0.3) * 5,    # above the field of view
                  _dir(els[-1] - 0.51 * de, 0.8) * 5,   # below it
                  _dir(els[2], 1.6) * 0.5,              # nearer than r_min
                  _dir(els[2], 2.4) * 1.000001,         # just beyond r_min: kept
                  _dir(els[3], 3.2) * 80.0])            # beyond r_max
    out = ref.scan_to_range(P, H, W, *EL, r_min=1.0, r_max=60.0)
    assert sorted(out["index"][out["index"] >= 0].tolist()) == [0, 4]


def test_normals_turned_to_face_the_sensor():
    H, W = 8, 32
    els, azs, _, _ = _grid(H, W)
    rng = np.random.default_rng(4)
    K, J = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    d = _dir(els[K.reshape(-1)], azs[J.reshape(-1)])
    pts = rng.uniform(2, 20, (H * W, 1)) * d
    nrm = rng.normal(size=(H * W, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    out = ref.scan_to_range(pts, H, W, *EL, normals=nrm)
    assert (np.einsum("ij,ij->i", out["normal"], d) <= 0).all()
    np.testing.assert_allclose(np.abs(out["normal"]), np.abs(nrm), rtol=0, atol=0)
    flipped = np.einsum("ij,ij->i", nrm, d) > 0
    np.testing.assert_array_equal(out["normal"][flipped], -nrm[flipped])


def test_raycast_image_survives_points_and_back():
    """Range image of the street-block scene -> points along the (float32-table) beams ->
    range image again: the same returns, ranges to the tables' rounding."""
    H, W = 32, 512
    rows, cols = scenegen.beam_tables(H, W, -25.0, 15.0)
    sc = scenegen.make_scene("block", 3, 400)
    depth, _ = scenegen.targets_for_pose(sc, scenegen.make_pose(0.4, 2.0, 1.0), rows, cols)
    d = scenegen.ray_dirs_f64(rows, cols).reshape(-1, 3)
    D = depth.reshape(-1).astype(np.float64)
    has = np.flatnonzero(D > 0)
    out = ref.scan_to_range(D[has, None] * d[has], H, W, math.radians(-25.0), math.radians(15.0))
    assert (out["index"] >= 0).sum() == has.size
    np.testing.assert_array_equal(has[out["index"][has]], has)
    np.testing.assert_allclose(out["depth"][has], D[has], rtol=1e-6)


def test_target_covariance_eigenstructure():
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(7)
    n = 500
    q = rng.normal(size=(n, 4)) * rng.uniform(0.3, 3.0, (n, 1))  # (w, x, y, z), any norm and sign
    ls = np.log(rng.uniform(0.01, 2.0, (n, 2)))
    eps = 0.01
    cov = ref.target_cov(q, ls, eps)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    s = np.exp(ls)
    epsf = float(np.float32(eps))
    for i in range(n):
        S = np.array([[cov[i, 0], cov[i, 1], cov[i, 2]], [cov[i, 1], cov[i, 3], cov[i, 4]],
                      [cov[i, 2], cov[i, 4], cov[i, 5]]])
        a, b, nn = R[i][:, 0], R[i][:, 1], R[i][:, 2]
        tol = 1e-12 * max(s[i].max() ** 2, 1.0)
        np.testing.assert_allclose(S @ a, s[i, 0] ** 2 * a, atol=tol)
        np.testing.assert_allclose(S @ b, s[i, 1] ** 2 * b, atol=tol)
        np.testing.assert_allclose(S @ nn, epsf ** 2 * nn, atol=tol)
    np.testing.assert_allclose(ref.target_cov(-2.5 * q, ls, eps), cov, rtol=1e-12, atol=1e-15)
    ident = ref.target_cov(np.array([[1.0, 0, 0, 0]]), np.log([[2.0, 0.5]]), 0.1)
    np.testing.assert_allclose(ident, [[4.0, 0, 0, 0.25, 0, float(np.float32(0.1)) ** 2]], rtol=1e-12)
