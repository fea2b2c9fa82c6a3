"""Seeded input generator: determinism, exact analytic raycasts, beam-table conventions and
the ray-drop rate of the spinning-LiDAR workloads."""
import math

import numpy as np

import scenegen
from scenegen.scene import GROUND_Z, Scene


def test_deterministic_per_seed():
    a = scenegen.make_workload("room32x256_1k")
    b = scenegen.make_workload("room32x256_1k")
    for k in ("means", "quats", "log_scales", "opacity_logits", "pose", "target_depth", "target_normal"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["means"].dtype == np.float32 and a["means"].shape == (1000, 3)


def test_raycast_matches_analytic_planes():
    scene = Scene(walls=np.array([(0, 20.0, -50.0, 50.0, 5.0)]), boxes=np.zeros((0, 6)),
                  extent=(-50, 20, -50, 50))
    el = np.radians([-10.0, -3.0, 2.0])
    d = np.stack([np.cos(el), np.zeros(3), np.sin(el)], 1)
    t, n = scenegen.raycast(scene, np.zeros((1, 3)), d)
    # ground at -1.7 for the steep ray, wall x = 20 for the others
    t_ground = -GROUND_Z / math.sin(-el[0])
    t_wall = 20.0 / np.cos(el)
    exp = np.where(t_ground < t_wall, [t_ground] * 3, t_wall)
    exp[1:] = np.minimum(t_wall[1:], np.where(np.sin(el[1:]) < 0, -GROUND_Z / -np.sin(el[1:]), np.inf))
    np.testing.assert_allclose(t, exp, rtol=1e-14)
    assert np.all(np.einsum("ij,ij->i", n, d) < 0)  # normals face the sensor


def test_beam_tables():
    row, col = scenegen.beam_tables(64, 1024, -22.5, 22.5)
    assert row.dtype == np.float32 and row.shape == (64, 2) and col.shape == (1024, 2)
    assert row[0, 0] > 0 > row[-1, 0]  # row 0 is the top beam
    assert abs(math.degrees(math.asin(row[0, 0])) - 22.5) < 1e-5
    q = 256
    np.testing.assert_array_equal(col[q:2 * q, 0], col[0:q, 1])  # sin(th + pi/2) = cos th
    np.testing.assert_array_equal(col[q:2 * q, 1], -col[0:q, 0])
    assert col[0, 0] == 0 and col[0, 1] == 1


def test_drop_rate_and_target_conventions():
    w = scenegen.make_workload("block64x1024_300k", n=2000)
    hit = scenegen.make_workload("block64x1024_300k", n=2000)  # same seeds: same targets
    np.testing.assert_array_equal(w["target_depth"], hit["target_depth"])
    # rays that the scene returns (without drop) vs what survives the 10% Bernoulli drop
    nodrop, _ = scenegen.targets_for_pose(w["scene"], w["pose"], w["row_sincos"], w["col_sincos"])
    returned = nodrop > 0
    kept = (w["target_depth"] > 0)[returned].mean()
    n = returned.sum()
    assert abs((1 - kept) - 0.1) < 3 * math.sqrt(0.1 * 0.9 / n)
    nn = np.linalg.norm(w["target_normal"], axis=-1)
    np.testing.assert_allclose(nn[w["target_depth"] > 0], 1.0, atol=1e-6)
    assert np.all(nn[w["target_depth"] == 0] == 0)


def test_surfel_scales_follow_range():
    w = scenegen.make_workload("room32x256_1k")
    r = np.linalg.norm(w["means"].astype(np.float64), axis=1)  # sampled from the origin
    s = np.exp(w["log_scales"].astype(np.float64))
    ratio = s / (r[:, None] * w["delta"])
    assert ratio.min() >= 0.8 - 1e-6 and ratio.max() <= 1.5 + 1e-6
    assert np.all(s[:, 0] >= s[:, 1])  # first tangent axis is the major one
    qn = np.linalg.norm(w["quats"], axis=1)
    assert qn.min() > 0.79 and qn.max() < 1.26  # stored unnormalised on purpose
