"""Pins of the oracle's tie outputs against closed forms.

The GPU parity tests drop a ray from value parity when the oracle reports that one of its
threshold decisions lies within 1e-4 relative of the threshold (`margin`) or that two
consecutive contributors' centre ranges are within 2.4e-7 relative (`order_gap`).  A mistake
that inflated or dropped one of these quantities would silently hide rays, or hide a real
disagreement, so each is pinned here on constructed scenes where the deciding quantity
is known in closed form:

* alpha G at a stated relative distance from alpha_thr and from alpha_max (head-on surfel,
  G = 1 on its axis ray);
* q^2 at a stated distance from k^2 = 9 (the hit point from an independent 3x3 solve);
* the transmittance after three composites at a stated distance from T_min;
* |n'.d| at a stated distance from den_eps (normal from scipy's rotation);
* a hit range t and a centre range r at a stated distance from `near`, each on its own,
  both for a surfel that is rendered and for one cut for its centre range;
* surfels rejected by several tests, one of them marginally: only a decision that could
  change which surfels the ray composites counts, so a rejected surfel is as far from
  flipping as the largest gap among the tests that reject it (a surfel the ray crosses at
  t = near but 20 sigma from its centre, or at the 3-sigma edge but too faint there, is no
  tie; a surfel cut for its centre range whose hit tests reject it counts with the larger
  gap);
* three contributors at known relative range gaps (order_gap is the smallest gap between
  consecutive contributors in compositing order);
* den_min, the smallest |n'.d| over a ray's contributors, of a tilted surfel.

Paper: arXiv 2607.04127, Sec. 3.1 (the rendered quantities) and Sec. 3.4 (the outputs
compared); the thresholds are the stabilisers of the rasterizer readings (R4, R11).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenegen
from tests import _util as U

PRM = dict(cutoff_sigma=3.0, alpha_thr=1 / 255, alpha_max=0.99, T_min=1e-4, near=0.2, den_eps=1e-6,
           drop_tau=0.5)
F32 = {k: float(np.float32(v)) for k, v in PRM.items()}  # the thresholds as the oracle receives them
ROWS, COLS = scenegen.beam_tables(32, 256, -15.0, 15.0)
D = scenegen.ray_dirs_f64(ROWS, COLS).reshape(-1, 3)
I0 = 13 * 256 + 40
D0 = D[I0]


@pytest.fixture(scope="module")
def ref(oracle_lib):
    return oracle_lib


def _rel(x, thr):
    return abs(x - thr) / abs(thr)


def _logit(alpha):
    return math.log(alpha) - math.log1p(-alpha)


def _sigmoid(o):
    return 1.0 / (1.0 + math.exp(-o))


def _one(ref, S, ray):
    out = ref.forward(S, U.identity_pose(), ROWS, COLS, PRM, ray_ids=[ray], extra=True)
    return {k: v[0] for k, v in out.items()}


def _head_on(alpha, r=10.0, scale=1.0):
    S = U.surfels([r * D0], [U.frame_facing(-D0, spin=0.3)], [(scale, scale)], [0.5])
    S["opacity_logits"][:] = _logit(alpha)
    return S


@pytest.mark.parametrize("delta", [1e-6, -3e-5, 2e-3])
def test_margin_alpha_threshold(ref, delta):
    """alpha G = alpha on the axis ray; every other decision is at least 0.9 away."""
    S = _head_on(F32["alpha_thr"] * (1 + delta))
    alpha = _sigmoid(float(S["opacity_logits"][0]))
    o = _one(ref, S, I0)
    assert o["margin"] == pytest.approx(_rel(alpha, F32["alpha_thr"]), rel=1e-6)
    assert o["K"] == (1 if delta > 0 else 0)


@pytest.mark.parametrize("delta", [2e-5, -7e-6])
def test_margin_alpha_max(ref, delta):
    S = _head_on(F32["alpha_max"] * (1 + delta))
    alpha = _sigmoid(float(S["opacity_logits"][0]))
    o = _one(ref, S, I0)
    assert o["margin"] == pytest.approx(_rel(alpha, F32["alpha_max"]), rel=1e-6)
    assert o["opacity"] == pytest.approx(min(alpha, F32["alpha_max"]), rel=1e-14)


def _q2_on_ray(mu, frame, scales, d):
    """(t, q2) of ray d against the surfel's plane by an independent 3x3 solve
    d t - a (s0 u) - b (s1 v) = mu."""
    a, b = frame[:, 0], frame[:, 1]
    t, su, sv = np.linalg.solve(np.stack([d, -a, -b], axis=1), mu)
    return t, (su / scales[0]) ** 2 + (sv / scales[1]) ** 2


@pytest.mark.parametrize("delta", [4e-6, -1e-5])
def test_margin_support_cutoff(ref, delta):
    """A neighbouring ray meets the head-on surfel at q^2 = 9 (1 + delta)."""
    ray = I0 + 2
    F = U.frame_facing(-D0, spin=0.3)
    _, q2_unit = _q2_on_ray(10 * D0, F, (1.0, 1.0), D[ray])
    s = math.sqrt(q2_unit / (9 * (1 + delta)))
    S = U.surfels([10 * D0], [F], [(s, s)], [0.9])
    frame = U.rot_of_wxyz(S["quats"][0])
    sr = np.exp(S["log_scales"][0])
    _, q2 = _q2_on_ray(S["means"][0], frame, sr, D[ray])
    o = _one(ref, S, ray)
    assert o["margin"] == pytest.approx(_rel(q2, 9.0), rel=1e-6)
    assert o["K"] == (0 if delta > 0 else 1)


@pytest.mark.parametrize("delta", [3e-5, -2e-6])
def test_margin_transmittance(ref, delta):
    """Three identical head-on surfels with (1 - alpha)^3 = T_min (1 + delta): the third
    composite decides termination; every other decision is at least 0.03 away."""
    a = 1 - (F32["T_min"] * (1 + delta)) ** (1 / 3)
    F = U.frame_facing(-D0)
    S = U.surfels([(10.0 + k) * D0 for k in range(3)], [F] * 3, [(1.0, 1.0)] * 3, [a] * 3)
    alpha = _sigmoid(float(S["opacity_logits"][0]))
    o = _one(ref, S, I0)
    assert o["K"] == 3
    assert o["t_final"] == pytest.approx((1 - alpha) ** 3, rel=1e-12)
    assert o["margin"] == pytest.approx(_rel((1 - alpha) ** 3, F32["T_min"]), rel=1e-6)


def test_margin_denominator(ref):
    """A surfel whose normal makes |n'.d| = 1.2e-6 with the ray through its centre: hit at
    its centre (t = r, q^2 = 0), alpha 0.5, so the den_eps decision (gap 0.2) is the
    closest."""
    h = np.cross(D0, [0.0, 0.0, 1.0])
    h /= np.linalg.norm(h)
    c = 1.2e-6
    nrm = -c * D0 + math.sqrt(1 - c * c) * h
    S = U.surfels([10 * D0], [U.frame_facing(nrm, spin=0.2)], [(1.0, 1.0)], [0.5])
    n_real = U.rot_of_wxyz(S["quats"][0])[:, 2]
    den = abs(float(n_real @ D0))
    o = _one(ref, S, I0)
    assert 0.1 < _rel(den, F32["den_eps"]) < 0.3
    assert o["margin"] == pytest.approx(_rel(den, F32["den_eps"]), rel=1e-6)
    assert o["den_min"] == pytest.approx(den, rel=1e-6)


def _plane_through(mu, p1, scale_factor=0.5):
    """Surfel centred at mu whose plane contains p1, normal facing the sensor, isotropic
    scale |p1 - mu| * scale_factor (so p1 sits at q^2 = 1 / scale_factor^2)."""
    e = p1 - mu
    n = -mu / np.linalg.norm(mu)
    n = n - e * (n @ e) / (e @ e)
    s = np.linalg.norm(e) * scale_factor
    return U.surfels([mu], [U.frame_facing(n, spin=0.1)], [(s, s)], [0.9])


@pytest.mark.parametrize("delta", [5e-6, -5e-6])
def test_margin_hit_near(ref, delta):
    """Centre 0.3 m away on the axis ray, plane met by a ray ten columns over at
    t = 0.2 (1 + delta): the per-hit near decision is the closest (q^2 = 4)."""
    ray = I0 + 10
    S = _plane_through(0.3 * D0, F32["near"] * (1 + delta) * D[ray])
    frame = U.rot_of_wxyz(S["quats"][0])
    t, q2 = _q2_on_ray(S["means"][0], frame, np.exp(S["log_scales"][0]), D[ray])
    assert q2 == pytest.approx(4.0, rel=1e-9)
    o = _one(ref, S, ray)
    assert o["margin"] == pytest.approx(_rel(t, F32["near"]), rel=1e-6)
    assert o["K"] == (1 if delta > 0 else 0)


@pytest.mark.parametrize("delta", [1e-6, 1e-3, -1e-6, -1e-3])
def test_margin_centre_near(ref, delta):
    """Centre at 0.2 (1 + delta) on the axis ray, plane met by a ray ten columns over at
    t = 0.3 with q^2 = 4: the centre-range cut is the closest decision on that ray, both
    when the surfel is rendered (delta > 0) and when it is cut (delta < 0)."""
    ray = I0 + 10
    S = _plane_through(F32["near"] * (1 + delta) * D0, 0.3 * D[ray])
    r = float(np.linalg.norm(S["means"][0]))
    o = _one(ref, S, ray)
    assert o["K"] == (1 if delta > 0 else 0)
    assert o["margin"] == pytest.approx(_rel(r, F32["near"]), rel=1e-6)


@pytest.mark.parametrize("delta", [4e-6, -4e-6])
def test_margin_rejected_surfel_takes_largest_gap(ref, delta):
    """A neighbouring ray meets a head-on surfel of opacity 0.2 at q^2 = 9 (1 + delta): at the
    3-sigma edge alpha G is about 0.0022, well under alpha_thr, so the surfel is rejected on
    either side of the support threshold and the margin is the opacity test's gap (0.43)."""
    ray = I0 + 2
    F = U.frame_facing(-D0, spin=0.3)
    _, q2_unit = _q2_on_ray(10 * D0, F, (1.0, 1.0), D[ray])
    s = math.sqrt(q2_unit / (9 * (1 + delta)))
    S = U.surfels([10 * D0], [F], [(s, s)], [0.2])
    frame = U.rot_of_wxyz(S["quats"][0])
    _, q2 = _q2_on_ray(S["means"][0], frame, np.exp(S["log_scales"][0]), D[ray])
    assert _rel(q2, 9.0) < 1e-5
    aG = _sigmoid(float(S["opacity_logits"][0])) * math.exp(-0.5 * q2)
    o = _one(ref, S, ray)
    assert o["K"] == 0
    assert o["margin"] == pytest.approx(_rel(aG, F32["alpha_thr"]), rel=1e-6)
    assert o["margin"] > 0.4


@pytest.mark.parametrize("delta", [1e-6, -1e-6])
def test_margin_far_surfel_crossed_near_the_sensor(ref, delta):
    """A surfel 3 m out whose plane a ray ten columns over crosses at t = 0.2 (1 + delta),
    20 sigma from its centre (q^2 = 400): the support test rejects it by a wide margin, so
    the hit-range decision next to `near` does not count and the margin is the largest gap
    of the rejecting tests, that of q^2 against 9."""
    ray = I0 + 10
    S = _plane_through(3.0 * D0, F32["near"] * (1 + delta) * D[ray], scale_factor=0.05)
    frame = U.rot_of_wxyz(S["quats"][0])
    t, q2 = _q2_on_ray(S["means"][0], frame, np.exp(S["log_scales"][0]), D[ray])
    assert _rel(t, F32["near"]) < 2e-6 and q2 == pytest.approx(400.0, rel=1e-9)
    o = _one(ref, S, ray)
    assert o["K"] == 0
    assert o["margin"] == pytest.approx(_rel(q2, 9.0), rel=1e-6)


def test_margin_cut_surfel_rejected_by_its_hit_tests(ref):
    """A surfel with its centre at 0.1 m (cut: 0.5 from `near`) whose plane a ray meets at
    q^2 = 4 with alpha G 1e-5 under alpha_thr: to render it both decisions would have to
    flip, so the margin is the larger gap, the centre range's."""
    ray = I0 + 10
    S = _plane_through(0.1 * D0, 0.3 * D[ray])
    S["opacity_logits"][:] = _logit(F32["alpha_thr"] * (1 - 1e-5) * math.exp(2.0))
    r = float(np.linalg.norm(S["means"][0]))
    o = _one(ref, S, ray)
    assert o["K"] == 0
    assert o["margin"] == pytest.approx(_rel(r, F32["near"]), rel=1e-6)


def test_order_gap(ref):
    """Three parallel surfels on the axis ray at ranges 10, 10 (1 + 3e-6) and
    10 (1 + 3e-6)(1 + 8e-7), listed far to near: order_gap is the smaller gap between
    neighbours in range order, not the gap to the first contributor or in index order."""
    r1 = 10.0
    r2 = r1 * (1 + 3e-6)
    r3 = r2 * (1 + 8e-7)
    F = U.frame_facing(-D0)
    S = U.surfels([r3 * D0, r1 * D0, r2 * D0], [F] * 3, [(1.0, 1.0)] * 3, [0.3] * 3)
    rr = np.linalg.norm(S["means"], axis=1)
    srt = np.sort(rr)
    expect = min((srt[1] - srt[0]) / srt[0], (srt[2] - srt[1]) / srt[1])
    o = _one(ref, S, I0)
    assert o["K"] == 3
    assert o["order_gap"] == pytest.approx(expect, rel=1e-6)
    assert o["order_gap"] == pytest.approx(8e-7, rel=1e-3)
    # a single contributor has no gap
    o1 = _one(ref, {k: v[1:2] for k, v in S.items()}, I0)
    assert o1["K"] == 1 and o1["order_gap"] == math.inf


def test_den_min_of_a_tilted_surfel(ref):
    """Normal 70 degrees from the view direction: |n'.d| on the axis ray is cos 70 degrees
    for the rotation scipy builds from the same quaternion; a head-on surfel gives 1."""
    h = np.cross(D0, [0.0, 0.0, 1.0])
    h /= np.linalg.norm(h)
    th = math.radians(70.0)
    nrm = -math.cos(th) * D0 + math.sin(th) * h
    S = U.surfels([10 * D0], [U.frame_facing(nrm)], [(1.0, 1.0)], [0.6])
    n_real = Rotation.from_quat(np.r_[S["quats"][0][1:], S["quats"][0][0]]).as_matrix()[:, 2]
    o = _one(ref, S, I0)
    assert o["K"] == 1
    assert o["den_min"] == pytest.approx(abs(n_real @ D0), rel=1e-12)
    assert o["den_min"] == pytest.approx(math.cos(th), rel=1e-6)  # the tables are unit to float32 rounding
    assert _one(ref, _head_on(0.6), I0)["den_min"] == pytest.approx(float(np.linalg.norm(D0)), rel=1e-12)


def test_order_and_contributors(ref):
    """lgsr_ref_order lists the rendering surfels by ascending centre range with equal
    ranges by index (ranges from numpy, duplicates planted); lgsr_ref_contributors gives each
    ray's composited surfels front to back, as many as the forward's hit count."""
    w = scenegen.make_workload("room32x256_1k")
    S = {k: np.concatenate([w[k], w[k][:50]]) for k in ("means", "quats", "log_scales", "opacity_logits")}
    P = np.asarray(w["pose"], np.float64)
    r = np.linalg.norm((np.asarray(S["means"], np.float64) - P[:, 3]) @ P[:, :3], axis=1)
    keep = r >= F32["near"]
    want = np.lexsort((np.arange(len(r)), r))
    want = want[keep[want]]
    o, rr = ref.order(S, P)
    np.testing.assert_array_equal(o, want)
    np.testing.assert_allclose(rr, r[want], rtol=1e-14)
    ids = np.arange(0, 8192, 37)
    c = ref.contributors(S, P, w["row_sincos"], w["col_sincos"], ids)
    f = ref.forward(S, P, w["row_sincos"], w["col_sincos"], ray_ids=ids)
    assert [len(x) for x in c] == list(f["K"])
    pos = np.empty(len(r), np.int64)
    pos[o] = np.arange(len(o))
    assert all(np.all(np.diff(pos[x]) > 0) for x in c)
    # two stacked surfels, far one first in index order: near then far
    F = U.frame_facing(-D0)
    S2 = U.surfels([9.5 * D0, 8.0 * D0], [F, F], [(1.0, 1.0)] * 2, [0.8, 0.6])
    assert list(ref.contributors(S2, U.identity_pose(), ROWS, COLS, [I0])[0]) == [1, 0]
