"""GPU parity of the scan-to-range-image projection (lgsr_scan_to_range) and the surfel
target covariances (lgsr_target_cov) against the FP64 oracle.

Scan: the winning point index per pixel is compared bit for bit.  Both sides take the
bin decisions in their own precision, so points that lie within 1e-4 of a bin boundary (in
bins, or relative to the range gates) may land differently: pixels they reach are left out
of the exact comparison, and so are pixels whose two nearest candidates are closer in range
than float32 separates (2e-7 relative).  Ranges agree to 1e-6 relative (float32 rounding of
the norm); normals are the winner's, with the facing decision taken away from ties.
Covariance: elementwise within 1e-5 of the largest eigenvalue of that surfel."""
import math

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


def _ambiguous(pts, out, H, W, el_min, el_max):
    """Pixels whose winner may differ between float32 and float64 bin or range decisions."""
    P = pts.astype(np.float64)
    r = np.linalg.norm(P, axis=1)
    el = np.arctan2(P[:, 2], np.hypot(P[:, 0], P[:, 1]))
    az = np.arctan2(P[:, 1], P[:, 0])
    f = (np.float32(el_max) - el) * (H - 1) / (float(np.float32(el_max)) - float(np.float32(el_min)))
    g = az * W / (2 * np.pi)
    near = out["bin_margin"] < 1e-4
    bad = np.zeros(H * W, bool)
    # every pixel an ambiguous point could reach (its rounded cell and the one across the boundary)
    for i in np.flatnonzero(near):
        for kk in {int(np.floor(f[i])), int(np.floor(f[i]) + 1)}:
            for jj in {int(np.floor(g[i])), int(np.floor(g[i]) + 1)}:
                if 0 <= kk < H:
                    bad[kk * W + jj % W] = True
    # near-equal ranges competing for one pixel
    k = np.floor(f + 0.5).astype(np.int64)
    j = np.floor(g + 0.5).astype(np.int64) % W
    ok = (k >= 0) & (k < H)
    pix = k[ok] * W + j[ok]
    rr = r[ok]
    order = np.lexsort((rr, pix))
    ps, rs = pix[order], rr[order]
    same = ps[1:] == ps[:-1]
    first = np.concatenate([[True], ~same])
    gap = np.abs(rs[1:] - rs[:-1])
    close = same & first[:-1] & (gap > 0) & (gap <= 2e-7 * rs[:-1])  # exact ties: both take the lower index
    bad[ps[1:][close]] = True
    return bad


def _scan_case(ctx, pts, nrm, H, W, el_deg, r_min=0.0, r_max=float("inf"), tag=""):
    from paper_2607_04127_amd import lgsr
    el_min, el_max = math.radians(el_deg[0]), math.radians(el_deg[1])
    o = ref.scan_to_range(pts, H, W, el_min, el_max, r_min, r_max, normals=nrm)
    dev = torch.device("cuda", 0)
    g = lgsr.lgsr_scan_to_range(ctx, torch.from_numpy(pts).to(dev), H, W, el_min, el_max, r_min, r_max,
                                normals=None if nrm is None else torch.from_numpy(nrm).to(dev))
    torch.cuda.synchronize()
    idx = g["index"].cpu().numpy().reshape(-1).astype(np.int64)
    dep = g["depth"].cpu().numpy().reshape(-1)
    nr = g["normal"].cpu().numpy().reshape(-1, 3)
    bad = _ambiguous(pts, o, H, W, el_min, el_max) if pts.shape[0] else np.zeros(H * W, bool)
    keep = ~bad
    assert np.array_equal(idx[keep], o["index"][keep]), (tag, int((idx[keep] != o["index"][keep]).sum()))
    np.testing.assert_allclose(dep[keep], o["depth"][keep], rtol=1e-6, atol=0)
    assert ((idx >= 0) | (dep == 0)).all() and (nr[idx < 0] == 0).all()
    if nrm is not None:
        hit = keep & (idx >= 0)
        p = pts[idx[hit]].astype(np.float64)
        facing = np.abs(np.einsum("ij,ij->i", nrm[idx[hit]].astype(np.float64), p)) / np.linalg.norm(p, axis=1)
        sure = facing > 1e-5
        np.testing.assert_array_equal(nr[hit][sure], o["normal"][hit][sure].astype(np.float32))
    else:
        assert not nr.any()
    # ambiguous pixels still hold a valid outcome: empty, or a point that could land there
    for q in np.flatnonzero(bad & (idx >= 0)):
        assert 0 <= idx[q] < pts.shape[0]
    print(f"\n[scan {tag} {H}x{W}] points={pts.shape[0]} returns={int((idx >= 0).sum())} "
          f"excluded={int(bad.sum())}", flush=True)
    return idx, o


@pytest.mark.parametrize("H,W,el", [(64, 1024, (-22.5, 22.5)), (128, 2048, (-45.0, 45.0)), (32, 1024, (-22.5, 22.5)),
                                    (16, 90, (-15.0, 15.0))])
def test_scan_matches_oracle(ctx, H, W, el):
    sc = scenegen.make_scene("block", 4, 400)
    rng = np.random.default_rng(H + W)
    pose = scenegen.make_pose(rng.uniform(0, 6.28), *rng.uniform(-5, 5, 2))
    pts, nrm = scenegen.synthetic_scan(sc, pose, H, W, el[0], el[1], seed=H * W)
    idx, o = _scan_case(ctx, pts, nrm, H, W, el, r_min=0.5, r_max=80.0, tag="street block")
    assert (idx >= 0).sum() > 0.3 * H * W


def test_scan_random_points_gates_and_ties(ctx):
    """Points anywhere (many outside the rows, some beyond the range gates), exact duplicates
    (equal ranges in one pixel: the lower index wins), no normals."""
    rng = np.random.default_rng(5)
    n = 200_000
    v = rng.normal(size=(n, 3))
    pts = (v / np.linalg.norm(v, axis=1, keepdims=True) * rng.uniform(0.1, 120.0, (n, 1))).astype(np.float32)
    pts = np.concatenate([pts, pts[:20_000]])
    _scan_case(ctx, pts, None, 24, 360, (-10.0, 10.0), r_min=1.0, r_max=100.0, tag="random")


@pytest.mark.parametrize("n,H,W", [(0, 8, 16), (5, 2, 1), (1000, 3, 7)])
def test_scan_edge_shapes(ctx, n, H, W):
    rng = np.random.default_rng(n + H)
    v = rng.normal(size=(n, 3))
    pts = (v / np.maximum(np.linalg.norm(v, axis=1, keepdims=True), 1e-9) * rng.uniform(1, 10, (n, 1)))
    pts = pts.astype(np.float32).reshape(n, 3)
    nrm = rng.normal(size=(n, 3)).astype(np.float32).reshape(n, 3)
    idx, _ = _scan_case(ctx, pts, nrm, H, W, (-60.0, 60.0), tag="edge")
    if n == 0:
        assert (idx == -1).all()


def test_scan_rejects_bad_grids(ctx):
    from paper_2607_04127_amd import lgsr
    p = torch.zeros((4, 3), device="cuda:0")
    for H, W, a, b in [(1, 8, -0.1, 0.1), (8, 0, -0.1, 0.1), (8, 8, 0.1, 0.1), (8, 8, 0.2, -0.1)]:
        with pytest.raises(lgsr.LgsrError):
            lgsr.lgsr_scan_to_range(ctx, p, H, W, a, b, out=dict(
                depth=torch.empty((H, W), device="cuda:0"), normal=torch.empty((H, W, 3), device="cuda:0"),
                index=torch.empty((H, W), device="cuda:0", dtype=torch.int32)))


@pytest.mark.parametrize("n", [300_000, 1, 0, 1000])
def test_target_covariance_matches_oracle(ctx, n):
    from paper_2607_04127_amd import lgsr
    if n == 300_000:
        w = scenegen.make_workload("block64x1024_300k", with_targets=False)
        q, ls = w["quats"].copy(), w["log_scales"]
    else:
        rng = np.random.default_rng(n)
        q = rng.normal(size=(n, 4)).astype(np.float32)
        ls = np.log(rng.uniform(0.01, 3.0, (n, 2))).astype(np.float32)
    if n >= 10:
        q[3] = 0.0  # no orientation: zero covariance
    want = ref.target_cov(q, ls, 0.01)
    dev = torch.device("cuda", 0)
    got = lgsr.lgsr_target_cov(ctx, torch.from_numpy(np.ascontiguousarray(q)).to(dev),
                               torch.from_numpy(np.ascontiguousarray(ls)).to(dev), 0.01)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    lam = np.maximum(np.exp(2 * ls.astype(np.float64)).max(axis=1), float(np.float32(0.01)) ** 2) if n else np.zeros(0)
    assert (np.abs(got - want) <= 1e-5 * lam[:, None] + 1e-30).all()
    if n >= 10:
        assert not got[3].any()
