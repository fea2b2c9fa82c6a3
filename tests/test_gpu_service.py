"""GPU tests of the batched render path (lgsr_render_batch) and the rendering service: a
batch mixing maps, poses, resolutions and render / render + gradient requests gives the
same frames and losses as one call per request (bit for bit) and the same gradients up to
float32 summation order; batches reuse their internal states correctly; the service loop
serves every request of a Poisson stream."""
import numpy as np
import pytest

import scenegen
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


def _requests(seed):
    room = scenegen.make_workload("room32x256_1k")
    block = scenegen.make_workload("block64x1024_300k", n=60_000)
    maps = [{k: torch.from_numpy(np.ascontiguousarray(w[k])).cuda() for k in G.SURF_KEYS} for w in (room, block)]
    beams = [(32, 256, -15, 15), (37, 250, -15, 15), (64, 1024, -22.5, 22.5), (16, 512, -10, 10)]
    tables = [tuple(torch.from_numpy(t).cuda() for t in scenegen.beam_tables(*b)) for b in beams]
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(9):
        mi = k % 2
        bi = int(rng.integers(len(beams)))
        w = (room, block)[mi]
        T = np.asarray(w["pose"], np.float64).copy()
        T[:, 3] += rng.normal(scale=0.3, size=3)
        q = dict(surfels=maps[mi], pose=T.astype(np.float32), row_sincos=tables[bi][0], col_sincos=tables[bi][1])
        if k % 3 == 0:
            H, W = beams[bi][0], beams[bi][1]
            q["target_depth"] = torch.from_numpy(rng.uniform(2, 30, (H, W)).astype(np.float32)).cuda()
            nrm = rng.normal(size=(H, W, 3))
            q["target_normal"] = torch.from_numpy((nrm / np.linalg.norm(nrm, axis=2, keepdims=True))
                                                  .astype(np.float32)).cuda()
        reqs.append(q)
    return reqs


def _close(a, b, what):
    a, b = a.detach().cpu().numpy().astype(np.float64), b.detach().cpu().numpy().astype(np.float64)
    scale = np.abs(b).max() if b.size else 0.0
    assert np.abs(a - b).max(initial=0.0) <= 1e-5 * scale + 1e-30, what


def test_batch_matches_single_calls(ctx):
    from paper_2607_04127_amd import lgsr
    reqs = _requests(3)
    for rep in range(2):  # the second batch reuses the internal per-request states
        res = lgsr.lgsr_render_batch(ctx, reqs)
        torch.cuda.synchronize()
        for k, (q, r) in enumerate(zip(reqs, res)):
            fr, st = lgsr.lgsr_forward(ctx, q["surfels"], torch.from_numpy(np.asarray(q["pose"])), q["row_sincos"],
                                       q["col_sincos"])
            for key in ("depth", "opacity", "normal", "drop"):
                assert torch.equal(r["frame"][key], fr[key]), (rep, k, key)
            if "target_depth" in q:
                L, g = lgsr.lgsr_loss(ctx, fr, q["target_depth"], q["target_normal"])
                out, gp = lgsr.lgsr_backward(ctx, st, g)
                torch.cuda.synchronize()
                assert torch.equal(r["loss"], L), (rep, k)
                for key in G.SURF_KEYS:
                    _close(r["grads"][key], out[key], (rep, k, key))
                _close(r["grad_pose"], gp, (rep, k, "pose"))
            st.free()


def test_service_serves_a_poisson_stream(ctx):
    """Two small maps, 60 requests at a modest rate, batched and one-by-one: every request is
    served exactly once and the latency statistics are well formed."""
    from paper_2607_04127_amd import service as SV
    maps = SV.make_maps([2_000, 20_000], seed=41)
    pool = SV.make_pool(maps, [(32, 1024, -22.5, 22.5), (64, 1024, -22.5, 22.5)], poses_per=2, seed=45)
    stream = SV.poisson_stream(pool, n=60, rate=2000.0, grad_fraction=0.3, seed=45)
    for mode in ("batched", "single"):
        svc = SV.Service(ctx, pool, mode=mode, max_batch=8, hbm_budget=8 << 30)
        rep = svc.run(stream)
        assert rep["served"] == 60 and sorted(rep["ids"]) == list(range(60)), mode
        assert 0 < rep["p50_ms"] <= rep["p99_ms"], rep
