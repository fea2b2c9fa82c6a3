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


def _rel(a, b):
    return float((a - b).abs().max() / max(float(b.abs().max()), 1e-30))


def _near(a, b):
    return float((a - b).abs().max()) <= 1e-5 * float(b.abs().max()) + 1e-30


def _close(a, b, what):
    a, b = a.detach().cpu().numpy().astype(np.float64), b.detach().cpu().numpy().astype(np.float64)
    scale = np.abs(b).max() if b.size else 0.0
    assert np.abs(a - b).max(initial=0.0) <= 1e-5 * scale + 1e-30, what


@pytest.mark.parametrize("fused", [False, True])
def test_batch_matches_single_calls(ctx, fused):
    """Both batch modes: requests on four streams, and one launch per compositing stage for
    the whole batch (LGSR_FLAG_BATCH_FUSED)."""
    from paper_2607_04127_amd import lgsr
    reqs = _requests(3)
    opts = lgsr.default_opts(flags=lgsr.LGSR_FLAG_BATCH_FUSED if fused else 0)
    for rep in range(2):  # the second batch reuses the internal per-request states
        res = lgsr.lgsr_render_batch(ctx, reqs, opts=opts)
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
                bad = [key for key in G.SURF_KEYS if not _near(r["grads"][key], out[key])]
                if bad:
                    # tell which side moved: a second single-call backward of the same forward
                    out2, _ = lgsr.lgsr_backward(ctx, st, g)
                    torch.cuda.synchronize()
                    diag = {key: (_rel(r["grads"][key], out[key]), _rel(out2[key], out[key]),
                                  int(((r["grads"][key] - out[key]).abs() > 1e-5 * out[key].abs().max()).any(-1).sum()))
                            for key in bad}
                    raise AssertionError(f"request {k} rep {rep}: (batch vs single, single vs single, surfels) {diag}")
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


@pytest.mark.parametrize("fused", [False, True])
def test_batch_matches_oracle(ctx, fused):
    """One batch mixing two maps (the 1k-surfel room and a 20k-surfel street block), four beam
    models and render / render + gradient requests, every request against the FP64 oracle:
    frames at the parity bars on every ray (the 64 x 1024 one on 4096 sampled rays), the
    loss, and the parameter and pose gradients at the per-surfel bar.  Rays the oracle flags
    as ties get target depth 0, which takes them out of both losses."""
    from oracle import ref
    from paper_2607_04127_amd import lgsr
    room = scenegen.make_workload("room32x256_1k")
    block = scenegen.make_workload("block64x1024_300k", n=20_000)
    worlds = (room, block)
    beams = [(32, 256, -15, 15), (37, 250, -15, 15), (16, 512, -10, 10), (64, 1024, -22.5, 22.5)]
    plan = [(0, 0, True), (1, 2, True), (0, 1, False), (1, 3, False), (1, 0, True), (0, 2, False)]
    rng = np.random.default_rng(17)
    reqs, meta = [], []
    for mi, bi, grad in plan:
        w0 = worlds[mi]
        rows, cols = scenegen.beam_tables(*beams[bi])
        T = np.asarray(w0["pose"], np.float64).copy()
        T[:, 3] += rng.normal(scale=0.3, size=3)
        w = dict({k: w0[k] for k in G.SURF_KEYS}, row_sincos=rows, col_sincos=cols, pose=T.astype(np.float32))
        H, W = rows.shape[0], cols.shape[0]
        ids = None if H * W <= 16384 else np.sort(rng.choice(H * W, 4096, replace=False))
        of = G.oracle_forward(w, ray_ids=ids)
        q = dict(surfels={k: torch.from_numpy(np.ascontiguousarray(w[k])).cuda() for k in G.SURF_KEYS},
                 pose=w["pose"], row_sincos=torch.from_numpy(rows).cuda(), col_sincos=torch.from_numpy(cols).cuda())
        if grad:
            assert ids is None
            # targets off the rendered surfaces (a decided L1 sign), normals random; ties out
            td = np.where(of["K"] > 0, of["depth"] + rng.choice([-1, 1], H * W) * rng.uniform(0.1, 0.5, H * W), 5.0)
            td[G.tie_mask(of)] = 0.0
            nrm = rng.normal(size=(H * W, 3))
            tn = nrm / np.linalg.norm(nrm, axis=1, keepdims=True)
            tn[td == 0] = 0.0
            w["target_depth"], w["target_normal"] = td.astype(np.float32).reshape(H, W), tn.astype(np.float32).reshape(H, W, 3)
            q["target_depth"] = torch.from_numpy(w["target_depth"]).cuda()
            q["target_normal"] = torch.from_numpy(w["target_normal"]).cuda()
        reqs.append(q)
        meta.append((w, of, ids, grad))
    res = lgsr.lgsr_render_batch(ctx, reqs, opts=lgsr.default_opts(flags=lgsr.LGSR_FLAG_BATCH_FUSED if fused else 0))
    torch.cuda.synchronize()
    assert all(lgsr.lgsr_batch_poll(ctx, len(reqs)))
    for k, (r, (w, of, ids, grad)) in enumerate(zip(res, meta)):
        stats = G.compare_forward(r["frame"], of, ray_ids=ids)
        line = f"\n[batch vs oracle {k}] {w['row_sincos'].shape[0]}x{w['col_sincos'].shape[0]} N={w['means'].shape[0]} " \
               f"hit={stats['hit']} tie={stats['tie']} depth={stats['max_rel_depth']:.1e} " \
               f"opacity={stats['max_rel_opacity']:.1e}"
        if grad:
            td = w["target_depth"].reshape(-1)
            tn = w["target_normal"].reshape(-1, 3)
            L_ref, gd, go, gn = ref.loss(of, td, tn)
            np.testing.assert_allclose(r["loss"].cpu().numpy()[:3], L_ref[:3], rtol=1e-5)
            assert tuple(r["loss"].cpu().numpy()[3:]) == tuple(L_ref[3:])
            g_ref = ref.backward(w, w["pose"], w["row_sincos"], w["col_sincos"], gd, go, gn, with_mass=True)
            for c, key in enumerate(G.SURF_KEYS):
                nbad, cos, worst = G.grad_check(r["grads"][key].cpu().numpy(), g_ref[key], mass=g_ref["mass"][:, c])
                assert nbad == 0 and cos > 0.99999, (k, key, nbad, cos, worst)
                line += f" {key}={worst:.3f}"
            nbad, cos, worst = G.grad_check(r["grad_pose"].cpu().numpy(), g_ref["pose"], mass=g_ref["pose_mass"],
                                            per_row=False)
            assert nbad == 0, (k, "pose", worst)
            line += f" pose={worst:.3f}"
        print(line, flush=True)
