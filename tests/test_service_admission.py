"""Host logic of the rendering service (no GPU): Poisson arrivals and admission of queued
requests into a batch by count and by the estimated HBM working set."""
import collections

import numpy as np
import pytest

from paper_2607_04127_amd import service as SV


def _pool():
    # templates by size only: admission reads n (surfels), the beam model and the pair count
    return [dict(n=100_000, rays=32 * 1024, H=32, W=1024, pairs=None),
            dict(n=2_000_000, rays=128 * 2048, H=128, W=2048, pairs=None),
            dict(n=400_000, rays=64 * 1024, H=64, W=1024, pairs=300_000)]


def test_poisson_stream_statistics():
    pool = _pool()
    s = SV.poisson_stream(pool, 20_000, rate=500.0, grad_fraction=0.3, seed=7)
    t = np.array([r.t for r in s])
    assert np.all(np.diff(t) >= 0) and [r.id for r in s] == list(range(20_000))
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 500.0) < 0.03 / 500.0          # mean inter-arrival 1/rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.03            # exponential: cv = 1
    assert abs(np.mean([r.grad for r in s]) - 0.3) < 0.015
    counts = np.bincount([r.template for r in s], minlength=3)
    assert counts.min() > 0.3 * 20_000
    # same seed, same stream
    assert SV.poisson_stream(pool, 20_000, 500.0, grad_fraction=0.3, seed=7) == s


def test_working_set_grows_with_gradients_and_size():
    a, b = _pool()[0], _pool()[1]
    assert SV.working_bytes(a, True) > SV.working_bytes(a, False) > 0
    assert SV.working_bytes(b, False) > SV.working_bytes(a, False)


def test_working_set_covers_the_library_account():
    """The admission model is at least the library's own account of a request's buffers
    (lgsr_request_bytes, sized as the library allocates them, slots of the chunk summaries,
    pair lists and sort workspace included) for the benchmark shape and the service's
    shapes, at the measured or the assumed pair count; an unmeasured template is budgeted
    with more pairs than the measured one of the same shape."""
    from paper_2607_04127_amd import lgsr
    cfg2 = dict(n=300_000, rays=64 * 1024, H=64, W=1024, pairs=229_247)
    for tp in [cfg2] + _pool():
        P = tp["pairs"] if tp["pairs"] is not None else SV.PAIRS_PER_SURFEL_BOUND * tp["n"]
        for g in (False, True):
            assert SV.working_bytes(tp, g) >= lgsr.lgsr_request_bytes(tp["n"], tp["H"], tp["W"], P, g)
    # per-chunk summaries dominate at 64 x 1024 / 300k: 9 x 256 floats per chunk
    assert lgsr.lgsr_request_bytes(300_000, 64, 1024, 229_247, False) > 9 * 256 * 4 * (256 + 229_247 // 48)
    assert SV.working_bytes(dict(cfg2, pairs=None), False) > SV.working_bytes(cfg2, False)


def _queue(pool, spec):
    return collections.deque(SV.Request(i, 0.0, tpl, g) for i, (tpl, g) in enumerate(spec))


def test_admission_fifo_count_and_budget():
    pool = _pool()
    spec = [(0, False), (2, True), (1, False), (0, True), (0, False)]
    need = [SV.working_bytes(pool[t], g) for t, g in spec]
    # by count: the first max_batch requests, in arrival order
    svc = SV.Service(None, pool, "batched", max_batch=3, hbm_budget=1 << 60)
    q = _queue(pool, spec)
    assert [r.id for r in svc._admit(q)] == [0, 1, 2]
    assert [r.id for r in svc._admit(q)] == [3, 4]
    assert not q
    # by memory: stop before the request that would exceed the budget (no reordering)
    svc = SV.Service(None, pool, "batched", max_batch=16, hbm_budget=need[0] + need[1] + need[2] - 1)
    q = _queue(pool, spec)
    assert [r.id for r in svc._admit(q)] == [0, 1]
    # a request larger than the whole budget still runs, alone
    svc = SV.Service(None, pool, "batched", max_batch=16, hbm_budget=1)
    q = _queue(pool, spec)
    assert [r.id for r in svc._admit(q)] == [0]
    # one request per call in single mode
    svc = SV.Service(None, pool, "single", max_batch=16)
    q = _queue(pool, spec)
    assert [r.id for r in svc._admit(q)] == [0]
    with pytest.raises(ValueError):
        SV.Service(None, pool, "other")
