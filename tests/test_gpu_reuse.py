"""Buffer reuse across forwards: the tile lists are emitted and sorted before the host reads
the frame's pair count, on buffers sized from the state's previous frame, and emitted again
when a buffer was too small or the chunk length changed.  Every path must give exactly the
frame a fresh context gives (the forward is deterministic), and the pair counts must agree.

Scenes: the 64x1024 street block with 20,000 and with 300,000 surfels (chunk lengths 32
and 48), and a crowded 32x256 room.  Sequence on one context, for the scratch state (no state
kept) and for pooled states (state kept and freed): small, large (buffers too small: emitted
again), large (lists reused), small (lists reused, chunk list rebuilt), room, large."""
import numpy as np
import pytest

import scenegen
from tests import _gpu as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def scenes():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    small = scenegen.make_workload("block64x1024_300k", n=20_000, with_targets=False)
    large = scenegen.make_workload("block64x1024_300k", with_targets=False)
    room = scenegen.make_workload("room32x256_1k", with_targets=False)
    return {k: G.to_dev(w) for k, w in (("small", small), ("large", large), ("room", room))}


def _frame(ctx, dw, keep):
    from paper_2607_04127_amd import lgsr
    fr, st = G.gpu_forward(ctx, dw, want_state=keep)
    torch.cuda.synchronize()
    pairs = None
    if keep:
        pairs = lgsr.lgsr_query(ctx, st)["pairs"]
        st.free()
    return {k: v.detach().cpu().clone() for k, v in fr.items()}, pairs


@pytest.mark.parametrize("keep", [False, True])
def test_reused_buffers_give_the_fresh_frame(scenes, keep):
    from paper_2607_04127_amd import lgsr
    want = {}
    for name, dw in scenes.items():
        c = lgsr.Context(0)
        want[name] = _frame(c, dw, True)
        c.close()
    ctx = lgsr.Context(0)
    try:
        for step, name in enumerate(["small", "large", "large", "small", "room", "large"]):
            got, pairs = _frame(ctx, scenes[name], keep)
            ref, ref_pairs = want[name]
            print(f"\n[reuse keep={keep}] step {step} {name}: pairs {pairs} (fresh {ref_pairs})", flush=True)
            for k in ref:
                assert torch.equal(got[k], ref[k]), (step, name, k)
            if keep:
                assert pairs == ref_pairs, (step, name)
    finally:
        ctx.close()
