"""GPU: the continuous-batching server.  Every served frame is bit-identical
to the same request rendered alone, whatever batch and stream slot it ran in."""
import numpy as np
import pytest

from paper_2405_13364_amd import scenes
from paper_2405_13364_amd.serving import GpuBackend, Server, poisson_trace, summarize

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_13364_amd import lucidraster
    return lucidraster


def test_served_frames_equal_standalone_renders(lr):
    ctx = lr.Context(arena_bytes=1 << 30, batch_slots=2, graphs=False)
    rng = np.random.default_rng(3)
    meta = []
    for s in range(8):
        W, H = int(rng.integers(16, 320)), int(rng.integers(16, 240))
        sc = scenes.small(W, H, int(rng.integers(200, 20000)), 2000 + s, side=(1.0, 24.0),
                          gaussian=bool(s % 2), alpha=(0.05, 0.8))
        meta.append((ctx.upload(sc.v, sc.rgba), W, H))
    for h, W, H in meta:  # warm-up: plans each scene's capacity
        ctx.render(h, scenes.Camera(), W, H)
    trace = poisson_trace(20000.0, 80, meta, seed=3000)
    be = GpuBackend(ctx, slots=2, keep_outputs=True)
    srv = Server(be, budget_bytes=256 << 20, slots=2, max_batch=8)
    be.start_clock()
    done = srv.run(trace)
    ctx.sync()
    assert sorted(c.rid for c in done) == list(range(len(trace)))
    summ = summarize(done)
    assert summ["batches"] < len(trace)  # requests were batched
    for r in trace:
        alone = ctx.render(r.scene, r.camera, r.width, r.height).cpu().numpy()
        np.testing.assert_array_equal(be.outputs[r.rid].cpu().numpy(), alone, err_msg=f"request {r.rid}")
    ctx.close()
