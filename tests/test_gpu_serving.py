"""GPU: the continuous-batching server.  Every served frame is bit-identical
to the same request rendered alone, whatever batch and stream slot it ran in,
and matches the oracle (RGBA8 within 1 LSB).  A frame whose first render
overflows its bin lists is found from its batch's status words and rendered
again, so no request completes with a stale image."""
import numpy as np
import pytest

import oracle
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


def check_against_oracle(r, out, by_handle):
    sc = by_handle[r.scene]
    ref = oracle.render(sc.v, sc.rgba, r.camera, r.width, r.height, want_order=False)
    d8 = np.abs(out.astype(np.int32) - ref["rgba8"].astype(np.int32))
    assert d8.max(initial=0) <= 1, f"request {r.rid}: off by {d8.max()}"


def test_served_frames_equal_standalone_renders(lr):
    ctx = lr.Context(arena_bytes=1 << 30, batch_slots=2, graphs=False)
    rng = np.random.default_rng(3)
    meta, by_handle = [], {}
    for s in range(8):
        W, H = int(rng.integers(16, 320)), int(rng.integers(16, 240))
        sc = scenes.small(W, H, int(rng.integers(200, 20000)), 2000 + s, side=(1.0, 24.0),
                          gaussian=bool(s % 2), alpha=(0.05, 0.8))
        h = ctx.upload(sc.v, sc.rgba)
        meta.append((h, W, H))
        by_handle[h] = sc
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
        served = be.outputs[r.rid].cpu().numpy()
        alone = ctx.render(r.scene, r.camera, r.width, r.height).cpu().numpy()
        np.testing.assert_array_equal(served, alone, err_msg=f"request {r.rid}")
        check_against_oracle(r, served, by_handle)
    ctx.close()


def test_status_words_report_capacity_overflow(lr):
    """lr_request.status: 0 for a frame whose image was written, the capacity
    bit for a frame whose bin lists overflowed on its first render."""
    import torch
    ctx = lr.Context(arena_bytes=1 << 30, graphs=False)
    big = scenes.small(320, 240, 3000, 91, side=(80.0, 140.0), alpha=(0.05, 0.4))  # ~35 bins per quad
    light = scenes.small(96, 72, 500, 92, side=(2.0, 10.0))
    hb, hl = ctx.upload(big.v, big.rgba), ctx.upload(light.v, light.rgba)
    ob, ol = ctx.new_image(320, 240), ctx.new_image(96, 72)
    status = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    reqs = [(hb, big.camera, 320, 240, ob, 16, 8, 8), (hl, light.camera, 96, 72, ol, 16, 8, 8)]
    ctx.render_batch(reqs, check=False, status=status)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [lr.LR_FRAME_ERR_CAPACITY, 0]
    with pytest.raises(lr.LRError):
        ctx.sync()  # reports the overflow and raises the capacity hint
    ctx.render_batch(reqs, check=False, status=status)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0, 0]
    ref = oracle.render(big.v, big.rgba, big.camera, 320, 240, want_order=False)
    assert np.abs(ob.cpu().numpy().astype(np.int32) - ref["rgba8"].astype(np.int32)).max() <= 1
    ctx.close()


def test_server_renders_overflowed_frames_again(lr):
    """No warm-up: the first batch holding a scene of large quads overflows
    its bin lists; the server finds it from the status words, raises the
    capacity and renders those frames again.  Every served frame matches the
    oracle."""
    ctx = lr.Context(arena_bytes=1 << 30, batch_slots=2, graphs=False)
    meta, by_handle = [], {}
    for s in range(4):
        if s % 2 == 0:
            sc = scenes.small(320, 240, 3000, 93 + s, side=(80.0, 140.0), alpha=(0.05, 0.4))
        else:
            sc = scenes.small(128, 96, 2000, 93 + s, side=(2.0, 16.0))
        h = ctx.upload(sc.v, sc.rgba)
        meta.append((h, sc.width, sc.height))
        by_handle[h] = sc
    trace = poisson_trace(50000.0, 24, meta, seed=3100)
    for r in trace:
        r.tune = (16, 8, 8)
    be = GpuBackend(ctx, slots=2, keep_outputs=True)
    srv = Server(be, budget_bytes=512 << 20, slots=2, max_batch=6)
    be.start_clock()
    done = srv.run(trace)
    ctx.sync()
    assert sorted(c.rid for c in done) == list(range(len(trace)))
    assert be.retried  # some frames overflowed and were rendered again
    for r in trace:
        check_against_oracle(r, be.outputs[r.rid].cpu().numpy(), by_handle)
    ctx.close()


def test_admission_binds_under_a_tight_budget(lr):
    """A budget of about two and a half of the largest request footprints:
    requests arriving together are admitted a few at a time (batches closed
    by the budget, free slots waiting for memory), bytes in flight never
    exceed the budget, and every served frame still matches the oracle."""
    ctx = lr.Context(arena_bytes=1 << 30, batch_slots=2, graphs=False)
    rng = np.random.default_rng(4)
    meta, by_handle = [], {}
    for s in range(6):
        W, H = int(rng.integers(64, 320)), int(rng.integers(48, 240))
        sc = scenes.small(W, H, int(rng.integers(2000, 20000)), 2100 + s, side=(1.0, 24.0), alpha=(0.05, 0.8))
        h = ctx.upload(sc.v, sc.rgba)
        meta.append((h, W, H))
        by_handle[h] = sc
    for h, W, H in meta:  # warm-up: plans each scene's capacity
        ctx.render(h, scenes.Camera(), W, H)
    trace = poisson_trace(1e7, 40, meta, seed=3200)  # all but simultaneous
    be = GpuBackend(ctx, slots=2, keep_outputs=True)
    budget = int(2.5 * max(be.footprint(r) for r in trace))
    srv = Server(be, budget_bytes=budget, slots=2, max_batch=16)
    be.start_clock()
    done = srv.run(trace)
    ctx.sync()
    assert sorted(c.rid for c in done) == list(range(len(trace)))
    assert srv.stats["budget_cut_batches"] > 0
    assert srv.stats["max_inflight"] <= budget
    for r in trace:
        check_against_oracle(r, be.outputs[r.rid].cpu().numpy(), by_handle)
    ctx.close()
