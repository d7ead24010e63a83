"""lr_render_noalloc, the render whose frame workspace is the library's fixed
device array (for callers that cannot allocate), against lr_render through
the C ABI: two calls in a row, the second on a smaller frame with fewer
quads, each bit-identical to lr_render of the same request and within the
oracle's bars; a frame too large for the array is refused before anything
is launched."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2405_13364_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_13364_amd import lucidraster
    return lucidraster


def check_against_oracle(img, st, sc):
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, want_order=False)
    d8 = np.abs(img.cpu().numpy().astype(np.int32) - ref["rgba8"].astype(np.int32))
    assert d8.max(initial=0) <= 1
    assert st["fragments"] == ref["total"]
    assert st["error_word"] & lr_err_capacity() == 0


def lr_err_capacity():
    from paper_2405_13364_amd import lucidraster
    return lucidraster.LR_FRAME_ERR_CAPACITY


@pytest.mark.parametrize("bin_size,k,bh", [(32, 8, 8), (16, 4, 4)])
def test_noalloc_matches_render_twice_second_smaller(lr, bin_size, k, bh):
    import torch
    big = scenes.small(200, 150, 30000, 61, side=(1.0, 20.0), gaussian=True, alpha=(0.05, 0.5))
    small = scenes.small(70, 45, 900, 62, side=(2.0, 16.0))
    ctx = lr.Context(arena_bytes=256 << 20, bin_size=bin_size, sorter_depth=k, block_h=bh)
    hb = ctx.upload(big.v, big.rgba)
    hs = ctx.upload(small.v, small.rgba)
    for h, sc in ((hb, big), (hs, small)):
        # poison the output so an unwritten image cannot pass
        got = torch.full((sc.height, sc.width, 4), 0x5A, dtype=torch.uint8, device="cuda")
        ctx.render_noalloc(h, sc.camera, sc.width, sc.height, out=got)
        st = ctx.stats()
        want = ctx.render(h, sc.camera, sc.width, sc.height)
        st_want = ctx.stats()
        assert torch.equal(got, want), f"{sc.width}x{sc.height}: noalloc image differs from lr_render"
        for key in ("visible", "bin_pairs", "block_entries", "fragments", "flagged_pixels"):
            assert st[key] == st_want[key], key
        check_against_oracle(got, st, sc)
    ctx.close()


def test_noalloc_on_a_second_stream_after_the_first(lr):
    import torch
    sc = scenes.small(160, 120, 20000, 63, side=(1.0, 20.0), gaussian=True, alpha=(0.05, 0.5))
    ctx = lr.Context(arena_bytes=256 << 20)
    h = ctx.upload(sc.v, sc.rgba)
    s2 = torch.cuda.Stream()
    a = ctx.render_noalloc(h, sc.camera, sc.width, sc.height)
    b = ctx.render_noalloc(h, sc.camera, sc.width, sc.height, stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(a, ctx.render(h, sc.camera, sc.width, sc.height))
    ctx.close()


def test_noalloc_refuses_a_frame_larger_than_its_array(lr):
    sc = scenes.small(64, 64, 1000, 64, side=(2.0, 10.0))
    ctx = lr.Context(arena_bytes=64 << 20, bin_size=64)
    h = ctx.upload(sc.v, sc.rgba)
    # an 8192 x 8192 frame (16384 bins of 64 px) needs a flagged-pixel queue
    # of 256 MiB alone; the output is full size all the same
    with pytest.raises(lr.LRError) as e:
        ctx.render_noalloc(h, sc.camera, 8192, 8192, out=ctx.new_image(8192, 8192))
    assert e.value.status == lr.LR_ERR_OUT_OF_MEMORY
    assert "static scratch" in str(e.value)
    # the library's figure for a 1280x720 frame of 200k quads is within the array
    c2 = scenes.scene("c2")
    ctx2 = lr.Context(arena_bytes=64 << 20)
    h2 = ctx2.upload(c2.v, c2.rgba)
    assert ctx2.request_bytes(h2, c2.camera, c2.width, c2.height, 32, 8, 8) <= 128 << 20
    ctx2.close()
    ctx.close()
