"""GPU parity over a seeded sweep of frame shapes, scene kinds and tunings,
each frame checked whole against the CPU oracle (counts, order, colour) and
its fragment statistics against the oracle's total.

The cases reach paths the fixed scenes do not: frames with more than 8192
bins (the one-wave binning kernels), quads spanning hundreds of bins (one
quad filling several 64-pair scatter windows), frames whose every quad is
culled, single quads, and every sorter depth and block shape."""
import numpy as np
import pytest

import oracle
from paper_2405_13364_amd import scenes
from test_gpu_parity import check_frame, general_quads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_13364_amd import lucidraster
    return lucidraster


def behind_camera(W, H, n, seed):
    """Every quad behind the near plane: an empty (transparent) frame."""
    sc = scenes.small(W, H, n, seed)
    v = sc.v.copy()
    v[:, :, 2] = -np.abs(v[:, :, 2]) - 1.0
    return scenes.Scene(v=v, rgba=sc.rgba, width=W, height=H, camera=sc.camera, name="behind")


def partly_culled(W, H, n, seed):
    """Every third quad behind the near plane: culled and visible quads
    interleave within each setup workgroup."""
    sc = scenes.small(W, H, n, seed, side=(2.0, 20.0))
    v = sc.v.copy()
    v[::3, :, 2] = -np.abs(v[::3, :, 2]) - 1.0
    return scenes.Scene(v=v, rgba=sc.rgba, width=W, height=H, camera=sc.camera, name="partly_culled")


def sweep_cases():
    cases = [
        # more than 8192 bins at bin 16: the one-wave count and scatter kernels
        ("many_bins", lambda: scenes.small(2100, 1100, 3000, 41, side=(2.0, 30.0)), (16, 8, 8)),
        # quads hundreds of pixels across: hundreds of bins per quad
        ("huge_quads", lambda: scenes.small(640, 480, 40, 42, side=(150.0, 700.0), z=(1.0, 2.0),
                                            alpha=(0.1, 0.4)), (16, 4, 8)),
        ("huge_quads_bin64", lambda: scenes.small(640, 480, 40, 42, side=(150.0, 700.0), z=(1.0, 2.0),
                                                  alpha=(0.1, 0.4)), (64, 12, 4)),
        ("all_culled", lambda: behind_camera(123, 77, 300, 43), (32, 8, 8)),
        ("one_quad", lambda: scenes.small(50, 40, 1, 44, side=(10.0, 30.0)), (32, 2, 8)),
        # setup stages a workgroup's 256 records and stores them together: a
        # last workgroup holding one quad, whole workgroups, and culled rows
        ("setup_tail_row", lambda: scenes.small(200, 150, 513, 47, side=(2.0, 20.0)), (32, 8, 8)),
        ("setup_whole_groups", lambda: scenes.small(200, 150, 512, 48, side=(2.0, 20.0)), (32, 4, 4)),
        ("setup_partly_culled", lambda: partly_culled(200, 150, 700, 49), (16, 8, 8)),
        ("general_bin16", lambda: general_quads(150, 90, 3000, 45, extent=(1.0, 20.0)), (16, 24, 8)),
        ("general_bin64", lambda: general_quads(150, 90, 3000, 46, extent=(1.0, 20.0)), (64, 32, 4)),
    ]
    rng = np.random.default_rng(4000)
    for i in range(8):
        W, H = int(rng.integers(1, 400)), int(rng.integers(1, 300))
        n = int(rng.integers(1, 6000))
        lo = float(rng.uniform(0.5, 8.0))
        side = (lo, lo + float(rng.uniform(0.5, 40.0)))
        gauss = bool(rng.integers(0, 2))
        tune = (int(rng.choice([16, 32, 64])), int(rng.choice([2, 4, 8, 12, 16, 24, 32])), int(rng.choice([8, 4])))
        seed = 4100 + i
        cases.append((f"random{i}", lambda W=W, H=H, n=n, side=side, gauss=gauss, seed=seed:
                      scenes.small(W, H, n, seed, side=side, gaussian=gauss, alpha=(0.05, 0.9)), tune))
    return cases


CASES = sweep_cases()
_ctx = {}


@pytest.mark.parametrize("name,make,tune", CASES, ids=[c[0] for c in CASES])
def test_sweep_frame(lr, name, make, tune):
    bin_size, k, bh = tune
    key = tune
    if key not in _ctx:
        _ctx[key] = lr.Context(arena_bytes=1 << 30, bin_size=bin_size, sorter_depth=k, block_h=bh)
    ctx = _ctx[key]
    sc = make()
    print(f"[sweep] {name}: {sc.width}x{sc.height}, {sc.n} quads, bin {bin_size}, K {k}, 8x{bh}", flush=True)
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    h = ctx.upload(sc.v, sc.rgba)
    try:
        got = ctx.render_debug(h, sc.camera, sc.width, sc.height, order=True)
        st = ctx.stats()
    finally:
        ctx.release(h)
    check_frame(got, ref, name)
    assert st["fragments"] == ref["total"], name
