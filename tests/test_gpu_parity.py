"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: setup records, bin lists, per-pixel fragment counts and blend order
bit-exact; RGBA8 within 1 LSB and fp32 colour within 1e-5 of the oracle's
fp64 result; fp32 colour bit-identical across sorter depths and bin sizes."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2405_13364_amd import scenes

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_scenes.json")


@pytest.fixture(scope="module")
def lr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_13364_amd import lucidraster
    return lucidraster


_ctx_cache = {}


def ctx_for(lr, bin_size=32, k=8, arena=512 << 20, block_h=8):
    key = (bin_size, k, arena, block_h)
    if key not in _ctx_cache:
        _ctx_cache[key] = lr.Context(arena_bytes=arena, bin_size=bin_size, sorter_depth=k, block_h=block_h)
    return _ctx_cache[key]


def hand_scene():
    data = json.load(open(GOLDEN))
    quads = []
    for case in data["cases"]:
        for q in case["quads"]:
            quads.append((scenes.screen_quad(q["corners"], q["z"], data["width"], data["height"]),
                          int(scenes.pack_rgba(*q["rgba"]))))
    return scenes.from_quads(quads, data["width"], data["height"], name="hand")


def wide_scene():
    # quads up to ~1500 px across on a 700x500 frame: the fp64 coverage path
    return scenes.small(700, 500, 40, 21, side=(200.0, 1500.0), z=(1.0, 3.0), alpha=(0.2, 0.6))


def general_quads(W=80, H=60, n=4000, seed=31, extent=(2.0, 12.0), centre=None):
    """Fronto-parallel quads whose four corners are drawn independently in a
    small box: convex, concave and self-intersecting (bow-tie) shapes mixed,
    so coverage takes both the four-edge and the two-triangle path inside one
    batch.  With a centre, every quad sits around that point (dense blocks)."""
    rng = np.random.default_rng(seed)
    quads = []
    for _ in range(n):
        if centre is None:
            cx, cy = rng.uniform(0.0, W), rng.uniform(0.0, H)
        else:
            cx, cy = centre[0] + rng.uniform(-4.0, 4.0), centre[1] + rng.uniform(-4.0, 4.0)
        e = rng.uniform(*extent)
        corners = [(cx + rng.uniform(-e, e), cy + rng.uniform(-e, e)) for _ in range(4)]
        rgb = rng.integers(0, 256, 3)
        rgba = int(scenes.pack_rgba(int(rgb[0]), int(rgb[1]), int(rgb[2]), int(rng.integers(20, 236))))
        quads.append((scenes.screen_quad(corners, float(rng.uniform(1.0, 10.0)), W, H), rgba))
    return scenes.from_quads(quads, W, H, name="general")


def thin_large(W=320, H=240, n=150, seed=51):
    """Long thin fronto-parallel quads (80-300 px by 2-6 px) turned in the
    screen plane: their bboxes meet many bins their area never reaches."""
    rng = np.random.default_rng(seed)
    quads = []
    for _ in range(n):
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        L, T = rng.uniform(80.0, 300.0), rng.uniform(2.0, 6.0)
        th = rng.uniform(0.0, np.pi)
        u, v = np.array([np.cos(th), np.sin(th)]), np.array([-np.sin(th), np.cos(th)])
        corners = [tuple(np.array([cx, cy]) + su * L / 2 * u + sv * T / 2 * v)
                   for su, sv in ((-1, -1), (1, -1), (1, 1), (-1, 1))]
        rgb = rng.integers(0, 256, 3)
        rgba = int(scenes.pack_rgba(int(rgb[0]), int(rgb[1]), int(rgb[2]), int(rng.integers(40, 200))))
        quads.append((scenes.screen_quad(corners, float(rng.uniform(1.0, 10.0)), W, H), rgba))
    return scenes.from_quads(quads, W, H, name="thin_large")


SCENES = {
    "small": lambda: scenes.small(96, 72, 3000, 11, side=(2.0, 24.0)),
    "ragged": lambda: scenes.small(101, 37, 1500, 12, side=(1.0, 30.0)),
    "tiny_frame": lambda: scenes.small(9, 7, 200, 13, side=(1.0, 6.0)),
    "one_pixel": lambda: scenes.small(1, 1, 50, 14, side=(1.0, 3.0)),
    "c1": lambda: scenes.scene("c1"),
    "hand": hand_scene,
    "wide": wide_scene,
    "gauss": lambda: scenes.small(160, 120, 20000, 15, side=(1.0, 20.0), gaussian=True, alpha=(0.05, 0.5)),
    "general": lambda: general_quads(),
    "general_dense": lambda: general_quads(64, 48, 900, 32, extent=(2.0, 14.0), centre=(28.0, 20.0)),
    # non-planar quads: fragments whose plane depth is not positive (key 0)
    "twisted": lambda: scenes.twisted(72, 56, 1500, 41),
    # long thin quads turned in the screen plane: the large-quad binning path
    "thin_large": lambda: thin_large(),
}


def moved_camera():
    cam = scenes.Camera.jittered(3.0, -2.0)
    cam.pos = (0.02, -0.03, 0.05)
    return cam


def gpu_render(lr, ctx, sc, cam=None, order=True):
    cam = cam or sc.camera
    h = ctx.upload(sc.v, sc.rgba)
    try:
        return ctx.render_debug(h, cam, sc.width, sc.height, order=order)
    finally:
        ctx.release(h)


def check_frame(got, ref, where=""):
    cnt = got["count"].cpu().numpy().astype(np.uint32)
    np.testing.assert_array_equal(cnt, ref["count"], err_msg=f"counts {where}")
    if "order_ids" in got:
        ids = got["order_ids"].cpu().numpy().astype(np.uint32)
        np.testing.assert_array_equal(ids, ref["order_ids"], err_msg=f"order {where}")
    d8 = np.abs(got["rgba8"].cpu().numpy().astype(np.int32) - ref["rgba8"].astype(np.int32))
    assert d8.max(initial=0) <= 1, f"rgba8 off by {d8.max()} {where}"
    df = np.abs(got["rgba_f32"].cpu().numpy().astype(np.float64) - ref["rgba_f64"])
    assert df.max(initial=0) <= F32_TOL, f"fp32 colour off by {df.max()} {where}"


@pytest.mark.parametrize("name", sorted(SCENES))
def test_setup_parity(lr, name):
    sc = SCENES[name]()
    for cam in (sc.camera, moved_camera()):
        ctx = ctx_for(lr)
        h = ctx.upload(sc.v, sc.rgba)
        got = ctx.debug_setup(h, cam, sc.width, sc.height, sc.n)
        ctx.release(h)
        st = oracle.setup(sc.v, cam, sc.width, sc.height)
        np.testing.assert_array_equal(got["cull"], st.cull)
        vis = st.cull == 0
        np.testing.assert_array_equal(got["X"][vis], st.X[vis])
        np.testing.assert_array_equal(got["Y"][vis], st.Y[vis])
        np.testing.assert_array_equal(got["bbox"][vis], st.bbox[vis])
        pl = np.stack([st.A, st.B, st.C0], axis=1)
        np.testing.assert_array_equal(got["plane"][vis].view(np.uint64), pl[vis].view(np.uint64))


def large_quads(st):
    """Quads whose bbox meets more than 4 bins of 32 px (Stage 1's
    small/large split)."""
    b = st.bbox
    return ((b[:, 1] // 32 - b[:, 0] // 32 + 1) * (b[:, 3] // 32 - b[:, 2] // 32 + 1) > 4) & (st.cull == 0)


def check_bin_lists(counts, ids, sc, st, bin_size):
    """Small quads: every bin their bbox meets (the oracle's bbox lists), in
    ascending order within each list.  Large quads: a subset of those bins
    that holds every bin with a covered sample (the trivial reject only
    drops bins with none), anywhere in the list, once."""
    W, H = sc.width, sc.height
    rc, roff, rids = oracle.bins(st, W, H, bin_size)
    large = large_quads(st)
    ref = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    nbx = (W + bin_size - 1) // bin_size
    covered = {}
    off = ref["order_offsets"]
    for p in range(W * H):
        q = ref["order_ids"][int(off[p]):int(off[p + 1])]
        if len(q):
            b = (p // W // bin_size) * nbx + (p % W) // bin_size
            covered.setdefault(b, set()).update(int(x) for x in q)
    got_off = np.zeros(counts.size + 1, np.int64)
    got_off[1:] = np.cumsum(counts.reshape(-1).astype(np.int64))
    for b in range(counts.size):
        g = ids[got_off[b]:got_off[b + 1]]
        r = rids[int(roff[b]):int(roff[b + 1])]
        small = np.array([q for q in g if not large[q]], np.int64)
        assert np.all(np.diff(small) > 0), f"bin {b}: small quads not ascending"
        assert len(set(g.tolist())) == len(g), f"bin {b}: a quad listed twice"
        assert set(g.tolist()) <= set(r.tolist()), f"bin {b}: quads outside the bbox lists"
        must = {int(q) for q in r if not large[q]} | covered.get(b, set())
        assert must <= set(g.tolist()), f"bin {b}: missing {sorted(must - set(g.tolist()))[:5]}"
    return int(large.sum())


@pytest.mark.parametrize("name,bands", [("c2", 2), ("c3", 4)])
def test_bins_parity_in_row_bands(lr, name, bands):
    """Frames of more than 2048 bins of 16 px scatter in bands of bin rows
    (1280x720: two bands of 23 and 22 rows; 1920x1080: four of 17): every
    bin list holds the oracle's bbox list of small quads in ascending order,
    and large quads (the 1920x1080 frame has a few) only from its bbox list,
    once each."""
    sc = scenes.scene(name)
    st = oracle.setup(sc.v, sc.camera, sc.width, sc.height)
    large = large_quads(st)
    nby = (sc.height + 15) // 16
    nbx = (sc.width + 15) // 16
    b = 1
    while 2 * b <= nby and ((nby + b - 1) // b) * nbx > 2048:
        b *= 2
    assert b == bands
    ctx = lr.Context(arena_bytes=2 << 30, bin_size=16)
    h = ctx.upload(sc.v, sc.rgba)
    counts, ids = ctx.debug_bins(h, sc.camera, sc.width, sc.height, 16)
    ctx.close()
    rc, roff, rids = oracle.bins(st, sc.width, sc.height, 16)
    counts = np.asarray(counts).reshape(-1).astype(np.int64)
    goff = np.concatenate([[0], np.cumsum(counts)])
    ids = np.asarray(ids, np.int64)
    rids = rids.astype(np.int64)
    if not large.any():
        np.testing.assert_array_equal(counts, rc.reshape(-1))
        np.testing.assert_array_equal(ids, rids)
        return
    for b in range(counts.size):
        g = ids[goff[b]:goff[b + 1]]
        r = rids[int(roff[b]):int(roff[b + 1])]
        np.testing.assert_array_equal(g[~large[g]], r[~large[r]], err_msg=f"bin {b}: small quads")
        gl = g[large[g]]
        assert len(np.unique(gl)) == len(gl) and np.isin(gl, r).all(), f"bin {b}: large quads"


@pytest.mark.parametrize("bin_size", [16, 32, 64])
@pytest.mark.parametrize("name", ["small", "c1", "ragged", "wide", "thin_large"])
def test_bins_parity(lr, name, bin_size):
    sc = SCENES[name]()
    ctx = ctx_for(lr)
    h = ctx.upload(sc.v, sc.rgba)
    counts, ids = ctx.debug_bins(h, sc.camera, sc.width, sc.height, bin_size)
    ctx.release(h)
    st = oracle.setup(sc.v, sc.camera, sc.width, sc.height)
    nlarge = check_bin_lists(counts, ids, sc, st, bin_size)
    if name == "thin_large":
        assert nlarge > 0 and counts.sum() < oracle.bins(st, sc.width, sc.height, bin_size)[0].sum()
    # with LR_FLAG_BBOX_BINNING every quad takes its whole bbox: the oracle's lists
    c2 = lr.Context(arena_bytes=256 << 20, bbox_binning=True)
    h2 = c2.upload(sc.v, sc.rgba)
    counts2, ids2 = c2.debug_bins(h2, sc.camera, sc.width, sc.height, bin_size)
    c2.close()
    rc, roff, rids = oracle.bins(st, sc.width, sc.height, bin_size)
    np.testing.assert_array_equal(counts2, rc)
    np.testing.assert_array_equal(ids2, rids)


@pytest.mark.parametrize("name", sorted(SCENES))
def test_render_parity(lr, name):
    sc = SCENES[name]()
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    got = gpu_render(lr, ctx_for(lr), sc)
    check_frame(got, ref, name)


def test_render_parity_moved_camera(lr):
    sc = SCENES["small"]()
    cam = moved_camera()
    ref = oracle.render(sc.v, sc.rgba, cam, sc.width, sc.height)
    got = gpu_render(lr, ctx_for(lr), sc, cam)
    check_frame(got, ref, "moved camera")


@pytest.mark.parametrize("name", ["small", "gauss", "c1", "ragged"])
def test_unsorted_parity(lr, name):
    import torch
    sc = SCENES[name]()
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, unsorted=True, want_order=False)
    ctx = ctx_for(lr)
    h = ctx.upload(sc.v, sc.rgba)
    f32 = torch.zeros((sc.height, sc.width, 4), dtype=torch.float32, device="cuda")
    out = ctx.render_unsorted(h, sc.camera, sc.width, sc.height, rgba_f32=f32)
    ctx.release(h)
    d8 = np.abs(out.cpu().numpy().astype(np.int32) - ref["rgba8"].astype(np.int32)).max()
    df = np.abs(f32.cpu().numpy().astype(np.float64) - ref["rgba_f64"]).max()
    assert d8 <= 1 and df <= F32_TOL, (d8, df)


def test_invariance_over_sorter_depth_and_bins(lr):
    """Sorter depth, bin size, block shape and repetition never change a single bit."""
    sc = SCENES["gauss"]()
    base = gpu_render(lr, ctx_for(lr), sc, order=False)
    b32 = base["rgba_f32"].cpu().numpy()
    b8 = base["rgba8"].cpu().numpy()
    flagged = {}
    for bh in (8, 4):
        for bin_size in (16, 32, 64):
            for k in ((2, 4, 8, 16, 32) if bh == 8 else (2, 8, 32)):
                got = gpu_render(lr, ctx_for(lr, bin_size, k, block_h=bh), sc, order=False)
                np.testing.assert_array_equal(got["rgba_f32"].cpu().numpy().view(np.uint32),
                                              b32.view(np.uint32), err_msg=f"bin {bin_size} K {k} block h {bh}")
                np.testing.assert_array_equal(got["rgba8"].cpu().numpy(), b8)
                flagged[(bh, bin_size, k)] = int(got["flagged"].cpu().numpy().sum())
    # a shallower sorter sends more pixels down the exact path
    assert flagged[(8, 32, 2)] >= flagged[(8, 32, 32)]


@pytest.mark.parametrize("name", ["gauss", "c1", "ragged", "wide", "general", "general_dense"])
def test_half_block_parity(lr, name):
    """8x4 half-block sort keys: counts, order and colour against the oracle."""
    sc = SCENES[name]()
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    got = gpu_render(lr, ctx_for(lr, 32, 8, block_h=4), sc)
    check_frame(got, ref, f"{name} 8x4")


def test_forced_fallback_is_exact(lr):
    """K = 2 on a dense cloud: many pixels overflow the sorter and are
    recomputed; the frame is still exact."""
    sc = SCENES["gauss"]()
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    got = gpu_render(lr, ctx_for(lr, 32, 2), sc)
    check_frame(got, ref, "K=2")
    assert int(got["flagged"].cpu().numpy().sum()) > 0


def stacked_block_scene(nq, W=64, H=48, seed=5):
    """nq small fronto-parallel quads stacked over the same 8x8 block at
    random depths: the block's list exceeds the on-chip capacity."""
    rng = np.random.default_rng(seed)
    quads = []
    for q in range(nq):
        x0, y0 = rng.uniform(16.2, 20.0), rng.uniform(8.2, 12.0)
        w, h = rng.uniform(3, 12, 2)
        z = float(rng.uniform(1.0, 9.0))
        corners = [[x0, y0], [x0 + w, y0], [x0 + w, y0 + h], [x0, y0 + h]]
        quads.append((scenes.screen_quad(corners, z, W, H), int(rng.integers(0, 2**32))))
    return scenes.from_quads(quads, W, H, name=f"stack{nq}")


@pytest.mark.parametrize("bh", [8, 4])
@pytest.mark.parametrize("nq", [1500, 9000])
def test_dense_block_paths(lr, nq, bh):
    sc = stacked_block_scene(nq)
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    ctx = ctx_for(lr, block_h=bh)
    got = gpu_render(lr, ctx, sc)
    check_frame(got, ref, f"stack {nq}")
    st = ctx.stats()
    assert st["dense_blocks"] >= 1
    assert st["fragments"] == ref["total"]


def test_repeat_is_deterministic(lr):
    sc = SCENES["gauss"]()
    ctx = ctx_for(lr)
    h = ctx.upload(sc.v, sc.rgba)
    a = ctx.render_debug(h, sc.camera, sc.width, sc.height)
    b = ctx.render_debug(h, sc.camera, sc.width, sc.height)
    ctx.release(h)
    for k in ("rgba8", "rgba_f32", "count", "flagged"):
        assert bool((a[k] == b[k]).all()), k


def test_stats_match_oracle(lr):
    sc = SCENES["small"]()
    ctx = ctx_for(lr)
    h = ctx.upload(sc.v, sc.rgba)
    ctx.render(h, sc.camera, sc.width, sc.height)
    st = ctx.stats()
    ctx.release(h)
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, want_order=False)
    cc = ref["setup"].cull_counts()
    assert st["visible"] == cc["visible"]
    assert st["culled"][1:7] == [cc["near"], cc["guard"], cc["degenerate"], cc["no_sample"], cc["edge_on"],
                                 cc["backface"]]
    assert st["fragments"] == ref["total"]
    counts, _, _ = oracle.bins(ref["setup"], sc.width, sc.height, 32)
    assert st["bin_pairs"] == int(counts.sum())


def test_render_batch_matches_single(lr):
    import torch
    ctx = ctx_for(lr)
    frames = [scenes.small(64 + 8 * i, 40 + 4 * i, 500 + 300 * i, 30 + i, side=(2, 16)) for i in range(4)]
    hs = [ctx.upload(s.v, s.rgba) for s in frames]
    outs = [ctx.new_image(s.width, s.height) for s in frames]
    ctx.render_batch([(h, s.camera, s.width, s.height, o, 0, 0) for h, s, o in zip(hs, frames, outs)])
    for h, s, o in zip(hs, frames, outs):
        single = ctx.render(h, s.camera, s.width, s.height)
        assert bool((single == o).all())
    for h in hs:
        ctx.release(h)


def test_c2_full_frame(lr):
    sc = scenes.scene("c2")
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    got = gpu_render(lr, ctx_for(lr), sc)
    check_frame(got, ref, "c2")


def rule_tuning(sc):
    """(bin, sorter depth, block height) the library's rule table picks."""
    from paper_2405_13364_amd import autotune
    return tuple(autotune.resolve(autotune.load_rules(), sc.width, sc.height, sc.n))


_c3_ref = {}


def c3_reference():
    if "ref" not in _c3_ref:
        sc = scenes.scene("c3")
        _c3_ref["sc"] = sc
        _c3_ref["ref"] = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    return _c3_ref["sc"], _c3_ref["ref"]


@pytest.mark.parametrize("tune", ["rules", (16, 8, 8), (32, 8, 4)])
def test_c3_full_frame(lr, tune):
    """The whole 1920x1080 frame of 1M quads (106 M fragments, up to ~300 per
    pixel at the centre): every pixel's count, blend order and colour, at the
    tuning the rule table picks for it (the one the benchmark times) and at
    two others."""
    sc, ref = c3_reference()
    b, k, bh = rule_tuning(sc) if tune == "rules" else tune
    ctx = lr.Context(arena_bytes=1 << 30, bin_size=b, sorter_depth=k, block_h=bh)
    got = gpu_render(lr, ctx, sc, order=True)
    assert int(got["flagged"].sum().item()) > 0  # the exact pass took part
    check_frame(got, ref, f"c3 bin {b} K {k} 8x{bh}")
    ctx.close()


def test_c3_production_kernels(lr):
    """The same frame through lr_render (no parity dumps: the kernels the
    benchmark times) at the rule-table tuning: RGBA8 on every pixel and the
    fragment statistics against the oracle."""
    from paper_2405_13364_amd import autotune
    sc, ref = c3_reference()
    ctx = lr.Context(arena_bytes=1 << 30, tuning=autotune.load_rules())
    h = ctx.upload(sc.v, sc.rgba)
    img = ctx.render(h, sc.camera, sc.width, sc.height)
    st = ctx.stats()
    d8 = np.abs(img.cpu().numpy().astype(np.int32) - ref["rgba8"].astype(np.int32))
    assert d8.max() <= 1
    assert st["fragments"] == ref["total"]
    assert st["visible"] == ref["setup"].cull_counts()["visible"]
    assert st["flagged_pixels"] > 0 and st["error_word"] == 0
    ctx.close()


def test_c2b_full_frame(lr):
    sc = scenes.scene("c2b")
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    ctx = lr.Context(arena_bytes=1 << 30, bin_size=32, sorter_depth=8)
    got = gpu_render(lr, ctx, sc)
    check_frame(got, ref, "c2b")
    ctx.close()


def test_equal_depth_stack_takes_the_exact_pass(lr):
    """1,200 quads at one depth over the same 16x16 pixels: every block holds
    more equal-key entries than one on-chip sort, so no depth slice fits and
    the blocks' pixels go to the exact per-pixel sort.  Order is by quad
    index alone."""
    W, H = 48, 40
    rng = np.random.default_rng(77)
    quads = []
    for q in range(1200):
        rgb = rng.integers(0, 256, 3)
        rgba = int(scenes.pack_rgba(int(rgb[0]), int(rgb[1]), int(rgb[2]), int(rng.integers(5, 60))))
        quads.append((scenes.screen_quad([(8.1, 8.1), (23.9, 8.1), (23.9, 23.9), (8.1, 23.9)], 4.0, W, H), rgba))
    sc = scenes.from_quads(quads, W, H, name="equal_depth_stack")
    ref = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    assert int(ref["count"].max()) == 1200
    for k, bh in [(8, 8), (32, 4)]:
        ctx = lr.Context(arena_bytes=256 << 20, bin_size=32, sorter_depth=k, block_h=bh)
        h = ctx.upload(sc.v, sc.rgba)
        got = ctx.render_debug(h, sc.camera, W, H, order=True)
        st = ctx.stats()
        check_frame(got, ref, f"equal-depth stack K {k} 8x{bh}")
        assert st["error_word"] & lr.LR_FRAME_ERR_DENSE
        assert st["dense_blocks"] >= 4 and st["flagged_pixels"] == 256
        ctx.close()


@pytest.mark.parametrize("k", [8, 12])
@pytest.mark.parametrize("name", ["gauss", "c1", "twisted"])
def test_sixteen_wave_raster_without_dumps(lr, name, k):
    """Bin 64 at sorter depth 8 or 12 runs the raster with 16 waves per
    workgroup, a configuration the parity dumps (which keep 8 waves past
    depth 4) never take: RGBA8 and fragment statistics against the oracle."""
    sc = SCENES[name]()
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, want_order=False)
    ctx = lr.Context(arena_bytes=256 << 20, bin_size=64, sorter_depth=k)
    h = ctx.upload(sc.v, sc.rgba)
    img = ctx.render(h, sc.camera, sc.width, sc.height)
    st = ctx.stats()
    d8 = np.abs(img.cpu().numpy().astype(np.int32) - ref["rgba8"].astype(np.int32))
    assert d8.max(initial=0) <= 1
    assert st["fragments"] == ref["total"]
    ctx.close()


def test_upload_from_device_memory(lr):
    """lr_upload_scene from a device buffer of packed 52-byte quads gives the
    same image as the host upload; the buffer may be freed on return."""
    import torch
    sc = SCENES["gauss"]()
    ctx = ctx_for(lr)
    dev = torch.from_numpy(sc.quad_records().view(np.uint8).reshape(-1).copy()).cuda()
    h_dev = ctx.upload_device(dev)
    del dev
    torch.cuda.empty_cache()
    junk = torch.full((sc.n * 52,), 0xAB, dtype=torch.uint8, device="cuda")  # reuses the freed memory
    h_host = ctx.upload(sc.v, sc.rgba)
    a = ctx.render(h_dev, sc.camera, sc.width, sc.height).cpu().numpy()
    b = ctx.render(h_host, sc.camera, sc.width, sc.height).cpu().numpy()
    np.testing.assert_array_equal(a, b)
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, want_order=False)
    assert np.abs(a.astype(np.int32) - ref["rgba8"].astype(np.int32)).max() <= 1
    del junk
    ctx.release(h_dev)
    ctx.release(h_host)


def test_c3_sampled_pixels(lr):
    """Full-size dense cloud: the oracle computes sampled pixels one by one
    (the densest centre region plus random pixels)."""
    sc = scenes.scene("c3")
    ctx = ctx_for(lr, arena=1 << 30)
    got = gpu_render(lr, ctx, sc, order=True)
    W, H = sc.width, sc.height
    rng = np.random.default_rng(0)
    cy, cx = H // 2, W // 2
    centre = [(cy + dy) * W + (cx + dx) for dy in range(-4, 4) for dx in range(-4, 4)]
    pix = np.array(centre + list(rng.choice(W * H, 192, replace=False)), np.uint32)
    ref = oracle.pixels(sc.v, sc.rgba, sc.camera, W, H, pix)
    cnt = got["count"].cpu().numpy().reshape(-1)[pix].astype(np.uint32)
    np.testing.assert_array_equal(cnt, ref["count"])
    f32 = got["rgba_f32"].cpu().numpy().reshape(-1, 4)[pix].astype(np.float64)
    assert np.abs(f32 - ref["rgba_f64"]).max() <= F32_TOL
    r8 = got["rgba8"].cpu().numpy().reshape(-1, 4)[pix].astype(np.int32)
    assert np.abs(r8 - oracle.to_u8(ref["rgba_f64"]).astype(np.int32)).max() <= 1
    off = got["order_offsets"].cpu().numpy()
    ids = got["order_ids"].cpu().numpy().astype(np.uint32)
    for k, p in enumerate(pix):
        a = ids[int(off[p]):int(off[p + 1])]
        b = ref["ids"][int(ref["offsets"][k]):int(ref["offsets"][k + 1])]
        np.testing.assert_array_equal(a, b)
    assert int(ref["count"].max()) > 200  # the sampled centre is the deep part


@pytest.mark.parametrize("b,k,bh", [(16, 8, 8), (32, 12, 4), (64, 16, 8), (16, 4, 8)])
def test_density_classes_do_not_change_the_image(lr, b, k, bh):
    """Density classes (dense bins first, sparse ones with a depth-4 sorter,
    one launch) against one class in screen order: fp32 colour and counts
    bit-identical, and both against the oracle."""
    sc = scenes.small(200, 150, 40000, 16, side=(1.0, 20.0), gaussian=True, alpha=(0.05, 0.5))
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    outs = []
    for classes in (True, False):
        ctx = lr.Context(arena_bytes=512 << 20, bin_size=b, sorter_depth=k, block_h=bh, density_classes=classes)
        got = gpu_render(lr, ctx, sc)
        check_frame(got, ref, f"bin {b} K {k} classes {classes}")
        outs.append((got["rgba_f32"].cpu().numpy(), got["count"].cpu().numpy()))
        ctx.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


def test_density_classes_in_a_batch(lr):
    """Batched frames with density classes (graph replay included) equal the
    single renders, and the oracle."""
    import torch
    frames = [scenes.small(200, 150, 40000, 17, side=(1.0, 20.0), gaussian=True, alpha=(0.05, 0.5)),
              scenes.small(160, 120, 8000, 18, side=(2.0, 12.0)),
              scenes.small(256, 256, 60000, 19, side=(1.0, 16.0), gaussian=True, alpha=(0.1, 0.6))]
    ctx = lr.Context(arena_bytes=1 << 30, density_classes=True)
    hs = [ctx.upload(s.v, s.rgba) for s in frames]
    outs = [ctx.new_image(s.width, s.height) for s in frames]
    reqs = [(h, s.camera, s.width, s.height, o, b, k, 8) for h, s, o, (b, k) in
            zip(hs, frames, outs, [(16, 8), (32, 12), (32, 8)])]
    ctx.render_batch(reqs)
    ctx.render_batch(reqs)
    for h, s, o, r in zip(hs, frames, outs, reqs):
        c2 = lr.Context(arena_bytes=256 << 20, bin_size=r[5], sorter_depth=r[6], density_classes=True)
        single = c2.render(c2.upload(s.v, s.rgba), s.camera, s.width, s.height)
        assert torch.equal(single, o)
        c2.close()
        ref = oracle.render(s.v, s.rgba, s.camera, s.width, s.height, want_order=False)
        assert np.abs(o.cpu().numpy().astype(np.int32) - ref["rgba8"].astype(np.int32)).max() <= 1
    ctx.close()


@pytest.mark.parametrize("b", [16, 32, 64])
def test_large_quad_binning_keeps_the_image(lr, b):
    """The trivial reject of large quads' bins drops bin pairs but no
    fragment: the same image, counts and order as bbox binning, and the
    oracle's."""
    sc = thin_large(480, 360, 400, 52)
    ref = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    res = {}
    for bbox in (False, True):
        ctx = lr.Context(arena_bytes=512 << 20, bin_size=b, sorter_depth=8, bbox_binning=bbox)
        got = gpu_render(lr, ctx, sc)
        check_frame(got, ref, f"bin {b} bbox {bbox}")
        h = ctx.upload(sc.v, sc.rgba)
        ctx.render(h, sc.camera, sc.width, sc.height)
        res[bbox] = (ctx.stats()["bin_pairs"], got["rgba_f32"].cpu().numpy())
        ctx.close()
    assert res[False][0] < res[True][0]
    np.testing.assert_array_equal(res[False][1], res[True][1])


@pytest.mark.parametrize("name", ["small", "c1", "general", "twisted"])
def test_backface_culling(lr, name):
    """LR_FLAG_CULL_BACKFACES: setup culls exactly the quads the oracle culls
    as back-facing (bit-exact records for the rest), and the frame matches
    the oracle's with the same culling: counts, order, colour, statistics."""
    sc = SCENES[name]()
    cam = moved_camera()
    st = oracle.setup(sc.v, cam, sc.width, sc.height, cull_backfaces=True)
    assert np.count_nonzero(st.cull == 6) > 0
    ctx = lr.Context(arena_bytes=256 << 20, cull_backfaces=True)
    h = ctx.upload(sc.v, sc.rgba)
    got = ctx.debug_setup(h, cam, sc.width, sc.height, sc.n)
    np.testing.assert_array_equal(got["cull"], st.cull)
    vis = st.cull == 0
    np.testing.assert_array_equal(got["bbox"][vis], st.bbox[vis])
    ref = oracle.render(sc.v, sc.rgba, cam, sc.width, sc.height, st=st)
    check_frame(ctx.render_debug(h, cam, sc.width, sc.height, order=True), ref, f"{name} culled")
    ctx.render(h, cam, sc.width, sc.height)
    stats = ctx.stats()
    assert stats["culled"][6] == int(np.count_nonzero(st.cull == 6))
    assert stats["fragments"] == ref["total"]
    ctx.close()
