"""Oracle invariants: watertightness, order independence, closed-form depth,
cull rules that need exact arithmetic, unsorted blend, binning."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2405_13364_amd import scenes


def test_watertight_mesh():
    """A quad mesh whose interior vertices are shared covers every sample in
    its (axis-aligned, on-centre) outline exactly once."""
    W = H = 32
    rng = np.random.default_rng(3)
    nx, ny = 5, 4
    x0, y0, step = 3.5, 4.5, 5.0
    gx = np.zeros((ny + 1, nx + 1))
    gy = np.zeros((ny + 1, nx + 1))
    gz = rng.uniform(1.0, 3.0, (ny + 1, nx + 1))
    for b in range(ny + 1):
        for a in range(nx + 1):
            jx = rng.uniform(-1.7, 1.7) if 0 < a < nx else 0.0
            jy = rng.uniform(-1.7, 1.7) if 0 < b < ny else 0.0
            gx[b, a] = x0 + a * step + jx
            gy[b, a] = y0 + b * step + jy
    cam = scenes.Camera()
    f = scenes.focal_pixels(H, cam.fov_y)
    verts = {}
    for b in range(ny + 1):
        for a in range(nx + 1):
            z = gz[b, a]
            verts[(a, b)] = np.array([(gx[b, a] - W / 2) * z / f, -(gy[b, a] - H / 2) * z / f, z],
                                     np.float32)
    quads = []
    for b in range(ny):
        for a in range(nx):
            v = np.stack([verts[(a, b)], verts[(a + 1, b)], verts[(a + 1, b + 1)], verts[(a, b + 1)]])
            quads.append((v, int(scenes.pack_rgba(100, 100, 100, 100))))
    sc = scenes.from_quads(quads, W, H)
    res = oracle.render(sc.v, sc.rgba, sc.camera, W, H, want_order=False)
    cnt = res["count"]
    # outline: x in [3.5, 28.5], y in [4.5, 24.5] on pixel centres -> i 3..27, j 4..23
    expect = np.zeros((H, W), np.uint32)
    expect[4:24, 3:28] = 1
    np.testing.assert_array_equal(cnt, expect)


@pytest.mark.parametrize("seed", range(3))
def test_permutation_invariance(seed):
    sc = scenes.small(64, 48, 300, seed, side=(3, 20))
    base = oracle.render(sc.v, sc.rgba, sc.camera, 64, 48)
    st = base["setup"]
    perm = np.random.default_rng(seed + 10).permutation(sc.n)
    res = oracle.render(sc.v[perm], sc.rgba[perm], sc.camera, 64, 48)
    np.testing.assert_array_equal(res["count"], base["count"])
    # blend order is fixed by the keys alone unless two covering fragments tie
    off, ids = base["order_offsets"], base["order_ids"]
    tie = np.zeros((48, 64), bool)
    for p in range(64 * 48):
        i, j = p % 64, p // 64
        ks = [float(oracle.key(st, int(q), i, j)) for q in ids[int(off[p]):int(off[p + 1])]]
        tie[j, i] = len(ks) != len(set(ks))
    same = ~tie
    np.testing.assert_array_equal(res["rgba_f64"][same], base["rgba_f64"][same])
    # ids map through the permutation
    off2, ids2 = res["order_offsets"], res["order_ids"]
    for p in np.flatnonzero(same.reshape(-1))[:500]:
        a = [int(q) for q in ids[int(off[p]):int(off[p + 1])]]
        b = [int(perm[q]) for q in ids2[int(off2[p]):int(off2[p + 1])]]
        assert a == b


@pytest.mark.parametrize("Z", [1.0, 1.5, 2.0, 3.0, 7.25, 9.99, 1e-1 + 1e-3, 100.0, 12345.0])
def test_fronto_parallel_key(Z):
    W = H = 16
    q = scenes.screen_quad([[2.3, 2.2], [12.7, 2.9], [13.1, 12.2], [1.9, 13.4]], Z, W, H)
    sc = scenes.from_quads([(q, 0xff00ff00)], W, H)
    st = oracle.setup(sc.v, sc.camera, W, H)
    assert st.cull[0] == 0
    z32 = np.float32(Z)
    assert st.A[0] == 0.0 and st.B[0] == 0.0
    want = np.float32(1.0 / float(z32))
    for (i, j) in [(5, 5), (8, 9), (11, 3)]:
        k = oracle.key(st, 0, i, j)
        assert abs(float(k) - float(want)) <= float(np.spacing(want))


def test_random_keys_within_two_ulp():
    """Reciprocal depth keys of tilted quads against the exact ray/plane value."""
    W, H = 48, 40
    sc = scenes.small(W, H, 60, 5, side=(4, 24))
    st = oracle.setup(sc.v, sc.camera, W, H)
    res = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    cs = brute.camera_space(sc.v, sc.camera.as_record())
    f = Fraction(st.f)
    off, ids = res["order_offsets"], res["order_ids"]
    rng = np.random.default_rng(1)
    checked = 0
    for p in rng.choice(W * H, 300, replace=False):
        i, j = int(p % W), int(p // W)
        for q in ids[int(off[p]):int(off[p + 1])]:
            k = float(oracle.key(st, int(q), i, j))
            d = brute.inv_depth(cs[int(q)], f, Fraction(W, 2), Fraction(H, 2), i, j)
            if d is not None and d > 0 and k > 0:
                assert abs(k - float(d)) <= 2 * float(np.spacing(np.float32(k)))
                checked += 1
    assert checked > 100


def test_edge_on_plane_through_eye():
    """A quad whose plane contains the eye projects to a line; snapping can
    leave it with a non-zero triangle, which the depth-plane test then culls."""
    W = H = 16
    # all four vertices satisfy z = x + 2y: the plane passes through the origin
    v = np.array([[[1, 1, 3], [3, 1, 5], [3, 2, 7], [1, 3, 7]]], np.float32)
    sc = scenes.from_quads([(v[0], 0xffffffff)], W, H)
    st = oracle.setup(sc.v, sc.camera, W, H)
    X, Y, in_front, _ = brute.snap_quads(sc.v, sc.camera.as_record(), W, H, st.f)
    P = [(int(X[0, k]), int(Y[0, k])) for k in range(4)]
    area0 = (P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[1][1] - P[0][1]) * (P[2][0] - P[0][0])
    area1 = (P[2][0] - P[0][0]) * (P[3][1] - P[0][1]) - (P[2][1] - P[0][1]) * (P[3][0] - P[0][0])
    if area0 == 0 and area1 == 0:
        assert oracle.CULL_NAMES[st.cull[0]] == "degenerate"
    else:
        assert oracle.CULL_NAMES[st.cull[0]] in ("edge_on", "no_sample")


def test_unsorted_over_closed_form():
    W = H = 16
    c0, c1 = (255, 0, 0, 128), (0, 0, 255, 64)
    r = [[2.5, 2.5], [6.5, 2.5], [6.5, 5.5], [2.5, 5.5]]
    sc = scenes.from_quads([(scenes.screen_quad(r, 2.0, W, H), int(scenes.pack_rgba(*c0))),
                            (scenes.screen_quad(r, 4.0, W, H), int(scenes.pack_rgba(*c1)))], W, H)
    res = oracle.render(sc.v, sc.rgba, sc.camera, W, H, unsorted=True)
    a0, a1 = 128 / 255, 64 / 255
    col0, col1 = np.array([1.0, 0, 0]), np.array([0, 0, 1.0])
    rgb = a1 * col1 + (1 - a1) * (a0 * col0)
    al = a1 + (1 - a1) * a0
    np.testing.assert_allclose(res["rgba_f64"][3, 3], np.append(rgb, al), atol=1e-15)
    # ids in quad order
    p = 3 * W + 3
    assert list(res["order_ids"][int(res["order_offsets"][p]):int(res["order_offsets"][p + 1])]) == [0, 1]


@pytest.mark.parametrize("bs", [16, 32, 64])
def test_bins_are_bbox_overlaps(bs):
    W, H = 200, 120
    sc = scenes.small(W, H, 500, 9, side=(2, 40))
    st = oracle.setup(sc.v, sc.camera, W, H)
    counts, off, ids = oracle.bins(st, W, H, bs)
    nbx = (W + bs - 1) // bs
    for b in range(counts.size):
        bx, by = b % nbx, b // nbx
        want = [q for q in range(sc.n) if st.cull[q] == 0 and
                st.bbox[q, 0] <= bx * bs + bs - 1 and st.bbox[q, 1] >= bx * bs and
                st.bbox[q, 2] <= by * bs + bs - 1 and st.bbox[q, 3] >= by * bs]
        assert [int(x) for x in ids[int(off[b]):int(off[b + 1])]] == want


def test_pixels_agree_with_frame():
    W, H = 64, 48
    sc = scenes.small(W, H, 400, 4, side=(3, 25))
    res = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    pix = np.random.default_rng(0).choice(W * H, 200, replace=False).astype(np.uint32)
    for uns in (False, True):
        full = oracle.render(sc.v, sc.rgba, sc.camera, W, H, unsorted=uns)
        pr = oracle.pixels(sc.v, sc.rgba, sc.camera, W, H, pix, unsorted=uns)
        np.testing.assert_array_equal(pr["count"], full["count"].reshape(-1)[pix])
        np.testing.assert_array_equal(pr["rgba_f64"], full["rgba_f64"].reshape(-1, 4)[pix])
        for k, p in enumerate(pix):
            a = full["order_ids"][int(full["order_offsets"][p]):int(full["order_offsets"][p + 1])]
            b = pr["ids"][int(pr["offsets"][k]):int(pr["offsets"][k + 1])]
            np.testing.assert_array_equal(a, b)
