"""Oracle against an exact-rational brute force on tiny frames.

The brute force derives coverage from a shifted-sample orientation test (no
fill rule written anywhere), depth from the exact ray/plane intersection and
the blend in Fractions, so a dropped term, a sign error or a swapped index in
the oracle shows up here."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2405_13364_amd import scenes

W = H = 16


def tiny_scene(seed, n=10, side=(2.0, 10.0)):
    return scenes.small(W, H, n, seed, side=side, z=(1.0, 10.0), alpha=(0.1, 0.9))


def ulp32(x):
    x = np.float32(abs(x))
    return float(np.spacing(x))


@pytest.mark.parametrize("seed", range(6))
def test_snap_matches_exact_projection(seed):
    sc = tiny_scene(seed)
    st = oracle.setup(sc.v, sc.camera, W, H)
    X, Y, in_front, near_tie = brute.snap_quads(sc.v, sc.camera.as_record(), W, H, st.f)
    checked = 0
    for q in range(sc.n):
        assert in_front[q] == (st.cull[q] != 1)
        if st.cull[q] in (1, 2) or q in near_tie:
            continue
        assert list(st.X[q]) == list(X[q]) and list(st.Y[q]) == list(Y[q]), q
        checked += 1
        if st.cull[q] == 0:
            # bbox: by enumeration, the on-screen sample columns/rows inside the vertex bounds
            cols = [i for i in range(W) if X[q].min() <= 256 * i + 128 <= X[q].max()]
            rows = [j for j in range(H) if Y[q].min() <= 256 * j + 128 <= Y[q].max()]
            assert list(st.bbox[q]) == [cols[0], cols[-1], rows[0], rows[-1]], q
    assert checked >= sc.n // 2


@pytest.mark.parametrize("seed", range(6))
def test_frame_matches_brute_force(seed):
    sc = tiny_scene(seed)
    res = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    st = res["setup"]
    ex = brute.render(sc.v, sc.rgba, sc.camera.as_record(), W, H, st.f, X=st.X, Y=st.Y,
                      visible=st.visible)
    np.testing.assert_array_equal(res["count"], ex["count"])
    off, ids = res["order_offsets"], res["order_ids"]
    cs = brute.camera_space(sc.v, sc.camera.as_record())
    f = Fraction(st.f)
    for j in range(H):
        for i in range(W):
            p = j * W + i
            got = [int(x) for x in ids[int(off[p]):int(off[p + 1])]]
            assert sorted(got) == sorted(ex["order"][j][i])
            # keys within 2 ulp of the exact reciprocal depth
            for q in got:
                k = oracle.key(st, q, i, j)
                d = brute.inv_depth(cs[q], f, Fraction(W, 2), Fraction(H, 2), i, j)
                if d is not None and d > 0 and k > 0:
                    assert abs(float(k) - float(d)) <= 2 * ulp32(k), (q, i, j)
            # order: no inversion beyond fp32 rounding of the exact depths
            for a, b in zip(got, got[1:]):
                da = brute.inv_depth(cs[a], f, Fraction(W, 2), Fraction(H, 2), i, j)
                db = brute.inv_depth(cs[b], f, Fraction(W, 2), Fraction(H, 2), i, j)
                assert float(da) >= float(db) - 4 * ulp32(db), (i, j, a, b)
            # colour: exact blend in the oracle's order
            T = Fraction(1)
            C = [Fraction(0)] * 3
            for q in got:
                c = int(sc.rgba[q])
                a = Fraction(c >> 24, 255)
                for ch in range(3):
                    C[ch] += T * a * Fraction((c >> (8 * ch)) & 255, 255)
                T *= 1 - a
            exact = [float(C[0]), float(C[1]), float(C[2]), float(1 - T)]
            np.testing.assert_allclose(res["rgba_f64"][j, i], exact, atol=1e-13, rtol=0)


def test_order_matches_exact_depth_when_separated():
    """With layers well separated in depth the oracle order is exactly the
    exact-depth order of the brute force."""
    quads = []
    rng = np.random.default_rng(7)
    for k in range(8):
        x0, y0 = rng.uniform(1, 7, 2)
        corners = [[x0, y0], [x0 + 7, y0 + 1], [x0 + 6, y0 + 7], [x0 - 1, y0 + 6]]
        quads.append((scenes.screen_quad(corners, 1.0 + k * 1.3, W, H), int(rng.integers(0, 2**32))))
    perm = rng.permutation(len(quads))
    sc = scenes.from_quads([quads[p] for p in perm], W, H)
    res = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    st = res["setup"]
    ex = brute.render(sc.v, sc.rgba, sc.camera.as_record(), W, H, st.f, X=st.X, Y=st.Y,
                      visible=st.visible)
    off, ids = res["order_offsets"], res["order_ids"]
    for j in range(H):
        for i in range(W):
            p = j * W + i
            assert [int(x) for x in ids[int(off[p]):int(off[p + 1])]] == ex["order"][j][i]
            exact = [float(x) for x in ex["rgba"][j][i]]
            np.testing.assert_allclose(res["rgba_f64"][j, i], exact, atol=1e-13, rtol=0)


@pytest.mark.parametrize("seed", range(4))
def test_fill_rule_equals_shifted_sample(seed):
    """Corners on the half-pixel lattice put many samples exactly on edges and
    vertices; the top-left rule must agree with the shifted-sample test."""
    rng = np.random.default_rng(100 + seed)
    for _ in range(60):
        X = (rng.integers(0, 9, 4) * 128).astype(np.int32)
        Y = (rng.integers(0, 9, 4) * 128).astype(np.int32)
        for j in range(5):
            for i in range(5):
                assert oracle.covers(X, Y, i, j) == brute.covers(X, Y, i, j), (X, Y, i, j)


@pytest.mark.parametrize("seed", range(3))
def test_moved_camera_matches_brute_force(seed):
    """A turned and moved camera: exercises every term of the camera
    transform (a transposed matrix or a dropped translation fails here)."""
    rng = np.random.default_rng(50 + seed)
    sc = tiny_scene(seed + 20, n=12, side=(3.0, 9.0))
    cam = scenes.Camera.jittered(float(rng.uniform(-4, 4)), float(rng.uniform(-4, 4)))
    cam.pos = tuple(float(x) for x in rng.uniform(-0.05, 0.05, 3))
    res = oracle.render(sc.v, sc.rgba, cam, W, H)
    st = res["setup"]
    X, Y, in_front, near_tie = brute.snap_quads(sc.v, cam.as_record(), W, H, st.f)
    for q in range(sc.n):
        if st.cull[q] in (1, 2) or q in near_tie:
            continue
        assert list(st.X[q]) == list(X[q]) and list(st.Y[q]) == list(Y[q]), q
    ex = brute.render(sc.v, sc.rgba, cam.as_record(), W, H, st.f, X=st.X, Y=st.Y,
                      visible=st.visible)
    np.testing.assert_array_equal(res["count"], ex["count"])
    cs = brute.camera_space(sc.v, cam.as_record())
    f = Fraction(st.f)
    off, ids = res["order_offsets"], res["order_ids"]
    for p in range(W * H):
        i, j = p % W, p // W
        for q in ids[int(off[p]):int(off[p + 1])]:
            k = float(oracle.key(st, int(q), i, j))
            d = brute.inv_depth(cs[int(q)], f, Fraction(W, 2), Fraction(H, 2), i, j)
            if d is not None and d > 0 and k > 0:
                assert abs(k - float(d)) <= 2 * ulp32(k)
