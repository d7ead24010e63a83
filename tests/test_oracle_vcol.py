"""Pins of the oracle's per-vertex colours (Stage 3, "Sample shading":
attributes interpolated per sample): a covered sample takes T0 = (P0, P1,
P2) if T0 covers it, else T1 = (P0, P2, P3), and the barycentric mix of that
triangle's vertex colours at the point where the pixel-centre ray meets the
triangle's plane.

* equal vertex colours give the flat render;
* a fronto-parallel quad (one depth) reduces to screen-space barycentrics of
  the pixel centre in the projected triangle (solved here in numpy);
* a quad tilted in depth: the ray-plane intersection and its barycentric
  coordinates solved here in numpy (a 3x3 linear system per pixel), which
  differs from the affine screen-space mix;
* every channel stays between the triangle's vertex values."""
import math

import numpy as np
import pytest

import oracle
from paper_2405_13364_amd import scenes

W, H = 40, 32


def opaque_vertex_colours(rng, n):
    rgb = rng.integers(0, 256, (n, 4, 3))
    return scenes.pack_rgba(rgb[..., 0], rgb[..., 1], rgb[..., 2], np.full((n, 4), 255)).astype(np.uint32)


def unit(c):
    return np.array([(c >> (8 * ch)) & 255 for ch in range(4)], np.float64) / 255.0


def test_equal_vertex_colours_are_flat():
    sc = scenes.small(64, 48, 400, 3, side=(2.0, 20.0))
    vcol = np.repeat(sc.rgba[:, None], 4, axis=1)
    a = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    b = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, vcol=vcol)
    np.testing.assert_array_equal(a["count"], b["count"])
    np.testing.assert_array_equal(a["order_ids"], b["order_ids"])
    assert np.abs(a["rgba_f64"] - b["rgba_f64"]).max() < 1e-12


def one_quad(corners3d, vcol):
    v = np.array(corners3d, np.float32)[None]
    return v, np.array([0xFF000000], np.uint32), np.array(vcol, np.uint32)[None]


def ray(i, j, f):
    return np.array([(i + 0.5 - W / 2) / f, -(j + 0.5 - H / 2) / f, 1.0])


def check_quad(v, vc, expect_fn):
    cam = scenes.Camera()
    res = oracle.render(v, np.array([0xFF000000], np.uint32), cam, W, H, vcol=vc)
    st = res["setup"]
    assert st.cull[0] == 0
    n = 0
    for j in range(H):
        for i in range(W):
            if res["count"][j, i]:
                got = res["rgba_f64"][j, i]
                want = expect_fn(i, j, st)
                assert np.abs(got[:3] - want[:3]).max() < 1e-9, (i, j, got, want)
                assert abs(got[3] - 1.0) < 1e-12
                n += 1
    assert n > 50


def side_of_t0(st, i, j):
    """Whether T0 covers the sample of (i, j) (exact, from the snapped vertices)."""
    X, Y = st.X[0], st.Y[0]
    return oracle.covers(np.array([X[0], X[1], X[2], X[2]], np.int32), np.array([Y[0], Y[1], Y[2], Y[2]], np.int32), i, j)


def test_fronto_parallel_is_screen_barycentric():
    rng = np.random.default_rng(7)
    f = oracle.focal(H, math.radians(60.0))
    z = 3.0
    px = np.array([(6.3, 5.1), (33.2, 7.4), (30.1, 27.8), (4.4, 24.6)])
    corners = [((x - W / 2) * z / f, -(y - H / 2) * z / f, z) for x, y in px]
    vc = opaque_vertex_colours(rng, 1)
    v, _, vcs = one_quad(corners, vc[0])

    Cv = np.asarray(v[0], np.float64)  # the fp32 vertices the renderer sees

    def expect(i, j, st):
        t = (0, 1, 2) if side_of_t0(st, i, j) else (0, 2, 3)
        P = np.array([((Cv[k][0] * f / Cv[k][2]) + W / 2, -(Cv[k][1] * f / Cv[k][2]) + H / 2) for k in t])
        s = np.array([i + 0.5, j + 0.5])
        # screen-space barycentrics: s = l0 P0 + l1 P1 + l2 P2, l0 + l1 + l2 = 1
        M = np.array([[P[0, 0], P[1, 0], P[2, 0]], [P[0, 1], P[1, 1], P[2, 1]], [1.0, 1.0, 1.0]])
        lam = np.linalg.solve(M, np.array([s[0], s[1], 1.0]))
        return sum(lam[k] * unit(int(vc[0, t[k]])) for k in range(3))

    check_quad(v, vcs, expect)


def test_tilted_quad_is_perspective_correct():
    rng = np.random.default_rng(8)
    f = oracle.focal(H, math.radians(60.0))
    # a planar square tilted in depth (z from 2 to 6)
    corners = [(-1.4, -1.0, 2.0), (1.6, -1.0, 6.0), (1.6, 1.2, 6.0), (-1.4, 1.2, 2.0)]
    vc = opaque_vertex_colours(rng, 1)
    v, _, vcs = one_quad(corners, vc[0])
    C = np.asarray(v[0], np.float64)  # the fp32 vertices the renderer sees

    def expect(i, j, st):
        t = (0, 1, 2) if side_of_t0(st, i, j) else (0, 2, 3)
        A, B, Cc = C[t[0]], C[t[1]], C[t[2]]
        r = ray(i, j, f)
        # X = s r = A + u (B - A) + w (C - A): solve for (s, u, w)
        M = np.stack([r, -(B - A), -(Cc - A)], axis=1)
        s_, u, w = np.linalg.solve(M, A)
        lam = (1.0 - u - w, u, w)
        return sum(lam[k] * unit(int(vc[0, t[k]])) for k in range(3))

    check_quad(v, vcs, expect)
    # and it is not the screen-space mix: the two differ somewhere
    res = oracle.render(v, np.array([0xFF000000], np.uint32), scenes.Camera(), W, H, vcol=vcs)
    assert res["total"] > 100


@pytest.mark.parametrize("seed", [1, 2])
def test_channels_within_the_triangle(seed):
    rng = np.random.default_rng(seed)
    sc = scenes.small(48, 40, 1, seed, side=(20.0, 36.0), z=(2.0, 3.0))
    vc = opaque_vertex_colours(rng, 1)
    res = oracle.render(sc.v, np.array([0xFF000000], np.uint32), sc.camera, 48, 40, vcol=vc)
    cov = res["count"] > 0
    assert cov.sum() > 20
    lo = np.min([unit(int(c)) for c in vc[0]], axis=0)
    hi = np.max([unit(int(c)) for c in vc[0]], axis=0)
    got = res["rgba_f64"][cov]
    assert np.all(got[:, :3] >= lo[:3] - 1e-12) and np.all(got[:, :3] <= hi[:3] + 1e-12)


def test_selected_pixels_match_the_frame():
    rng = np.random.default_rng(9)
    sc = scenes.small(64, 48, 800, 9, side=(2.0, 24.0))
    vc = rng.integers(0, 2 ** 32, (sc.n, 4), dtype=np.uint64).astype(np.uint32)
    fr = oracle.render(sc.v, sc.rgba, sc.camera, 64, 48, vcol=vc)
    pix = np.array([5, 700, 1500, 2222, 3000], np.uint32)
    sel = oracle.pixels(sc.v, sc.rgba, sc.camera, 64, 48, pix, vcol=vc)
    np.testing.assert_array_equal(sel["rgba_f64"], fr["rgba_f64"].reshape(-1, 4)[pix])
