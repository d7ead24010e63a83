"""Pins of the oracle's back-face culling (Stage 1 culls primitives facing
away from the camera; the convention, as OpenGL's default: front faces wind
counter-clockwise on the display).

* Hand scene: one rectangle whose corners are listed bottom-left,
  bottom-right, top-right, top-left (counter-clockwise on a display whose y
  points up) stays; the same corners in the opposite order are culled.
* Geometry: a fronto-parallel quad turned about its own vertical axis by an
  angle t faces the camera while |t| < 90 degrees (its normal's depth
  component is cos t).
* Independent formula: for planar quads, back-facing is exactly a negative
  signed area (shoelace) of the projected corners on the display, computed
  here in numpy from the camera and the vertices."""
import math

import numpy as np
import pytest

import oracle
from paper_2405_13364_amd import scenes

W, H = 32, 24
CCW = [(4.5, 14.5), (20.5, 14.5), (20.5, 4.5), (4.5, 4.5)]  # BL, BR, TR, TL in screen pixels (y down)


def scene_of(corner_lists, z=2.0):
    quads = [(scenes.screen_quad(c, z, W, H), int(scenes.pack_rgba(200, 100, 50, 128))) for c in corner_lists]
    return scenes.from_quads(quads, W, H)


def test_winding_decides():
    sc = scene_of([CCW, CCW[::-1]])
    st = oracle.setup(sc.v, sc.camera, W, H, cull_backfaces=True)
    assert list(st.cull) == [0, 6]
    st0 = oracle.setup(sc.v, sc.camera, W, H)
    assert list(st0.cull) == [0, 0]
    full = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    cut = oracle.render(sc.v, sc.rgba, sc.camera, W, H, cull_backfaces=True)
    assert int(full["count"].max()) == 2 and int(cut["count"].max()) == 1
    np.testing.assert_array_equal(cut["count"], (full["count"] > 0).astype(np.uint32))


@pytest.mark.parametrize("deg,back", [(0, False), (60, False), (80, False), (100, True), (150, True), (-120, True)])
def test_turned_quad(deg, back):
    t = math.radians(deg)
    # a 2 x 2 square at depth 5, turned about its own vertical axis
    loc = np.array([(-1, -1), (1, -1), (1, 1), (-1, 1)], np.float64)
    v = np.zeros((1, 4, 3), np.float32)
    for k, (x, y) in enumerate(loc):
        v[0, k] = (x * math.cos(t), y, 5.0 + x * math.sin(t))
    st = oracle.setup(v, scenes.Camera(), 64, 64, cull_backfaces=True)
    assert oracle.setup(v, scenes.Camera(), 64, 64).cull[0] == 0  # visible without the test
    assert (st.cull[0] == 6) == back


def projected_area(v, W, H, fov_y=math.radians(60.0)):
    f = (0.5 * H) / math.tan(0.5 * fov_y)
    x, y, z = v[..., 0].astype(np.float64), v[..., 1].astype(np.float64), v[..., 2].astype(np.float64)
    u, w = f * x / z, f * y / z  # display coordinates, y up
    return 0.5 * np.sum(u * np.roll(w, -1, axis=1) - np.roll(u, -1, axis=1) * w, axis=1)


@pytest.mark.parametrize("seed", [1, 2])
def test_matches_projected_winding(seed):
    sc = scenes.small(120, 90, 3000, seed, side=(3.0, 30.0))
    st = oracle.setup(sc.v, sc.camera, sc.width, sc.height, cull_backfaces=True)
    st0 = oracle.setup(sc.v, sc.camera, sc.width, sc.height)
    area = projected_area(sc.v, sc.width, sc.height)
    vis0 = st0.cull == 0
    clear = vis0 & (np.abs(area) > 1e-3)
    assert np.array_equal(st.cull[clear] == 6, area[clear] < 0)
    assert 0.3 < np.mean(area[clear] < 0) < 0.7  # random orientations: about half face away
    # culling only removes quads: the image equals that of the front-facing quads alone
    keep = st.cull == 0
    ref = oracle.render(sc.v[keep], sc.rgba[keep], sc.camera, sc.width, sc.height, want_order=False)
    got = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, want_order=False, cull_backfaces=True)
    np.testing.assert_array_equal(got["rgba_f64"], ref["rgba_f64"])
