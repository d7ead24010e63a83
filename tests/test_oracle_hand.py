"""Oracle against hand-derived scenes (tests/golden/hand_scenes.json)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2405_13364_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_scenes.json")
with open(GOLDEN) as fh:
    DATA = json.load(fh)
W, H = DATA["width"], DATA["height"]


def build(case):
    quads = []
    for q in case["quads"]:
        r, g, b, a = q["rgba"]
        quads.append((scenes.screen_quad(q["corners"], q["z"], W, H), int(scenes.pack_rgba(r, g, b, a))))
    return scenes.from_quads(quads, W, H)


def ids_at(res, i, j):
    p = j * W + i
    off = res["order_offsets"]
    return [int(x) for x in res["order_ids"][int(off[p]):int(off[p + 1])]]


@pytest.mark.parametrize("case", [c for c in DATA["cases"] if "covered" in c], ids=lambda c: c["name"])
def test_coverage(case):
    sc = build(case)
    res = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    for q, expected in enumerate(case["covered"]):
        got = set()
        for j in range(H):
            for i in range(W):
                if q in ids_at(res, i, j):
                    got.add((i, j))
        assert got == {tuple(p) for p in expected}, case["name"]
    assert res["setup"].cull_counts()["visible"] == len(case["quads"])


def _unit(rgba):
    return np.array(rgba[:3], np.float64) / 255.0, rgba[3] / 255.0


@pytest.mark.parametrize("case", [c for c in DATA["cases"] if "order_at" in c], ids=lambda c: c["name"])
def test_order_and_blend(case):
    sc = build(case)
    res = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    for (i, j), expected in case["order_at"]:
        assert ids_at(res, i, j) == expected
        got = res["rgba_f64"][j, i]
        layers = [_unit(case["quads"][q]["rgba"]) for q in expected]
        kind = case["closed_form"]
        if kind == "two":
            (c1, a1), (c2, a2) = layers
            rgb = a1 * c1 + (1 - a1) * a2 * c2
            alpha = 1 - (1 - a1) * (1 - a2)
        elif kind == "layers":
            c, a = layers[0]
            alpha = 1 - (1 - a) ** len(layers)
            rgb = c * alpha
        elif kind == "opaque_front":
            c, a = layers[0]
            assert a == 1.0
            rgb, alpha = c, 1.0
        np.testing.assert_allclose(got[:3], rgb, atol=1e-14, rtol=0)
        assert abs(got[3] - alpha) < 1e-14
        np.testing.assert_array_equal(res["rgba8"][j, i],
                                      np.clip(np.floor(255 * np.append(rgb, alpha) + 0.5), 0, 255))


def test_culls():
    case = [c for c in DATA["cases"] if c["name"] == "culls"][0]
    sc = build(case)
    st = oracle.setup(sc.v, sc.camera, W, H)
    names = [oracle.CULL_NAMES[c] for c in st.cull]
    assert names == case["cull"]
    res = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    assert res["total"] == 0
    assert not res["rgba_f64"].any()


def test_empty_scene():
    sc = scenes.from_quads([], W, H)
    res = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    assert res["total"] == 0 and not res["rgba8"].any()
