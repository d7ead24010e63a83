"""Pins of the oracle's transmittance cutoff (the tolerance-safe form of the
alpha threshold of Stage 3, "Sample blending"): a pixel stops after the
first fragment that brings its transmittance below 2^-20.

Closed forms: n identical layers of alpha a leave T = (1 - a)^n, so the
pixel stops after the smallest n with (1 - a)^n < 2^-20, and its colour is
c (1 - (1 - a)^n), alpha 1 - (1 - a)^n.  The stacks below are chosen so
that (1 - a)^n lies at least 5% away from 2^-20 for every n, so single
precision cannot move the decision.  Invariants: the cut order is a prefix
of the full order, and the colour moves by less than 2^-20 per channel."""
import math

import numpy as np
import pytest

import oracle
from paper_2405_13364_amd import scenes

CUT = 2.0 ** -20
W, H = 24, 20


def stack(alphas, rgb=(200, 120, 40), rect=((4.5, 3.5), (14.5, 3.5), (14.5, 11.5), (4.5, 11.5))):
    """Fronto-parallel quads over one rectangle, quad q at depth 1 + 0.1 q
    (quad 0 nearest)."""
    quads = []
    for q, a in enumerate(alphas):
        quads.append((scenes.screen_quad(list(rect), 1.0 + 0.1 * q, W, H),
                      int(scenes.pack_rgba(rgb[0], rgb[1], rgb[2], a))))
    return scenes.from_quads(quads, W, H, name="stack")


def stop_index(alphas):
    """Layers blended: the first n with prod(1 - a_i) < 2^-20 (real
    arithmetic), checked to be at least 5% away from the threshold."""
    T = 1.0
    for n, a8 in enumerate(alphas, 1):
        T *= 1.0 - a8 / 255.0
        assert abs(T / CUT - 1.0) > 0.05, "stack too close to the threshold for a closed form"
        if T < CUT:
            return n, T
    return len(alphas), T


@pytest.mark.parametrize("a8,expect", [(128, 20), (200, 10), (60, 52), (255, 1)])
def test_identical_layers_stop_at_the_closed_form(a8, expect):
    alphas = [a8] * 60
    n, T = stop_index(alphas)
    assert n == expect
    sc = stack(alphas)
    full = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    cut = oracle.render(sc.v, sc.rgba, sc.camera, W, H, cutoff=True)
    covered = full["count"] > 0
    assert int(covered.sum()) == 10 * 8
    assert np.all(full["count"][covered] == 60)
    assert np.all(cut["count"][covered] == n)
    assert np.all(cut["count"][~covered] == 0)
    assert cut["total"] == 80 * n and cut["covering"] == 80 * 60
    # nearest first: quads 0 .. n-1
    for p in np.flatnonzero(covered.reshape(-1)):
        ids = cut["order_ids"][int(cut["order_offsets"][p]):int(cut["order_offsets"][p + 1])]
        assert list(ids) == list(range(n))
    c = np.array([200, 120, 40]) / 255.0
    keep = (1.0 - a8 / 255.0) ** n
    got = cut["rgba_f64"][covered]
    np.testing.assert_allclose(got[:, :3], np.broadcast_to(c * (1.0 - keep), (80, 3)), rtol=0, atol=1e-12)
    np.testing.assert_allclose(got[:, 3], 1.0 - keep, rtol=0, atol=1e-12)


def test_mixed_alphas_stop_at_the_closed_form():
    rng = np.random.default_rng(5)
    alphas = [int(x) for x in rng.integers(40, 230, 80)]
    n, T = stop_index(alphas)
    assert 5 < n < 80
    sc = stack(alphas)
    cut = oracle.render(sc.v, sc.rgba, sc.camera, W, H, cutoff=True)
    covered = cut["count"] > 0
    assert np.all(cut["count"][covered] == n)
    np.testing.assert_allclose(cut["rgba_f64"][covered][:, 3], 1.0 - T, rtol=0, atol=1e-12)


def test_shallow_pixels_are_unchanged():
    """Alpha at most 0.2 over at most a few dozen layers never gets below
    2^-20: the cut render is the full one."""
    sc = scenes.small(64, 48, 600, 7, side=(2.0, 14.0), alpha=(0.02, 0.2))
    full = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    assert int(full["count"].max()) < math.log(CUT) / math.log(1.0 - 51 / 255.0)
    cut = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, cutoff=True)
    np.testing.assert_array_equal(cut["count"], full["count"])
    np.testing.assert_array_equal(cut["order_ids"], full["order_ids"])
    np.testing.assert_array_equal(cut["rgba_f64"], full["rgba_f64"])


@pytest.mark.parametrize("seed,alpha", [(11, (0.8, 1.0)), (12, (0.3, 0.9))])
def test_cut_is_a_prefix_within_the_residual(seed, alpha):
    sc = scenes.small(80, 60, 6000, seed, side=(2.0, 20.0), alpha=alpha, gaussian=True)
    full = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height)
    cut = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, cutoff=True)
    assert cut["total"] < full["total"]  # the scene is deep enough to stop somewhere
    assert np.all(cut["count"] <= full["count"])
    fo, co = full["order_offsets"], cut["order_offsets"]
    for p in range(sc.width * sc.height):
        a = full["order_ids"][int(fo[p]):int(fo[p]) + int(cut["count"].reshape(-1)[p])]
        b = cut["order_ids"][int(co[p]):int(co[p + 1])]
        assert np.array_equal(a, b)
    # the left-out fragments carry less than the stopping transmittance
    assert np.abs(cut["rgba_f64"] - full["rgba_f64"]).max() < CUT * (1.0 + 1e-3)
    stopped = cut["count"] < full["count"]
    assert np.all(cut["rgba_f64"][..., 3][stopped] > 1.0 - CUT * (1.0 + 1e-3))


def test_selected_pixels_match_the_frame():
    sc = scenes.small(80, 60, 6000, 11, side=(2.0, 20.0), alpha=(0.8, 1.0), gaussian=True)
    cut = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, cutoff=True)
    pix = np.array([0, 1234, 2400, 30 * 80 + 40, 4799], np.uint32)
    sel = oracle.pixels(sc.v, sc.rgba, sc.camera, sc.width, sc.height, pix, cutoff=True)
    np.testing.assert_array_equal(sel["count"], cut["count"].reshape(-1)[pix])
    np.testing.assert_array_equal(sel["rgba_f64"], cut["rgba_f64"].reshape(-1, 4)[pix])
    for k, p in enumerate(pix):
        np.testing.assert_array_equal(sel["ids"][int(sel["offsets"][k]):int(sel["offsets"][k + 1])],
                                      cut["order_ids"][int(cut["order_offsets"][p]):int(cut["order_offsets"][p + 1])])
