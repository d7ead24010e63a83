"""Oracle pins for the fragment key of non-planar quads and for the
row-band threading of whole-frame renders.

A quad whose corners do not lie in one plane gets the plane through its
vertex centroid normal to its diagonals (Stage 1, Phase 2 reads depth from
such a plane).  Over part of the quad's screen area that plane can lie behind
the camera, where the reciprocal depth it gives is negative; the key is then
clamped to +0 (the farthest possible key), and ties among such fragments are
broken by quad index.  The negative sign is established here in exact
rationals, independently of the oracle's floating point."""
from fractions import Fraction

import numpy as np

import oracle
from oracle import brute
from paper_2405_13364_amd import scenes

W = H = 32
# A twisted quad (corners at depths 1, 20, 60, 0.5): its fitted plane gives a
# negative reciprocal depth at pixel (18, 11), inside the quad.
TWIST = ([(15.985985465902477, 15.842401262928194), (20.17906270707796, 17.248386271955717),
          (17.196675698719094, 10.540218558927851), (25.097758661202043, 13.16218734339932)],
         [1.0, 20.0, 60.0, 0.5])
PIX = (18, 11)


def _scene():
    twist = scenes.screen_quad(TWIST[0], TWIST[1], W, H)
    front = scenes.screen_quad([(14.0, 8.0), (22.0, 8.0), (22.0, 14.0), (14.0, 14.0)], 5.0, W, H)
    quads = [(twist, int(scenes.pack_rgba(200, 40, 10, 90))),      # id 0
             (twist, int(scenes.pack_rgba(10, 220, 30, 60))),      # id 1: same geometry, equal key
             (front, int(scenes.pack_rgba(30, 60, 250, 120)))]     # id 2: planar, positive key
    return scenes.from_quads(quads, W, H)


def test_negative_plane_depth_clamps_to_zero_key():
    sc = _scene()
    cam = sc.camera.as_record()
    f = oracle.focal(H, float(cam["fov_y"]))
    cs = brute.camera_space(sc.v, cam)
    i, j = PIX
    exact = brute.inv_depth(cs[0], Fraction(f), Fraction(W, 2), Fraction(H, 2), i, j)
    assert exact is not None and exact < 0  # the fitted plane is behind the camera here
    res = oracle.render(sc.v, sc.rgba, sc.camera, W, H)
    st = res["setup"]
    assert list(st.cull) == [0, 0, 0]
    assert brute.covers(st.X[0], st.Y[0], i, j) and brute.covers(st.X[2], st.Y[2], i, j)
    k0 = oracle.key(st, 0, i, j)
    assert k0 == np.float32(0.0) and not np.signbit(k0)
    assert oracle.key(st, 2, i, j) > 0
    # the planar quad first, then the two zero keys by ascending index
    p = j * W + i
    off = res["order_offsets"]
    assert [int(x) for x in res["order_ids"][int(off[p]):int(off[p + 1])]] == [2, 0, 1]
    # colour: the three layers blended front to back in that order
    T, C = Fraction(1), [Fraction(0)] * 3
    for q in (2, 0, 1):
        c = int(sc.rgba[q])
        a = Fraction(c >> 24, 255)
        for ch in range(3):
            C[ch] += T * a * Fraction((c >> (8 * ch)) & 255, 255)
        T *= 1 - a
    want = [float(x) for x in C] + [float(1 - T)]
    np.testing.assert_allclose(res["rgba_f64"][j, i], want, rtol=0, atol=1e-15)


def test_twisted_frames_match_exact_order():
    """Every covered pixel of a frame of twisted quads: count and order
    against the brute force on the oracle's snapped corners, with a zero key
    wherever the exact plane depth is not positive."""
    sc = scenes.twisted(24, 20, 12, 4, extent=(3.0, 9.0))
    res = oracle.render(sc.v, sc.rgba, sc.camera, 24, 20)
    st = res["setup"]
    f = oracle.focal(20, sc.camera.fov_y)
    ref = brute.render(sc.v, sc.rgba, sc.camera.as_record(), 24, 20, f, st.X, st.Y, st.cull == 0)
    np.testing.assert_array_equal(res["count"], ref["count"])
    zero_seen = 0
    off = res["order_offsets"]
    for jj in range(20):
        for ii in range(24):
            p = jj * 24 + ii
            got = [int(x) for x in res["order_ids"][int(off[p]):int(off[p + 1])]]
            # exact order with non-positive depths mapped to key zero
            d = ref["inv_depth"][jj][ii]
            ids = ref["order"][jj][ii]
            want = sorted(zip(d, ids), key=lambda t: (-(t[0] if t[0] is not None and t[0] > 0 else 0), t[1]))
            zero_seen += sum(1 for x, _ in want if x is None or x <= 0)
            # fragments whose exact keys differ by less than fp32 resolution may
            # swap; compare only where neighbours are well separated
            sep = all(abs(float(a[0] or 0) - float(b[0] or 0)) > 1e-5 * max(abs(float(a[0] or 0)), 1e-30)
                      or ((a[0] is None or a[0] <= 0) and (b[0] is None or b[0] <= 0))
                      for a, b in zip(want, want[1:]))
            if sep:
                assert got == [q for _, q in want], (ii, jj)
    assert zero_seen > 0


def test_whole_frame_is_independent_of_threads():
    for sc in (scenes.scene("c1"), scenes.small(97, 61, 4000, 9, side=(1.0, 20.0), gaussian=True, alpha=(0.05, 0.6)),
               scenes.twisted(50, 33, 300, 5)):
        a = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, threads=1)
        b = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, threads=5)
        for k in ("rgba_f64", "rgba8", "count", "order_offsets", "order_ids"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)
        assert a["total"] == b["total"]
