"""Plant plausible mistakes in a copy of the oracle and check that the pins
(hand scenes, brute force, invariants) catch every one of them."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lr_oracle.c")

MUTANTS = {
    "top_left_flipped": ("int top_left = (dy < 0) || (dy == 0 && dx > 0);",
                         "int top_left = (dy > 0) || (dy == 0 && dx < 0);"),
    "no_half_pixel_in_plane": ("double u0 = ((double)imin + 0.5) - cx;",
                               "double u0 = ((double)imin) - cx;"),
    "sign_of_B": ("double b = (-nn[1]) / g;", "double b = (nn[1]) / g;"),
    "key_axes_swapped": ("fma(a, (double)(i - bb[0]), fma(b, (double)(j - bb[2]), c0))",
                         "fma(a, (double)(j - bb[2]), fma(b, (double)(i - bb[0]), c0))"),
    "blend_drops_transmittance": ("C[ch] = C[ch] + w * ", "C[ch] = C[ch] + a * "),
    "order_back_to_front": ("return ((uint64_t)(~bits) << 32) | (uint64_t)id;",
                            "return ((uint64_t)(bits) << 32) | (uint64_t)id;"),
    "wrong_second_triangle": ("tri_covers(X, Y, 0, 2, 3, sx, sy)", "tri_covers(X, Y, 1, 2, 3, sx, sy)"),
    "bbox_max_rounded_up": ("imax = floordiv256(xmax - 128);", "imax = floordiv256(xmax - 128 + 255);"),
    "camera_transposed": ("c[k][r] = fma(R[3 * r + 2], d2, fma(R[3 * r + 1], d1, R[3 * r + 0] * d0));",
                          "c[k][r] = fma(R[3 * 2 + r], d2, fma(R[3 * 1 + r], d1, R[3 * 0 + r] * d0));"),
    "camera_no_translation": ("double d0 = (double)vk[0] - P[0]", "double d0 = (double)vk[0]"),
    "projection_y_up": ("sy[k] = fma(-f, qy, cy);", "sy[k] = fma(f, qy, cy);"),
    "diagonal_normal_sign": ("p = e1[0] * e2[1]; s = e1[1] * e2[0]; nn[2] = p - s;",
                             "p = e1[0] * e2[1]; s = e1[1] * e2[0]; nn[2] = s - p;"),
    "key_clamp_dropped": ("    if (!(k > 0.0f))\n        k = 0.0f;\n    return k;", "    return k;"),
    "cutoff_counts_before_blending": ("        k++;\n        if (T32 < LRO_CUT_T)\n            break;",
                                      "        if (T32 < LRO_CUT_T)\n            break;\n        k++;"),
    "cutoff_threshold_too_high": ("#define LRO_CUT_T (1.0f / 1048576.0f)", "#define LRO_CUT_T (1.0f / 65536.0f)"),
    "backface_sign_flipped": ("if (cull_back && dd < 0.0) {", "if (cull_back && dd > 0.0) {"),
    "vcol_wrong_triangle": ("    if (!tri_covers(vq->X, vq->Y, 0, 1, 2, sx, sy)) {", "    if (tri_covers(vq->X, vq->Y, 0, 1, 2, sx, sy)) {"),
    "vcol_weights_rotated": ("cross3(vq->cv + 3 * t[(k + 1) % 3], vq->cv + 3 * t[(k + 2) % 3], n);",
                             "cross3(vq->cv + 3 * t[(k + 2) % 3], vq->cv + 3 * t[k], n);"),
    "unsorted_under": ("C[ch] = a * col[k].c[ch] + (1.0 - a) * C[ch];",
                       "C[ch] = (1.0 - a) * col[k].c[ch] + a * C[ch];"),
}

PINS = ["tests/test_oracle_hand.py", "tests/test_oracle_bruteforce.py", "tests/test_oracle_invariants.py",
        "tests/test_oracle_keys.py", "tests/test_oracle_cutoff.py",
        "tests/test_oracle_backface.py", "tests/test_oracle_vcol.py"]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found once"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-pthread", "-shared", "-fPIC",
                           "-o", str(lib), str(mut), "-lm"])
    env = dict(os.environ, LR_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PINS,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
