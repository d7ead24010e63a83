"""Exact-arithmetic brute force used to pin the C oracle (test infrastructure).

Every quantity here is derived a second way, in exact rationals, from the
problem statement rather than from the oracle's formulas:

* projection and snap: the pinhole projection evaluated exactly, then rounded
  to the 1/256 pixel grid (a tie within 1e-6 of a half step is reported so a
  caller can skip it);
* coverage: a point-in-triangle orientation test at the pixel centre moved by
  (eps, eps^2) with eps = 2^-40.  No fill rule is written anywhere: the tiny
  shift alone decides samples on edges, and for integer coordinates below
  2^25 its outcome is the limit as eps -> 0;
* depth: the exact ray/plane intersection (plane through the vertex centroid,
  normal from the diagonals), giving 1/z at the pixel centre as a Fraction;
* order: exact 1/z descending, quad index ascending;
* blend: front-to-back in Fractions.

It runs pure-Python loops, so it is only for tiny frames (a few hundred
pixels times a few dozen quads).
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, List, Optional, Tuple

import numpy as np

EPS = Fraction(1, 1 << 40)


def camera_space(v: np.ndarray, cam_rec) -> List[List[Tuple[Fraction, Fraction, Fraction]]]:
    """Exact camera-space vertices R (v - pos)."""
    pos = [Fraction(float(x)) for x in np.asarray(cam_rec["pos"], np.float32)]
    rot = [[Fraction(float(x)) for x in row] for row in np.asarray(cam_rec["rot"], np.float32)]
    out = []
    for quad in np.asarray(v, np.float32):
        cq = []
        for vert in quad:
            d = [Fraction(float(vert[k])) - pos[k] for k in range(3)]
            cq.append(tuple(sum(rot[r][k] * d[k] for k in range(3)) for r in range(3)))
        out.append(cq)
    return out


def project_exact(c, f: Fraction, cx: Fraction, cy: Fraction):
    return [(f * p[0] / p[2] + cx, -f * p[1] / p[2] + cy) for p in c]


def snap(x: Fraction) -> Tuple[int, bool]:
    """Round 256 x to the nearest integer (ties to even); flag near-ties."""
    y = x * 256
    fl = y.numerator // y.denominator
    frac = y - fl
    near_tie = abs(frac - Fraction(1, 2)) < Fraction(1, 10**6)
    if frac > Fraction(1, 2) or (frac == Fraction(1, 2) and fl % 2 == 1):
        return fl + 1, near_tie
    return fl, near_tie


def _orient(ax, ay, bx, by, px, py):
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax)


def _sign(x) -> int:
    return (x > 0) - (x < 0)


def tri_contains(P, ia, ib, ic, px, py) -> bool:
    (ax, ay), (bx, by), (cx_, cy_) = P[ia], P[ib], P[ic]
    s = _sign(_orient(ax, ay, bx, by, cx_, cy_))
    if s == 0:
        return False
    return (_sign(_orient(ax, ay, bx, by, px, py)) == s and
            _sign(_orient(bx, by, cx_, cy_, px, py)) == s and
            _sign(_orient(cx_, cy_, ax, ay, px, py)) == s)


def covers(X, Y, i: int, j: int) -> bool:
    """Quad (snapped integer corners) covers pixel (i, j): union of triangles
    (0,1,2) and (0,2,3), sampled at the shifted centre."""
    P = [(Fraction(int(X[k])), Fraction(int(Y[k]))) for k in range(4)]
    px = Fraction(256 * i + 128) + EPS
    py = Fraction(256 * j + 128) + EPS * EPS
    return tri_contains(P, 0, 1, 2, px, py) or tri_contains(P, 0, 2, 3, px, py)


def inv_depth(c, f: Fraction, cx: Fraction, cy: Fraction, i: int, j: int) -> Optional[Fraction]:
    """Exact 1/z where the ray through pixel centre (i, j) meets the quad's plane."""
    e1 = [c[2][k] - c[0][k] for k in range(3)]
    e2 = [c[3][k] - c[1][k] for k in range(3)]
    n = (e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0])
    m = [(c[0][k] + c[1][k] + c[2][k] + c[3][k]) / 4 for k in range(3)]
    nm = sum(n[k] * m[k] for k in range(3))
    if nm == 0:
        return None
    r = ((Fraction(i) + Fraction(1, 2) - cx) / f, -(Fraction(j) + Fraction(1, 2) - cy) / f, Fraction(1))
    return sum(n[k] * r[k] for k in range(3)) / nm


def snap_quads(v: np.ndarray, cam_rec, W: int, H: int, f: float):
    """Exact projection and snap of every quad in front of the near plane.
    Returns X, Y (int64 [n,4]), in_front (bool [n]) and the set of quads with
    a coordinate within 1e-6 of a rounding tie."""
    n = len(v)
    ff = Fraction(f)
    cx, cy = Fraction(W, 2), Fraction(H, 2)
    cs = camera_space(v, cam_rec)
    X = np.zeros((n, 4), np.int64)
    Y = np.zeros((n, 4), np.int64)
    in_front = np.ones(n, bool)
    near_tie = set()
    zn = Fraction(float(np.float32(cam_rec["z_near"])))
    for q in range(n):
        if any(p[2] <= zn for p in cs[q]):
            in_front[q] = False
            continue
        for k, (sx, sy) in enumerate(project_exact(cs[q], ff, cx, cy)):
            X[q, k], t1 = snap(sx)
            Y[q, k], t2 = snap(sy)
            if t1 or t2:
                near_tie.add(q)
    return X, Y, in_front, near_tie


def render(v: np.ndarray, rgba: np.ndarray, cam_rec, W: int, H: int, f: float,
           X: Optional[np.ndarray] = None, Y: Optional[np.ndarray] = None,
           visible: Optional[np.ndarray] = None) -> Dict[str, object]:
    """Exact frame.  When X, Y and visible are given (e.g. the oracle's own
    setup), coverage is evaluated on those corners; otherwise they are
    computed exactly here (quads with near-tie snaps are then marked).

    Returns counts [H][W], order (lists of quad ids), inv-depth lists,
    rgba (Fractions), near_tie set."""
    n = len(v)
    ff = Fraction(f)
    cx, cy = Fraction(W, 2), Fraction(H, 2)
    cs = camera_space(v, cam_rec)
    near_tie = set()
    if X is None:
        X, Y, visible, near_tie = snap_quads(v, cam_rec, W, H, f)
    counts = np.zeros((H, W), np.int64)
    order: List[List[List[int]]] = [[[] for _ in range(W)] for _ in range(H)]
    depths: List[List[List[Fraction]]] = [[[] for _ in range(W)] for _ in range(H)]
    colour = [[None for _ in range(W)] for _ in range(H)]
    for j in range(H):
        for i in range(W):
            frags = []
            for q in range(n):
                if not visible[q]:
                    continue
                if covers(X[q], Y[q], i, j):
                    d = inv_depth(cs[q], ff, cx, cy, i, j)
                    frags.append((d, q))
            frags.sort(key=lambda t: (-(t[0] if t[0] is not None else Fraction(0)), t[1]))
            counts[j, i] = len(frags)
            order[j][i] = [q for _, q in frags]
            depths[j][i] = [d for d, _ in frags]
            T = Fraction(1)
            C = [Fraction(0)] * 3
            for _, q in frags:
                c = int(rgba[q])
                a = Fraction(c >> 24, 255)
                for ch in range(3):
                    C[ch] += T * a * Fraction((c >> (8 * ch)) & 255, 255)
                T *= (1 - a)
            colour[j][i] = (C[0], C[1], C[2], 1 - T)
    return {"count": counts, "order": order, "inv_depth": depths, "rgba": colour,
            "near_tie": near_tie, "X": X, "Y": Y}
