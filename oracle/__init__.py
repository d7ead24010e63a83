"""CPU oracle for the exact-transparency rasterizer (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-timing leg may import
this package.  The rendering library never does: it has no CPU path.

`lr_oracle.c` holds the definition (see its header for every numeric reading
of the paper); this module builds it with gcc and wraps it with ctypes.
`brute.py` is an independent exact-arithmetic re-derivation used to pin it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lr_oracle.c")
LIB = os.path.join(HERE, "liblroracle.so")
# A test may point this at a deliberately broken build to check that the pins
# catch it (tests/test_oracle_mutations.py).
_LIB_OVERRIDE = os.environ.get("LR_ORACLE_LIB")

CULL_NAMES = ["visible", "near", "guard", "degenerate", "no_sample", "edge_on", "backface"]


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, no contraction of a*b+c)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                               "-pthread", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Cam(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_float * 3), ("rot", ctypes.c_float * 9),
                ("fov_y", ctypes.c_float), ("z_near", ctypes.c_float)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build(force=True)
            lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        lib.lro_focal.restype = ctypes.c_double
        lib.lro_focal.argtypes = [ctypes.c_uint32, ctypes.c_float]
        lib.lro_setup.restype = None
        lib.lro_setup.argtypes = [ctypes.c_uint32, P, ctypes.POINTER(_Cam), ctypes.c_uint32,
                                  ctypes.c_uint32, ctypes.c_double, P, P, P, P, P, P, P, ctypes.c_int, P]
        lib.lro_render.restype = ctypes.c_int64
        lib.lro_render.argtypes = [ctypes.c_uint32, P, P, P, P, P, P, P, P, ctypes.c_uint32,
                                   ctypes.c_uint32, ctypes.c_int, P, P, P, P, P, ctypes.c_uint32,
                                   P, P, ctypes.c_double]
        lib.lro_count.restype = ctypes.c_int64
        lib.lro_count.argtypes = [ctypes.c_uint32, P, P, P, P, ctypes.c_uint32, ctypes.c_uint32, P,
                                  ctypes.c_uint32]
        lib.lro_pixels.restype = ctypes.c_int64
        lib.lro_pixels.argtypes = [ctypes.c_uint32, P, P, P, P, P, P, P, P, ctypes.c_uint32,
                                   ctypes.c_int, ctypes.c_uint32, P, P, P, P, P, ctypes.c_uint64,
                                   P, P, ctypes.c_double, ctypes.c_uint32]
        lib.lro_bins.restype = ctypes.c_int64
        lib.lro_bins.argtypes = [ctypes.c_uint32, P, P, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint32, P, P, P, ctypes.c_uint64]
        lib.lro_covers.restype = ctypes.c_int
        lib.lro_covers.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32]
        lib.lro_key.restype = ctypes.c_float
        lib.lro_key.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, P,
                                ctypes.c_int32, ctypes.c_int32]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cam(camera) -> _Cam:
    c = _Cam()
    rec = camera.as_record() if hasattr(camera, "as_record") else camera
    for k in range(3):
        c.pos[k] = float(rec["pos"][k])
    rot = np.asarray(rec["rot"], np.float32).reshape(9)
    for k in range(9):
        c.rot[k] = float(rot[k])
    c.fov_y = float(rec["fov_y"])
    c.z_near = float(rec["z_near"])
    return c


def focal(height: int, fov_y: float) -> float:
    return _load().lro_focal(height, fov_y)


class Setup:
    """Per-quad setup records (snapped vertices, pixel bbox, depth plane, cull)."""

    def __init__(self, n: int):
        self.n = n
        self.X = np.zeros((n, 4), np.int32)
        self.Y = np.zeros((n, 4), np.int32)
        self.bbox = np.zeros((n, 4), np.int32)
        self.A = np.zeros(n, np.float64)
        self.B = np.zeros(n, np.float64)
        self.C0 = np.zeros(n, np.float64)
        self.cull = np.zeros(n, np.uint8)
        self.cam = np.zeros((n, 4, 3), np.float64)  # camera-space vertices
        self.f = 0.0

    @property
    def visible(self) -> np.ndarray:
        return self.cull == 0

    def cull_counts(self) -> Dict[str, int]:
        bc = np.bincount(self.cull, minlength=len(CULL_NAMES))
        return {name: int(bc[k]) for k, name in enumerate(CULL_NAMES)}


def setup(v: np.ndarray, camera, W: int, H: int, cull_backfaces: bool = False) -> Setup:
    """Per-quad setup; with cull_backfaces, quads winding clockwise on the
    display are culled (reason "backface")."""
    lib = _load()
    v = np.ascontiguousarray(v, np.float32).reshape(-1, 4, 3)
    n = v.shape[0]
    s = Setup(n)
    cam = _cam(camera)
    s.f = lib.lro_focal(H, cam.fov_y)
    if n:
        lib.lro_setup(n, _p(v), ctypes.byref(cam), W, H, s.f, _p(s.X), _p(s.Y), _p(s.bbox),
                      _p(s.A), _p(s.B), _p(s.C0), _p(s.cull), int(cull_backfaces), _p(s.cam))
    return s


def default_threads() -> int:
    """Worker threads of a whole-frame render: the host cores this process
    may run on, at most 16 (LR_ORACLE_THREADS overrides)."""
    env = os.environ.get("LR_ORACLE_THREADS")
    if env:
        return max(1, int(env))
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _mode(unsorted: bool, cutoff: bool) -> int:
    if unsorted and cutoff:
        raise ValueError("the transmittance cutoff applies to the sorted blend only")
    return 1 if unsorted else (2 if cutoff else 0)


def render(v: np.ndarray, rgba: np.ndarray, camera, W: int, H: int, unsorted: bool = False,
           want_order: bool = True, st: Optional[Setup] = None,
           threads: Optional[int] = None, cutoff: bool = False,
           cull_backfaces: bool = False, vcol: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """Whole-frame reference render.  Returns rgba_f64 [H,W,4], rgba8 [H,W,4],
    count [H,W], order_offsets [W*H+1], order_ids [total], setup, and the
    number of worker threads used (row bands; the result does not depend on
    it).  With cutoff, each pixel stops after the fragment that brings its
    single-precision transmittance below 2^-20: count, order and total are
    those of the blended prefixes ("covering" keeps the full total).  vcol:
    per-vertex colours uint32 [n, 4] (perspective-correct interpolation over
    the triangle covering each sample) instead of the flat rgba."""
    lib = _load()
    mode = _mode(unsorted, cutoff)
    if vcol is not None and cutoff:
        raise ValueError("the transmittance cutoff is defined for flat colours only")
    vc = None if vcol is None else np.ascontiguousarray(vcol, np.uint32).reshape(-1, 4)
    st = st or setup(v, camera, W, H, cull_backfaces)
    threads = default_threads() if threads is None else max(1, int(threads))
    rgba = np.ascontiguousarray(rgba, np.uint32)
    npix = W * H
    out_f = np.zeros((H, W, 4), np.float64)
    out_8 = np.zeros((H, W, 4), np.uint8)
    cnt = np.zeros((H, W), np.uint32)
    n = st.n
    res = {"rgba_f64": out_f, "rgba8": out_8, "count": cnt, "setup": st, "threads": threads}
    if want_order:
        # the fragment total sizes the id buffer
        total = lib.lro_count(n, _p(st.X), _p(st.Y), _p(st.bbox), _p(st.cull), W, H, _p(cnt),
                              threads) if n else 0
        off = np.zeros(npix + 1, np.uint64)
        ids = np.zeros(max(int(total), 1), np.uint32)
        if n:
            total = lib.lro_render(n, _p(st.X), _p(st.Y), _p(st.bbox), _p(st.A), _p(st.B), _p(st.C0),
                                   _p(st.cull), _p(rgba), W, H, mode, _p(out_f), _p(out_8),
                                   _p(cnt), _p(off), _p(ids), threads,
                                   None if vc is None else _p(vc), _p(st.cam), st.f)
        if total < 0:
            raise MemoryError("oracle render failed")
        ids = ids[:int(total)]
        if mode == 2:
            # keep each pixel's blended prefix of its full list
            full = np.diff(off).astype(np.int64)
            pos = np.arange(int(total), dtype=np.int64) - np.repeat(off[:-1].astype(np.int64), full)
            ids = ids[pos < np.repeat(cnt.reshape(-1).astype(np.int64), full)]
            off = np.zeros(npix + 1, np.uint64)
            off[1:] = np.cumsum(cnt.reshape(-1), dtype=np.uint64)
        res["order_offsets"] = off
        res["order_ids"] = ids
    else:
        total = lib.lro_render(n, _p(st.X), _p(st.Y), _p(st.bbox), _p(st.A), _p(st.B), _p(st.C0),
                               _p(st.cull), _p(rgba), W, H, mode, _p(out_f), _p(out_8),
                               _p(cnt), None, None, threads,
                               None if vc is None else _p(vc), _p(st.cam), st.f) if n else 0
    if total < 0:
        raise MemoryError("oracle render failed")
    res["covering"] = int(total)
    res["total"] = int(cnt.sum(dtype=np.uint64)) if mode == 2 else int(total)
    return res


def pixels(v: np.ndarray, rgba: np.ndarray, camera, W: int, H: int, pix: np.ndarray,
           unsorted: bool = False, want_ids: bool = True,
           st: Optional[Setup] = None, cutoff: bool = False,
           cull_backfaces: bool = False, vcol: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """Reference result for selected pixels (pix = j*W + i), each computed by
    testing every quad.  Returns rgba_f64 [k,4], count [k], offsets, ids
    (with cutoff: those of the blended prefixes)."""
    lib = _load()
    mode = _mode(unsorted, cutoff)
    if vcol is not None and cutoff:
        raise ValueError("the transmittance cutoff is defined for flat colours only")
    vc = None if vcol is None else np.ascontiguousarray(vcol, np.uint32).reshape(-1, 4)
    st = st or setup(v, camera, W, H, cull_backfaces)
    rgba = np.ascontiguousarray(rgba, np.uint32)
    pix = np.ascontiguousarray(pix, np.uint32)
    k = pix.shape[0]
    out_f = np.zeros((k, 4), np.float64)
    cnt = np.zeros(k, np.uint32)
    off = np.zeros(k + 1, np.uint64)
    cap = 1 << 16
    while True:
        ids = np.zeros(cap, np.uint32)
        total = lib.lro_pixels(st.n, _p(st.X), _p(st.Y), _p(st.bbox), _p(st.A), _p(st.B),
                               _p(st.C0), _p(st.cull), _p(rgba), W, mode, k, _p(pix),
                               _p(out_f), _p(cnt), _p(off) if want_ids else None,
                               _p(ids) if want_ids else None, cap, None if vc is None else _p(vc),
                               _p(st.cam), st.f, H)
        if total >= 0:
            break
        if not want_ids or cap > (1 << 31):
            raise MemoryError("oracle pixels failed")
        cap *= 8
    res = {"rgba_f64": out_f, "count": cnt, "setup": st}
    if want_ids:
        res["offsets"] = off
        res["ids"] = ids[:int(total)]
    return res


def bins(st: Setup, W: int, H: int, bin_size: int):
    """Bounding-box bin lists: (counts [nby, nbx], offsets [nbins+1], ids)."""
    lib = _load()
    nbx, nby = (W + bin_size - 1) // bin_size, (H + bin_size - 1) // bin_size
    counts = np.zeros(nbx * nby, np.uint32)
    total = lib.lro_bins(st.n, _p(st.bbox), _p(st.cull), W, H, bin_size, _p(counts), None, None, 0)
    off = np.zeros(nbx * nby + 1, np.uint64)
    ids = np.zeros(max(int(total), 1), np.uint32)
    lib.lro_bins(st.n, _p(st.bbox), _p(st.cull), W, H, bin_size, _p(counts), _p(off), _p(ids),
                 ids.shape[0])
    return counts.reshape(nby, nbx), off, ids[:int(total)]


def covers(X: np.ndarray, Y: np.ndarray, i: int, j: int) -> bool:
    X = np.ascontiguousarray(X, np.int32)
    Y = np.ascontiguousarray(Y, np.int32)
    return bool(_load().lro_covers(_p(X), _p(Y), i, j))


def key(st: Setup, q: int, i: int, j: int) -> np.float32:
    bb = np.ascontiguousarray(st.bbox[q], np.int32)
    return np.float32(_load().lro_key(st.A[q], st.B[q], st.C0[q], _p(bb), i, j))


def to_u8(x: np.ndarray) -> np.ndarray:
    return np.clip(np.floor(255.0 * np.asarray(x, np.float64) + 0.5), 0, 255).astype(np.uint8)
