"""Python binding of the HIP library (ctypes over include/lucidraster.h).

Argument marshalling only: every stage of a render runs in the library's
gfx950 kernels.  PyTorch supplies device memory (the arena and the output
tensors) and the current HIP stream.  There is no CPU fallback: when the
library is missing every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblucidraster.so")

LR_OK = 0
LR_ERR_INVALID_ARG = -1
LR_ERR_OUT_OF_MEMORY = -2
LR_ERR_DEVICE = -3
LR_ERR_CAPACITY = -4
LR_ERR_NOT_FOUND = -5
LR_ERR_BUSY = -6
LR_FLAG_TIMING = 1
LR_FLAG_NO_GRAPH = 2
LR_FLAG_ALPHA_CUTOFF = 4
LR_FLAG_DENSITY_CLASSES = 8
LR_FLAG_BBOX_BINNING = 16
LR_FLAG_CULL_BACKFACES = 32
LR_FRAME_ERR_CAPACITY = 1
LR_FRAME_ERR_DENSE = 4

SORTER_DEPTHS = (2, 4, 8, 12, 16, 24, 32)
BIN_SIZES = (16, 32, 64)
BLOCK_HEIGHTS = (4, 8)
STAGES = ("setup", "bin_count", "bin_scan", "bin_scatter", "raster", "unused", "fallback", "total")


class LRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class Camera(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_float * 3), ("rot", (ctypes.c_float * 3) * 3),
                ("fov_y", ctypes.c_float), ("z_near", ctypes.c_float)]


class Config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("arena", ctypes.c_void_p),
                ("arena_bytes", ctypes.c_uint64), ("bin_size", ctypes.c_uint32),
                ("block_h", ctypes.c_uint32), ("sorter_depth", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("hbm_budget_bytes", ctypes.c_uint64),
                ("batch_slots", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("quads", ctypes.c_uint64), ("visible", ctypes.c_uint64),
                ("culled", ctypes.c_uint64 * 8), ("bin_pairs", ctypes.c_uint64),
                ("block_entries", ctypes.c_uint64), ("fragments", ctypes.c_uint64),
                ("flagged_pixels", ctypes.c_uint64), ("dense_blocks", ctypes.c_uint64),
                ("error_word", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("stage_us", ctypes.c_float * 8)]


class Request(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_uint64), ("camera", Camera), ("width", ctypes.c_uint32),
                ("height", ctypes.c_uint32), ("out_rgba8", ctypes.c_void_p),
                ("bin_size", ctypes.c_uint32), ("sorter_depth", ctypes.c_uint32),
                ("block_h", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("status", ctypes.c_void_p)]


class TuneRule(ctypes.Structure):
    _fields_ = [("max_pixels", ctypes.c_uint32), ("max_quads_per_pixel", ctypes.c_float),
                ("bin_size", ctypes.c_uint32), ("block_h", ctypes.c_uint32),
                ("sorter_depth", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


EXPORTS = ["lr_status_string", "lr_last_error", "lr_create", "lr_destroy", "lr_upload_scene",
           "lr_upload_scene_vertex_colors", "lr_release_scene", "lr_render", "lr_render_noalloc", "lr_render_debug", "lr_render_unsorted",
           "lr_render_batch", "lr_set_tuning", "lr_request_bytes", "lr_sync", "lr_get_stats",
           "lr_get_stage_times", "lr_debug_setup", "lr_debug_bins"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library and declare its signatures (no device work)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    P, U32, U64, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
    CTX = ctypes.c_void_p
    lib.lr_status_string.restype = ctypes.c_char_p
    lib.lr_status_string.argtypes = [I32]
    lib.lr_last_error.restype = ctypes.c_char_p
    lib.lr_last_error.argtypes = [CTX]
    sig = {
        "lr_create": [ctypes.POINTER(Config), ctypes.POINTER(CTX)],
        "lr_destroy": [CTX],
        "lr_upload_scene": [CTX, P, U32, ctypes.c_int, ctypes.POINTER(U64)],
        "lr_upload_scene_vertex_colors": [CTX, P, U32, ctypes.POINTER(U64)],
        "lr_release_scene": [CTX, U64],
        "lr_render": [CTX, U64, ctypes.POINTER(Camera), U32, U32, P, P],
        "lr_render_noalloc": [CTX, U64, ctypes.POINTER(Camera), U32, U32, P, P],
        "lr_render_debug": [CTX, U64, ctypes.POINTER(Camera), U32, U32, P, P, P, P, P, P, P, U32],
        "lr_render_unsorted": [CTX, U64, ctypes.POINTER(Camera), U32, U32, P, P, P],
        "lr_render_batch": [CTX, ctypes.POINTER(Request), U32, P],
        "lr_set_tuning": [CTX, ctypes.POINTER(TuneRule), U32],
        "lr_request_bytes": [CTX, ctypes.POINTER(Request), ctypes.POINTER(U64)],
        "lr_sync": [CTX],
        "lr_get_stats": [CTX, ctypes.POINTER(Stats)],
        "lr_get_stage_times": [CTX, U32, P, ctypes.POINTER(U32)],
        "lr_debug_setup": [CTX, U64, ctypes.POINTER(Camera), U32, U32, P, P, P, P, P],
        "lr_debug_bins": [CTX, U64, ctypes.POINTER(Camera), U32, U32, U32, P, P, U64,
                          ctypes.POINTER(U64)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.restype = I32
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


def camera_struct(cam) -> Camera:
    """scenes.Camera (or a packed camera record) -> lr_camera."""
    rec = cam.as_record() if hasattr(cam, "as_record") else cam
    c = Camera()
    for k in range(3):
        c.pos[k] = float(rec["pos"][k])
    rot = np.asarray(rec["rot"], np.float32)
    for r in range(3):
        for k in range(3):
            c.rot[r][k] = float(rot[r, k])
    c.fov_y = float(rec["fov_y"])
    c.z_near = float(rec["z_near"])
    return c


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


class Context:
    """A rendering context on one GPU with a torch-owned device arena."""

    def __init__(self, arena_bytes: int = 1 << 30, device: int = 0, bin_size: int = 32,
                 sorter_depth: int = 8, timing: bool = False, stream=None, block_h: int = 8,
                 batch_slots: int = 2, graphs: bool = True, tuning=None, alpha_cutoff: bool = False,
                 density_classes: bool = False, bbox_binning: bool = False, cull_backfaces: bool = False):
        import torch
        self._torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm GPU visible to torch")
        self.device = device
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        self.stream = stream
        cfg = Config(device=device, stream=None if stream is None else int(stream.cuda_stream),
                     arena=self.arena.data_ptr(), arena_bytes=int(arena_bytes), bin_size=bin_size,
                     block_h=block_h, sorter_depth=sorter_depth,
                     flags=(LR_FLAG_TIMING if timing else 0) | (0 if graphs else LR_FLAG_NO_GRAPH) |
                     (LR_FLAG_ALPHA_CUTOFF if alpha_cutoff else 0) |
                     (LR_FLAG_DENSITY_CLASSES if density_classes else 0) |
                     (LR_FLAG_BBOX_BINNING if bbox_binning else 0) |
                     (LR_FLAG_CULL_BACKFACES if cull_backfaces else 0),
                     hbm_budget_bytes=0, batch_slots=batch_slots)
        self.bin_size, self.sorter_depth, self.block_h = bin_size, sorter_depth, block_h
        h = ctypes.c_void_p()
        self._check(self.lib.lr_create(ctypes.byref(cfg), ctypes.byref(h)), None)
        self.h = h
        if tuning:
            self.set_tuning(tuning)

    # -- plumbing
    def _check(self, st: int, h=None):
        if st != LR_OK:
            msg = self.lib.lr_last_error(h if h is not None else getattr(self, "h", None))
            name = self.lib.lr_status_string(st).decode()
            raise LRError(st, f"{name}: {msg.decode() if msg else ''}")

    def _stream(self, stream=None):
        s = stream if stream is not None else (self.stream or self._torch.cuda.current_stream(self.device))
        return int(s.cuda_stream)

    def close(self):
        if getattr(self, "h", None):
            self.lib.lr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- scenes
    def upload(self, v: np.ndarray, rgba: np.ndarray) -> int:
        """Make quads resident: v float32 [n,4,3], rgba uint32 [n]."""
        n = int(v.shape[0])
        rec = np.zeros(n, dtype=np.dtype([("v", "<f4", (4, 3)), ("rgba", "<u4")]))
        rec["v"] = v
        rec["rgba"] = rgba
        out = ctypes.c_uint64()
        self._check(self.lib.lr_upload_scene(self.h, rec.ctypes.data_as(ctypes.c_void_p), n, 0,
                                             ctypes.byref(out)), self.h)
        return int(out.value)

    def upload_vertex_colors(self, v: np.ndarray, vcol: np.ndarray) -> int:
        """Make quads with per-vertex colours resident: v float32 [n,4,3],
        vcol uint32 [n,4] (straight-alpha RGBA8 per vertex)."""
        n = int(v.shape[0])
        rec = np.zeros(n, dtype=np.dtype([("v", "<f4", (4, 3)), ("rgba", "<u4", (4,))]))
        rec["v"] = v
        rec["rgba"] = np.asarray(vcol, np.uint32).reshape(n, 4)
        out = ctypes.c_uint64()
        self._check(self.lib.lr_upload_scene_vertex_colors(self.h, rec.ctypes.data_as(ctypes.c_void_p), n,
                                                           ctypes.byref(out)), self.h)
        return int(out.value)

    def upload_device(self, quads) -> int:
        """Make quads resident from a device tensor of packed 52-byte records."""
        n = int(quads.numel() // 52)
        out = ctypes.c_uint64()
        self._check(self.lib.lr_upload_scene(self.h, quads.data_ptr(), n, 1, ctypes.byref(out)), self.h)
        return int(out.value)

    def release(self, scene: int):
        self._check(self.lib.lr_release_scene(self.h, scene), self.h)

    # -- rendering
    def new_image(self, W: int, H: int):
        return self._torch.empty((H, W, 4), dtype=self._torch.uint8, device=f"cuda:{self.device}")

    def render(self, scene: int, cam, W: int, H: int, out=None, stream=None, check: bool = True):
        """Sorted (exact) render -> uint8 [H, W, 4] device tensor.  With check,
        waits and re-renders once if a capacity was exceeded."""
        out = self.new_image(W, H) if out is None else out
        c = camera_struct(cam)
        for attempt in range(2):
            self._check(self.lib.lr_render(self.h, scene, ctypes.byref(c), W, H, out.data_ptr(),
                                           self._stream(stream)), self.h)
            if not check:
                return out
            st = self.lib.lr_sync(self.h)
            if st == LR_ERR_CAPACITY and attempt == 0:
                continue
            self._check(st, self.h)
            return out
        return out

    def render_noalloc(self, scene: int, cam, W: int, H: int, out=None, stream=None, check: bool = True):
        """Sorted render whose frame workspace is the library's fixed device
        array (lr_render_noalloc: the call allocates nothing).  With check,
        waits and renders once more if a capacity was exceeded."""
        out = self.new_image(W, H) if out is None else out
        c = camera_struct(cam)
        for attempt in range(2):
            self._check(self.lib.lr_render_noalloc(self.h, scene, ctypes.byref(c), W, H, out.data_ptr(),
                                                   self._stream(stream)), self.h)
            if not check:
                return out
            st = self.lib.lr_sync(self.h)
            if st == LR_ERR_CAPACITY and attempt == 0:
                continue
            self._check(st, self.h)
            return out
        return out

    def render_unsorted(self, scene: int, cam, W: int, H: int, out=None, rgba_f32=None, stream=None,
                        check: bool = True):
        out = self.new_image(W, H) if out is None else out
        c = camera_struct(cam)
        for attempt in range(2):
            self._check(self.lib.lr_render_unsorted(self.h, scene, ctypes.byref(c), W, H, out.data_ptr(),
                                                    self._stream(stream), _ptr(rgba_f32)), self.h)
            if not check:
                return out
            st = self.lib.lr_sync(self.h)
            if st == LR_ERR_CAPACITY and attempt == 0:
                continue
            self._check(st, self.h)
            return out
        return out

    def render_debug(self, scene: int, cam, W: int, H: int, order: bool = False) -> Dict[str, object]:
        """Sorted render plus parity artefacts (all device tensors):
        rgba8, rgba_f32 [H,W,4], count [H,W], flagged [H,W] and, with order,
        order_offsets [W*H+1] / order_ids (quad ids per pixel in blend order)."""
        torch = self._torch
        dev = f"cuda:{self.device}"
        out = self.new_image(W, H)
        f32 = torch.zeros((H, W, 4), dtype=torch.float32, device=dev)
        cnt = torch.zeros((H, W), dtype=torch.int32, device=dev)
        flg = torch.zeros((H, W), dtype=torch.uint8, device=dev)
        c = camera_struct(cam)

        def run(off=None, ids=None, cap=0):
            for attempt in range(2):
                self._check(self.lib.lr_render_debug(self.h, scene, ctypes.byref(c), W, H, out.data_ptr(),
                                                     self._stream(), f32.data_ptr(), cnt.data_ptr(),
                                                     flg.data_ptr(), _ptr(off), _ptr(ids), cap), self.h)
                st = self.lib.lr_sync(self.h)
                if st == LR_ERR_CAPACITY and attempt == 0:
                    continue
                self._check(st, self.h)
                return

        run()
        res = {"rgba8": out, "rgba_f32": f32, "count": cnt, "flagged": flg}
        if order:
            counts = cnt.reshape(-1).to(torch.int64)
            off = torch.zeros(W * H + 1, dtype=torch.int64, device=dev)
            off[1:] = torch.cumsum(counts, 0)
            total = int(off[-1].item())
            off32 = off.to(torch.int32)
            ids = torch.zeros(max(total, 1), dtype=torch.int32, device=dev)
            run(off32, ids, max(total, 1))
            res["order_offsets"] = off
            res["order_ids"] = ids[:total]
        return res

    @staticmethod
    def _request(req, out_ptr=None, status_ptr=None) -> Request:
        """(scene, cam, W, H, out[, bin_size[, sorter_depth[, block_h]]]) -> lr_request;
        missing or None tuning fields are 0 (tuning rules, then context defaults)."""
        scene, cam, W, H, out = req[:5]
        tune = list(req[5:8]) + [None] * (3 - len(req[5:8]))
        r = Request()
        r.scene = scene
        r.camera = camera_struct(cam)
        r.width, r.height = W, H
        r.out_rgba8 = out_ptr if out_ptr is not None else (out.data_ptr() if out is not None else None)
        r.bin_size = tune[0] or 0
        r.sorter_depth = tune[1] or 0
        r.block_h = tune[2] or 0
        r.status = status_ptr
        return r

    def render_batch(self, reqs, stream=None, check: bool = True, status=None):
        """Render a list of requests (scene, cam, W, H, out[, bin_size, sorter_depth,
        block_h]) in batched launches.  With check, waits and re-renders once if a
        capacity was exceeded.  status: an int32 device tensor of len(reqs)
        receiving each frame's LR_FRAME_ERR_* bits (stream ordered)."""
        arr = (Request * len(reqs))()
        for k, req in enumerate(reqs):
            sp = None if status is None else int(status.data_ptr()) + 4 * k
            arr[k] = self._request(req, status_ptr=sp)
        for attempt in range(2):
            self._check(self.lib.lr_render_batch(self.h, arr, len(reqs), self._stream(stream)), self.h)
            if not check:
                return
            st = self.lib.lr_sync(self.h)
            if st == LR_ERR_CAPACITY and attempt == 0:
                continue
            self._check(st, self.h)
            return

    def set_tuning(self, rules):
        """Tuning rules: dicts with max_pixels, max_quads_per_pixel, bin_size,
        block_h, sorter_depth (first match wins)."""
        arr = (TuneRule * max(len(rules), 1))()
        for k, u in enumerate(rules):
            arr[k] = TuneRule(int(u["max_pixels"]), float(u["max_quads_per_pixel"]), int(u["bin_size"]),
                              int(u["block_h"]), int(u["sorter_depth"]), 0)
        self._check(self.lib.lr_set_tuning(self.h, arr, len(rules)), self.h)

    def request_bytes(self, scene: int, cam, W: int, H: int, bin_size=None, sorter_depth=None,
                      block_h=None) -> int:
        """Device bytes one request holds while in flight (after tuning)."""
        r = self._request((scene, cam, W, H, None, bin_size, sorter_depth, block_h), out_ptr=0)
        b = ctypes.c_uint64()
        self._check(self.lib.lr_request_bytes(self.h, ctypes.byref(r), ctypes.byref(b)), self.h)
        return int(b.value)

    def sync(self):
        self._check(self.lib.lr_sync(self.h), self.h)

    def stats(self) -> Dict[str, object]:
        s = Stats()
        self._check(self.lib.lr_get_stats(self.h, ctypes.byref(s)), self.h)
        return {"quads": s.quads, "visible": s.visible, "culled": list(s.culled),
                "bin_pairs": s.bin_pairs, "block_entries": s.block_entries, "fragments": s.fragments,
                "flagged_pixels": s.flagged_pixels, "dense_blocks": s.dense_blocks,
                "error_word": s.error_word, "stage_us": dict(zip(STAGES, list(s.stage_us)))}

    def stage_times(self, max_frames: int = 1024) -> np.ndarray:
        """Per-frame stage times in microseconds, [frames, 8] (see STAGES)."""
        buf = np.zeros((max_frames, 8), np.float32)
        n = ctypes.c_uint32()
        self._check(self.lib.lr_get_stage_times(self.h, max_frames, buf.ctypes.data_as(ctypes.c_void_p),
                                                ctypes.byref(n)), self.h)
        return buf[:n.value]

    # -- parity dumps
    def debug_setup(self, scene: int, cam, W: int, H: int, n: int) -> Dict[str, np.ndarray]:
        X = np.zeros((n, 4), np.int32)
        Y = np.zeros((n, 4), np.int32)
        bb = np.zeros((n, 4), np.int32)
        pl = np.zeros((n, 3), np.float64)
        cl = np.zeros(n, np.uint8)
        c = camera_struct(cam)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._check(self.lib.lr_debug_setup(self.h, scene, ctypes.byref(c), W, H, p(X), p(Y), p(bb), p(pl),
                                            p(cl)), self.h)
        return {"X": X, "Y": Y, "bbox": bb, "plane": pl, "cull": cl}

    def debug_bins(self, scene: int, cam, W: int, H: int, bin_size: int):
        nbx, nby = (W + bin_size - 1) // bin_size, (H + bin_size - 1) // bin_size
        counts = np.zeros(nbx * nby, np.uint32)
        total = ctypes.c_uint64()
        c = camera_struct(cam)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        for attempt in range(2):
            st = self.lib.lr_debug_bins(self.h, scene, ctypes.byref(c), W, H, bin_size, p(counts), None, 0,
                                        ctypes.byref(total))
            if st == LR_ERR_CAPACITY and attempt == 0:
                continue
            self._check(st, self.h)
            break
        ids = np.zeros(max(int(total.value), 1), np.uint32)
        self._check(self.lib.lr_debug_bins(self.h, scene, ctypes.byref(c), W, H, bin_size, p(counts), p(ids),
                                           ids.shape[0], ctypes.byref(total)), self.h)
        return counts.reshape(nby, nbx), ids[:int(total.value)]
