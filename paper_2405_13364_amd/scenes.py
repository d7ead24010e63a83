"""Seeded synthetic quad scenes shaped like the paper's transparency workloads.

This module only *builds inputs*: world-space quads, colours and a camera.  It
holds none of the rasterizer's arithmetic (no projection to the sample grid, no
coverage, depth keys or blending); both the CPU oracle and the HIP path consume
what it produces.

The paper evaluates on twelve textured scenes (Section 3, "Test scenes") that
are not available here, so every workload is synthetic.  A scene is a set of
planar rectangles placed so that their projected centre, projected side
lengths and view depth follow simple distributions:

* centre on screen: uniform, or a Gaussian cloud around the screen centre;
* view depth z: uniform in a range;
* side lengths w, h in *pixels at that depth*: uniform in a range;
* orientation: yaw and pitch uniform on [-pi, pi);
* colour: uniform RGB bytes, alpha uniform in a range, rounded to 8 bits.

Random draws are vectorised and taken in a fixed order so that a seed fixes
the scene bit for bit.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Tuple

import numpy as np

# Camera layout shared with the C ABI: pos[3], rot[3][3] (rows are the camera
# x, y, z axes in world space), fov_y (radians), z_near.
CAMERA_DTYPE = np.dtype([("pos", "<f4", (3,)), ("rot", "<f4", (3, 3)),
                         ("fov_y", "<f4"), ("z_near", "<f4")])


@dataclasses.dataclass
class Camera:
    pos: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    rot: Tuple[Tuple[float, float, float], ...] = ((1.0, 0.0, 0.0),
                                                   (0.0, 1.0, 0.0),
                                                   (0.0, 0.0, 1.0))
    fov_y: float = math.radians(60.0)
    z_near: float = 0.1

    def as_record(self) -> np.ndarray:
        """The camera as one packed record (float32 fields, 56 bytes)."""
        rec = np.zeros((), dtype=CAMERA_DTYPE)
        rec["pos"] = np.asarray(self.pos, dtype=np.float32)
        rec["rot"] = np.asarray(self.rot, dtype=np.float32)
        rec["fov_y"] = np.float32(self.fov_y)
        rec["z_near"] = np.float32(self.z_near)
        return rec

    @staticmethod
    def jittered(yaw_deg: float, pitch_deg: float, fov_y: float = math.radians(60.0),
                 z_near: float = 0.1) -> "Camera":
        """Camera at the origin turned by small yaw/pitch angles (degrees)."""
        y, p = math.radians(yaw_deg), math.radians(pitch_deg)
        ry = np.array([[math.cos(y), 0, math.sin(y)], [0, 1, 0], [-math.sin(y), 0, math.cos(y)]])
        rx = np.array([[1, 0, 0], [0, math.cos(p), -math.sin(p)], [0, math.sin(p), math.cos(p)]])
        r = (ry @ rx).T  # rows = camera axes expressed in world space
        return Camera(rot=tuple(tuple(float(x) for x in row) for row in r), fov_y=fov_y,
                      z_near=z_near)


@dataclasses.dataclass
class Scene:
    """Quads as float32 [n, 4, 3] world-space vertices and packed RGBA8 [n]."""
    v: np.ndarray
    rgba: np.ndarray
    width: int
    height: int
    camera: Camera
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.v.shape[0])

    def quad_records(self) -> np.ndarray:
        """The quads in the 52-byte packed layout of the C ABI (12 floats + rgba)."""
        rec = np.zeros(self.n, dtype=QUAD_DTYPE)
        rec["v"] = self.v
        rec["rgba"] = self.rgba
        return rec


QUAD_DTYPE = np.dtype([("v", "<f4", (4, 3)), ("rgba", "<u4")])
assert QUAD_DTYPE.itemsize == 52


@dataclasses.dataclass(frozen=True)
class Recipe:
    width: int
    height: int
    n: int
    seed: int
    gaussian: bool          # centres ~ N(screen centre, sigma*screen) instead of uniform
    sigma: float
    z: Tuple[float, float]
    side: Tuple[float, float]   # projected side length range, pixels
    alpha: Tuple[float, float]


def pack_rgba(r, g, b, a) -> np.ndarray:
    return (np.asarray(r, np.uint32) | (np.asarray(g, np.uint32) << 8)
            | (np.asarray(b, np.uint32) << 16) | (np.asarray(a, np.uint32) << 24)).astype(np.uint32)


def focal_pixels(height: int, fov_y: float) -> float:
    """Focal length in pixels, used only to size quads when building a scene."""
    return (0.5 * height) / math.tan(0.5 * float(np.float32(fov_y)))


def generate(rc: Recipe, name: str = "") -> Scene:
    """Draw a scene from a recipe.  Draw order is fixed: centre pair, z, w, h,
    yaw, pitch, rgb, alpha."""
    rng = np.random.default_rng(rc.seed)
    n, W, H = rc.n, rc.width, rc.height
    cam = Camera()
    f = focal_pixels(H, cam.fov_y)
    cx, cy = 0.5 * W, 0.5 * H
    if rc.gaussian:
        ga = rng.standard_normal(n)
        gb = rng.standard_normal(n)
        sx = cx + rc.sigma * W * ga
        sy = cy + rc.sigma * H * gb
    else:
        ua = rng.random(n)
        ub = rng.random(n)
        sx = ua * W
        sy = ub * H
    z = rng.uniform(rc.z[0], rc.z[1], n)
    w = rng.uniform(rc.side[0], rc.side[1], n)
    h = rng.uniform(rc.side[0], rc.side[1], n)
    yaw = rng.uniform(-math.pi, math.pi, n)
    pitch = rng.uniform(-math.pi, math.pi, n)
    rgb = rng.integers(0, 256, size=(n, 3))
    alpha = rng.uniform(rc.alpha[0], rc.alpha[1], n)

    centre = np.stack([(sx - cx) * z / f, -(sy - cy) * z / f, z], axis=1)
    hw = 0.5 * w * z / f
    hh = 0.5 * h * z / f
    # corner order (-,-), (+,-), (+,+), (-,+) in the quad's local frame
    sgn = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
    local = np.zeros((n, 4, 3))
    local[:, :, 0] = sgn[None, :, 0] * hw[:, None]
    local[:, :, 1] = sgn[None, :, 1] * hh[:, None]
    cyw, syw = np.cos(yaw), np.sin(yaw)
    cp, sp = np.cos(pitch), np.sin(pitch)
    # R = Ry(yaw) @ Rx(pitch), applied to (lx, ly, 0)
    lx, ly = local[:, :, 0], local[:, :, 1]
    rx_y = ly * cp[:, None]
    rx_z = ly * sp[:, None]
    wx = cyw[:, None] * lx + syw[:, None] * rx_z
    wy = rx_y
    wz = -syw[:, None] * lx + cyw[:, None] * rx_z
    verts = centre[:, None, :] + np.stack([wx, wy, wz], axis=2)
    v = verts.astype(np.float32)
    a8 = np.rint(255.0 * alpha).astype(np.uint32)
    rgba = pack_rgba(rgb[:, 0], rgb[:, 1], rgb[:, 2], a8)
    return Scene(v=v, rgba=rgba, width=W, height=H, camera=cam, name=name)


# The paper's workloads, re-created synthetically (shapes, sizes and densities
# follow the configurations the benchmark is quoted on).
RECIPES: Dict[str, Recipe] = {
    # 256x256, 1k quads of 4-40 px, z in [1, 10], alpha U[0.2, 0.8]: tiny frame
    "c1": Recipe(256, 256, 1_000, 0, False, 0.0, (1.0, 10.0), (4.0, 40.0), (0.2, 0.8)),
    # 1280x720, 200k quads of 2-8 px uniformly over the screen, z in [1, 50]
    "c2": Recipe(1280, 720, 200_000, 1, False, 0.0, (1.0, 50.0), (2.0, 8.0), (0.1, 0.9)),
    # the same with 4-16 px sides: mean depth complexity about 11
    "c2b": Recipe(1280, 720, 200_000, 1, False, 0.0, (1.0, 50.0), (4.0, 16.0), (0.1, 0.9)),
    # 1920x1080, 1M quads in a Gaussian cloud (sigma 0.15 screen), 1-30 px,
    # alpha U[0.05, 0.5]: hundreds of layers at the centre
    "c3": Recipe(1920, 1080, 1_000_000, 2, True, 0.15, (1.0, 10.0), (1.0, 30.0), (0.05, 0.5)),
    # the same cloud with alpha U[0.8, 1.0]: mostly opaque layers, where the
    # transmittance cutoff (the paper's alpha threshold experiments) pays
    "c3o": Recipe(1920, 1080, 1_000_000, 2, True, 0.15, (1.0, 10.0), (1.0, 30.0), (0.8, 1.0)),
}

RESOLUTIONS: List[Tuple[int, int]] = [(256, 256), (640, 480), (1280, 720), (1920, 1080)]


def scene(name: str) -> Scene:
    return generate(RECIPES[name], name)


def mixed_recipe(seed: int) -> Recipe:
    """One frame of a mixed batch: resolution from a fixed set, quad count
    log-uniform in [1e3, 5e5], and the shape of one of the three base workloads
    at that resolution and count."""
    rng = np.random.default_rng(seed)
    W, H = RESOLUTIONS[int(rng.integers(0, len(RESOLUTIONS)))]
    n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(5e5)))))
    base = ["c1", "c2", "c3"][int(rng.integers(0, 3))]
    b = RECIPES[base]
    return Recipe(W, H, n, seed, b.gaussian, b.sigma, b.z, b.side, b.alpha)


def mixed_scene(seed: int) -> Scene:
    return generate(mixed_recipe(seed), f"mix{seed}")


def small(width: int, height: int, n: int, seed: int, side=(2.0, 12.0), z=(1.0, 10.0),
          alpha=(0.1, 0.9), gaussian: bool = False, sigma: float = 0.15) -> Scene:
    """A small random scene for tests."""
    return generate(Recipe(width, height, n, seed, gaussian, sigma, z, side, alpha),
                    f"small{width}x{height}n{n}s{seed}")


def screen_quad(corners_px, z, width: int, height: int,
                cam: Camera | None = None) -> np.ndarray:
    """World-space vertices (float32 [4, 3]) of a fronto-parallel quad whose
    corners project to the given pixel coordinates at view depth z, for an
    identity camera.  Used to build hand-checked scenes."""
    cam = cam or Camera()
    f = focal_pixels(height, cam.fov_y)
    cx, cy = 0.5 * width, 0.5 * height
    out = np.zeros((4, 3), np.float32)
    for k, (px, py) in enumerate(corners_px):
        zz = z[k] if isinstance(z, (list, tuple)) else z
        out[k] = ((px - cx) * zz / f, -(py - cy) * zz / f, zz)
    return out


def from_quads(quads: List[Tuple[np.ndarray, int]], width: int, height: int,
               cam: Camera | None = None, name: str = "hand") -> Scene:
    v = np.stack([q[0] for q in quads]).astype(np.float32) if quads else np.zeros((0, 4, 3), np.float32)
    rgba = np.array([q[1] for q in quads], dtype=np.uint32)
    return Scene(v=v, rgba=rgba, width=width, height=height, camera=cam or Camera(), name=name)


def twisted(width: int, height: int, n: int, seed: int, extent=(2.0, 10.0),
            depths=(0.5, 1.0, 20.0, 60.0)) -> Scene:
    """Non-planar quads: four corners drawn independently around a random
    centre, each at a view depth drawn from `depths`.  The plane fitted to
    such a quad can pass behind the camera over part of its screen area, so
    these frames hold fragments whose depth key is clamped to zero."""
    rng = np.random.default_rng(seed)
    quads = []
    for _ in range(n):
        cx, cy = rng.uniform(0.0, width), rng.uniform(0.0, height)
        e = rng.uniform(*extent)
        corners = [(cx + rng.uniform(-e, e), cy + rng.uniform(-e, e)) for _ in range(4)]
        zs = [float(z) for z in rng.choice(np.asarray(depths, np.float64), 4)]
        rgb = rng.integers(0, 256, 3)
        rgba = int(pack_rgba(int(rgb[0]), int(rgb[1]), int(rgb[2]), int(rng.integers(20, 236))))
        quads.append((screen_quad(corners, zs, width, height), rgba))
    return from_quads(quads, width, height, name=f"twisted{width}x{height}n{n}s{seed}")


def with_long_quads(base: Scene, n: int, seed: int, length=(300.0, 700.0), width=(3.0, 8.0),
                    z=(1.0, 50.0), alpha=(0.1, 0.9)) -> Scene:
    """The base scene plus n long thin fronto-parallel quads turned in the
    screen plane at uniform angles (drawn vectorised: centre pair, length,
    width, angle, depth, RGB, alpha).  Their bboxes span many bins that their
    area never reaches: the workload of the large-primitive binning path."""
    rng = np.random.default_rng(seed)
    W, H = base.width, base.height
    cxy = rng.uniform(0.0, 1.0, (n, 2)) * np.array([W, H])
    L = rng.uniform(*length, n)
    T = rng.uniform(*width, n)
    th = rng.uniform(0.0, math.pi, n)
    zz = rng.uniform(*z, n)
    rgb = rng.integers(0, 256, (n, 3))
    a8 = np.rint(255.0 * rng.uniform(*alpha, n)).astype(np.uint32)
    u = np.stack([np.cos(th), np.sin(th)], 1)
    v = np.stack([-np.sin(th), np.cos(th)], 1)
    f = focal_pixels(H, base.camera.fov_y)
    quads = np.zeros((n, 4, 3), np.float64)
    for k, (su, sv) in enumerate(((-1, -1), (1, -1), (1, 1), (-1, 1))):
        p = cxy + (su * L / 2)[:, None] * u + (sv * T / 2)[:, None] * v
        quads[:, k, 0] = (p[:, 0] - 0.5 * W) * zz / f
        quads[:, k, 1] = -(p[:, 1] - 0.5 * H) * zz / f
        quads[:, k, 2] = zz
    rgba = pack_rgba(rgb[:, 0], rgb[:, 1], rgb[:, 2], a8)
    return Scene(v=np.concatenate([base.v, quads.astype(np.float32)]),
                 rgba=np.concatenate([base.rgba, rgba.astype(np.uint32)]),
                 width=W, height=H, camera=base.camera, name=f"{base.name}+{n}long")
