"""Seeded synthetic stereo inputs shared by the CPU oracle tests, the GPU parity
tests and the benchmark.

This module holds no part of the matching method (no Census, no cost, no
aggregation, no disparity selection).  It only paints scenes: a left-view
disparity field made of planes, a fractal texture per plane, the right view by
forward-splatting the left view along image rows (a rectified pair, so a left
pixel x with disparity d lands on right pixel x - d, the convention of the
paper's matching equation in section 3.1.2), and a per-view photometric change
plus Gaussian noise.

Every function takes an explicit seed or ``numpy.random.Generator``; nothing
reads global random state.  Seeds follow ``seed = 1000 * config + pair``
(and ``+ 100000 * camera`` for the multi-camera stream).

Workload recipes (the paper's own evaluation used KITTI Stereo 2015 crops, a
dataset not available here; these seeded scenes stand in for it at the same
frame shapes):

* ``small``  320x240, D=64: background d in [0,15] plus 6 fronto-parallel
  rectangles with integer d in [0,63]; no gain/offset change, noise sigma 2.
* ``kitti``  1242x375, D=128: background plane plus 8-20 slanted planes
  d = a*x + b*y + c (|a|,|b| <= 0.05) clamped to [0, D-1]; per-view gain
  0.9-1.1, offset +-10, noise sigma 2.
* ``large``  1920x1080, D=256: 30-50 slanted planes plus 2-6 thin
  fronto-parallel poles (width 4-12 px, height 30-100 % of H, d in
  [0.7 D, D-1]).
* ``paper``  640x360, D=60: the paper's own frame size and disparity range,
  slanted planes as in ``kitti``.
* ``mixed``  batch of pairs with sizes drawn from {320x240, 640x480,
  1242x375, 1280x720} and D from {64, 128}.
* ``camera`` frames of a moving scene: planes drift 0-3 px per frame.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "fractal_texture", "Scene", "render_pair", "make_pair", "mixed_batch_specs",
    "camera_frame", "random_image", "random_cost", "poisson_trace", "RECIPES", "rectification_maps",
]

# (width, height, max_disp) of each named workload.
RECIPES = {
    "small": (320, 240, 64),
    "kitti": (1242, 375, 128),
    "large": (1920, 1080, 256),
    "paper": (640, 360, 60),
    "vga": (640, 480, 128),
}


def _smoothstep(t: np.ndarray) -> np.ndarray:
    return t * t * (3.0 - 2.0 * t)


def fractal_texture(rng: np.random.Generator, h: int, w: int,
                    cells=(32, 16, 8, 4, 2, 1)) -> np.ndarray:
    """Value noise summed over octaves (lattice cell sizes ``cells`` pixels,
    amplitude halving per octave), smoothstep-bilinear interpolation, mapped
    affinely to mean 128 and standard deviation 48 (float64, not clipped)."""
    acc = np.zeros((h, w), np.float64)
    amp = 1.0
    ys = np.arange(h, dtype=np.float64)
    xs = np.arange(w, dtype=np.float64)
    for c in cells:
        gh, gw = h // c + 2, w // c + 2
        lat = rng.random((gh, gw))
        fy, fx = ys / c, xs / c
        iy, ix = np.floor(fy).astype(np.int64), np.floor(fx).astype(np.int64)
        ty, tx = _smoothstep(fy - iy)[:, None], _smoothstep(fx - ix)[None, :]
        a = lat[iy][:, ix]
        b = lat[iy][:, ix + 1]
        cc = lat[iy + 1][:, ix]
        d = lat[iy + 1][:, ix + 1]
        acc += amp * ((a * (1 - tx) + b * tx) * (1 - ty) + (cc * (1 - tx) + d * tx) * ty)
        amp *= 0.5
    sd = acc.std()
    if sd == 0:
        return np.full((h, w), 128.0)
    return 128.0 + 48.0 * (acc - acc.mean()) / sd


@dataclasses.dataclass
class Plane:
    x0: int
    y0: int
    x1: int  # exclusive
    y1: int  # exclusive
    a: float
    b: float
    c: float
    vx: float = 0.0  # horizontal drift in px / frame (camera streams)


@dataclasses.dataclass
class Scene:
    width: int
    height: int
    max_disp: int
    planes: list  # painted in list order; later planes occlude earlier ones
    gain: tuple = (1.0, 1.0)
    offset: tuple = (0.0, 0.0)
    sigma: float = 2.0
    seed: int = 0


def _plane_disp(p: Plane, xs, ys, D):
    return np.clip(p.a * xs + p.b * ys + p.c, 0.0, D - 1.0)


def _slanted(rng, W, H, D, n, dlo=0.0, dhi=None, slope=0.05):
    dhi = D - 1.0 if dhi is None else dhi
    out = []
    for _ in range(n):
        pw = int(rng.integers(max(4, W // 10), max(5, W // 3) + 1))
        ph = int(rng.integers(max(4, H // 10), max(5, H // 3) + 1))
        x0 = int(rng.integers(0, max(1, W - pw)))
        y0 = int(rng.integers(0, max(1, H - ph)))
        a = float(rng.uniform(-slope, slope))
        b = float(rng.uniform(-slope, slope))
        cx, cy = x0 + pw / 2, y0 + ph / 2
        dc = float(rng.uniform(dlo, dhi))
        out.append(Plane(x0, y0, x0 + pw, y0 + ph, a, b, dc - a * cx - b * cy))
    return out


def make_scene(recipe: str, seed: int, width=None, height=None, max_disp=None) -> Scene:
    """Draw the random scene description of a named recipe."""
    W0, H0, D0 = RECIPES.get(recipe, (None, None, None))
    W = width or W0
    H = height or H0
    D = max_disp or D0
    rng = np.random.default_rng(seed)
    if recipe == "small":
        planes = [Plane(0, 0, W, H, 0.0, 0.0, float(rng.integers(0, 16)))]
        for _ in range(6):
            pw = int(rng.integers(max(1, W // 10), max(2, W // 3) + 1))
            ph = int(rng.integers(max(1, H // 10), max(2, H // 3) + 1))
            x0 = int(rng.integers(0, max(1, W - pw)))
            y0 = int(rng.integers(0, max(1, H - ph)))
            planes.append(Plane(x0, y0, x0 + pw, y0 + ph, 0.0, 0.0,
                                float(rng.integers(0, min(64, D)))))
        gain, off = (1.0, 1.0), (0.0, 0.0)
    else:
        bg_a = float(rng.uniform(-0.01, 0.01))
        bg_b = float(rng.uniform(0.0, 0.04))
        planes = [Plane(0, 0, W, H, bg_a, bg_b, float(rng.uniform(0, D * 0.2)))]
        if recipe == "large":
            planes += _slanted(rng, W, H, D, int(rng.integers(30, 51)))
        else:
            planes += _slanted(rng, W, H, D, int(rng.integers(8, 21)))
        if recipe == "large":
            for _ in range(int(rng.integers(2, 7))):
                pw = int(rng.integers(4, 13))
                ph = int(rng.uniform(0.3, 1.0) * H)
                x0 = int(rng.integers(0, W - pw))
                y0 = int(rng.integers(0, H - ph + 1))
                planes.append(Plane(x0, y0, x0 + pw, y0 + ph, 0.0, 0.0,
                                    float(rng.uniform(0.7 * D, D - 1.0))))
        gain = (float(rng.uniform(0.9, 1.1)), float(rng.uniform(0.9, 1.1)))
        off = (float(rng.uniform(-10, 10)), float(rng.uniform(-10, 10)))
    # paint far to near: ascending mean disparity, so nearer planes occlude
    def mean_d(p):
        return float(_plane_disp(p, np.array([(p.x0 + p.x1) / 2]),
                                 np.array([(p.y0 + p.y1) / 2]), D)[0])
    planes = [planes[0]] + sorted(planes[1:], key=mean_d)
    return Scene(W, H, D, planes, gain, off, 2.0, seed)


def render_pair(scene: Scene, frame: int = 0):
    """Render (left uint8, right uint8, gt int32 with -1 where undefined)."""
    W, H, D = scene.width, scene.height, scene.max_disp
    rng = np.random.default_rng(scene.seed * 7919 + 17 + frame)
    disp = np.zeros((H, W), np.float64)
    left = np.zeros((H, W), np.float64)
    for p in scene.planes:
        shift = int(round(p.vx * frame))
        x0, x1 = max(0, p.x0 + shift), min(W, p.x1 + shift)
        y0, y1 = max(0, p.y0), min(H, p.y1)
        if x1 <= x0 or y1 <= y0:
            continue
        tex = fractal_texture(rng, y1 - y0, x1 - x0)
        ys, xs = np.mgrid[y0:y1, x0:x1].astype(np.float64)
        disp[y0:y1, x0:x1] = _plane_disp(p, xs - shift, ys, D)
        left[y0:y1, x0:x1] = tex
    fill = fractal_texture(rng, H, W)
    dint = np.rint(disp).astype(np.int64)
    # forward splat with a z-buffer: the larger disparity wins a right pixel
    right = fill.copy()
    zbuf = np.full((H, W), -1, np.int64)
    yy, xx = np.mgrid[0:H, 0:W]
    xr = xx - dint
    ok = xr >= 0
    np.maximum.at(zbuf, (yy[ok], xr[ok]), dint[ok])
    visible = np.zeros((H, W), bool)
    visible[ok] = zbuf[yy[ok], xr[ok]] == dint[ok]
    # at most one source pixel per (row, x_r, d), so this write is unambiguous
    right[yy[visible], xr[visible]] = left[visible]
    gt = np.where(visible, dint, -1).astype(np.int32)

    def photometric(img, g, o):
        n = rng.normal(0.0, scene.sigma, img.shape)
        return np.clip(np.rint(g * img + o + n), 0, 255).astype(np.uint8)

    L = photometric(left, scene.gain[0], scene.offset[0])
    R = photometric(right, scene.gain[1], scene.offset[1])
    return L, R, gt


def make_pair(recipe: str, seed: int, width=None, height=None, max_disp=None):
    """Seeded pair of a named recipe: (left, right, gt)."""
    return render_pair(make_scene(recipe, seed, width, height, max_disp))


MIXED_SIZES = [(320, 240), (640, 480), (1242, 375), (1280, 720)]


def mixed_batch_specs(n: int = 32, seed: int = 2000):
    """(width, height, max_disp, seed) for a batch of uneven pairs."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        w, h = MIXED_SIZES[int(rng.integers(0, len(MIXED_SIZES)))]
        d = int(rng.choice([64, 128]))
        out.append((w, h, d, seed + i))
    return out


def camera_scene(camera: int, base_seed: int = 3000) -> Scene:
    """Scene of one simulated camera; cameras 0-1 are 640x480, 2-3 1242x375."""
    W, H = (640, 480) if camera % 4 < 2 else (1242, 375)
    sc = make_scene("kitti", base_seed + 100000 * camera, W, H, 128)
    rng = np.random.default_rng(base_seed + 100000 * camera + 1)
    for p in sc.planes[1:]:
        p.vx = float(rng.uniform(0, 3)) * (1 if rng.random() < 0.5 else -1)
    return sc


def camera_frame(camera: int, frame: int, base_seed: int = 3000):
    return render_pair(camera_scene(camera, base_seed), frame)


def poisson_trace(n_cameras: int, fps: float, seconds: float, seed: int):
    """Sorted arrival list [(t_seconds, camera, frame_index)] with exponential
    inter-arrival gaps of mean 1/fps per camera."""
    rng = np.random.default_rng(seed)
    ev = []
    for cam in range(n_cameras):
        t, k = 0.0, 0
        while True:
            t += float(rng.exponential(1.0 / fps))
            if t >= seconds:
                break
            ev.append((t, cam, k))
            k += 1
    ev.sort()
    return ev


def rectification_maps(w: int, h: int, src_w: int, src_h: int, seed: int, angle_deg: float = 1.5,
                       k1: float = -0.05):
    """Integer remap tables (uint16 [h][w] source column, source row) of a
    synthetic calibration: a small rotation about the image centre, a radial
    distortion term k1 and a random sub-pixel offset, rounded to the nearest
    source pixel.  Entries that fall outside the raw image are set to 65535
    (no source pixel)."""
    rng = np.random.default_rng(seed)
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    u, v = (xs - cx) / max(cx, 1.0), (ys - cy) / max(cy, 1.0)
    r2 = u * u + v * v
    t = np.deg2rad(angle_deg * float(rng.uniform(0.5, 1.0)))
    ud = (u * np.cos(t) - v * np.sin(t)) * (1 + k1 * r2)
    vd = (u * np.sin(t) + v * np.cos(t)) * (1 + k1 * r2)
    sx = ud * (src_w - 1) / 2.0 + (src_w - 1) / 2.0 + float(rng.uniform(-0.5, 0.5))
    sy = vd * (src_h - 1) / 2.0 + (src_h - 1) / 2.0 + float(rng.uniform(-0.5, 0.5))
    mx, my = np.rint(sx), np.rint(sy)
    out = (mx < 0) | (my < 0) | (mx >= src_w) | (my >= src_h)
    mx[out] = 65535
    my[out] = 65535
    return mx.astype(np.uint16), my.astype(np.uint16)


def random_image(rng: np.random.Generator, h: int, w: int, levels: int = 256) -> np.ndarray:
    """Uniform random uint8 image with values in [0, levels)."""
    return rng.integers(0, levels, size=(h, w), dtype=np.uint8)


def random_cost(rng: np.random.Generator, h: int, w: int, d: int, maxc: int) -> np.ndarray:
    """Uniform random uint16 cost volume [h][w][d] with values in [0, maxc]."""
    return rng.integers(0, maxc + 1, size=(h, w, d), dtype=np.uint16)
