"""Seeded synthetic inputs for the masked Gaussian-splatting rasterizer.

This module only draws inputs: Gaussian parameter sets, pinhole cameras,
building masks and upstream gradients.  It holds none of the rasterizer's
arithmetic (no projection of Gaussians, no colour evaluation, no
compositing), so that the GPU path and the FP64 oracle can both consume it
without sharing any of the method.

Everything is drawn in FP64 with ``numpy.random.default_rng(seed)`` and cast
to FP32; the FP32 arrays are the canonical inputs for both sides.

Layouts (planar structure-of-arrays, the layout the library consumes):
  means           float32 [3][n]
  log_scales      float32 [3][n]      natural log of the per-axis scale
  quats           float32 [4][n]      (w, x, y, z), any non-zero norm
  opacity_logits  float32 [n]
  sh              float32 [(deg+1)^2][3][n]
Cameras map world to camera coordinates as x_c = R x_w + t (R row-major,
camera looks along +z, image x right, image y down).  Masks are uint8 [H][W]
with 1 = building pixel.

The workloads follow the paper's setting (per-building-group optimisation
at the original aerial resolution, Sec. 4.1 and Sec. 5.1); the datasets
themselves are not available, so these generators stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
from typing import List, Optional

import numpy as np

# 2*sqrt(pi): a degree-0 SH coefficient of (u - 0.5) * 2*sqrt(pi) encodes a
# degree-0 colour of u under the real orthonormal basis with +0.5 offset.
_DC_FROM_COLOUR = 2.0 * math.sqrt(math.pi)


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # float32 [3,3], world -> camera rotation (row-major)
    t: np.ndarray  # float32 [3]

    def as_dict(self):
        return dict(width=self.width, height=self.height, fx=self.fx, fy=self.fy,
                    cx=self.cx, cy=self.cy, R=self.R, t=self.t)


@dataclass
class GaussianSet:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def arrays(self):
        return dict(means=self.means, log_scales=self.log_scales, quats=self.quats,
                    opacity_logits=self.opacity_logits, sh=self.sh)


@dataclass
class Render:
    set_index: int
    camera: Camera
    mask: Optional[np.ndarray]  # uint8 [H][W] or None (= every pixel)


@dataclass
class Scene:
    sets: List[GaussianSet]
    renders: List[Render]
    name: str = ""
    info: dict = field(default_factory=dict)


# ---------------------------------------------------------------- helpers

def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def random_unit_quats(rng, n):
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def sh_coefficients(rng, n, degree, dc_colour=None, sigma_rest=0.1):
    """SH coefficients [(deg+1)^2][3][n]: degree-0 colour U[0,1], rest N(0, sigma)."""
    k = (degree + 1) ** 2
    sh = np.zeros((k, 3, n))
    if dc_colour is None:
        dc_colour = rng.uniform(0.0, 1.0, size=(3, n))
    sh[0] = (dc_colour - 0.5) * _DC_FROM_COLOUR
    if k > 1:
        sh[1:] = rng.normal(0.0, sigma_rest, size=(k - 1, 3, n))
    return sh


def pinhole(width, height, fx, fy, cx=None, cy=None, R=None, t=None) -> Camera:
    cx = width / 2.0 if cx is None else cx
    cy = height / 2.0 if cy is None else cy
    R = np.eye(3) if R is None else R
    t = np.zeros(3) if t is None else t
    return Camera(int(width), int(height), float(np.float32(fx)), float(np.float32(fy)),
                  float(np.float32(cx)), float(np.float32(cy)), _f32(R), _f32(t))


def look_at(eye, target, up=(0.0, 0.0, 1.0)):
    """World->camera (R, t) for a camera at ``eye`` looking at ``target``.

    Camera rows are (right, down, forward) so that image x goes right and
    image y goes down.
    """
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, dtype=np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ eye
    return R, t


def rect_union_mask(rng, width, height, n_rects=20, target=0.40, tol=0.02,
                    frac=(0.08, 0.24), max_tries=10000):
    """Union of axis-aligned rectangles; redrawn until coverage is target +- tol."""
    for _ in range(max_tries):
        m = np.zeros((height, width), dtype=np.uint8)
        cxs = rng.uniform(0, width, n_rects)
        cys = rng.uniform(0, height, n_rects)
        ws = rng.uniform(frac[0], frac[1], n_rects) * width
        hs = rng.uniform(frac[0], frac[1], n_rects) * height
        for cx, cy, w, h in zip(cxs, cys, ws, hs):
            x0 = int(max(0, math.floor(cx - w / 2)))
            x1 = int(min(width, math.ceil(cx + w / 2)))
            y0 = int(max(0, math.floor(cy - h / 2)))
            y1 = int(min(height, math.ceil(cy + h / 2)))
            m[y0:y1, x0:x1] = 1
        cov = m.mean()
        if abs(cov - target) <= tol:
            return m
    raise RuntimeError("could not reach the requested mask coverage")


def _rot_to_quat(Rm):
    """Rotation matrices [n,3,3] -> unit quaternions [4,n] (w,x,y,z), Shepperd's method."""
    n = Rm.shape[0]
    q = np.zeros((4, n))
    tr = Rm[:, 0, 0] + Rm[:, 1, 1] + Rm[:, 2, 2]
    cand = np.stack([tr, Rm[:, 0, 0], Rm[:, 1, 1], Rm[:, 2, 2]], axis=1)
    k = np.argmax(cand, axis=1)
    for case in range(4):
        sel = k == case
        if not np.any(sel):
            continue
        R = Rm[sel]
        if case == 0:
            s = np.sqrt(1.0 + R[:, 0, 0] + R[:, 1, 1] + R[:, 2, 2]) * 2
            w = 0.25 * s
            x = (R[:, 2, 1] - R[:, 1, 2]) / s
            y = (R[:, 0, 2] - R[:, 2, 0]) / s
            z = (R[:, 1, 0] - R[:, 0, 1]) / s
        elif case == 1:
            s = np.sqrt(1.0 + R[:, 0, 0] - R[:, 1, 1] - R[:, 2, 2]) * 2
            w = (R[:, 2, 1] - R[:, 1, 2]) / s
            x = 0.25 * s
            y = (R[:, 0, 1] + R[:, 1, 0]) / s
            z = (R[:, 0, 2] + R[:, 2, 0]) / s
        elif case == 2:
            s = np.sqrt(1.0 + R[:, 1, 1] - R[:, 0, 0] - R[:, 2, 2]) * 2
            w = (R[:, 0, 2] - R[:, 2, 0]) / s
            x = (R[:, 0, 1] + R[:, 1, 0]) / s
            y = 0.25 * s
            z = (R[:, 1, 2] + R[:, 2, 1]) / s
        else:
            s = np.sqrt(1.0 + R[:, 2, 2] - R[:, 0, 0] - R[:, 1, 1]) * 2
            w = (R[:, 1, 0] - R[:, 0, 1]) / s
            x = (R[:, 0, 2] + R[:, 2, 0]) / s
            y = (R[:, 1, 2] + R[:, 2, 1]) / s
            z = 0.25 * s
        q[:, sel] = np.stack([w, x, y, z])
    return q


# ------------------------------------------------------ uniform-cube scenes

def cube_set(seed, n, sh_degree=0, extent=(1.0, 1.0, 1.0), depth=4.0,
             scale_range=(0.005, 0.05), logit_mu=0.0, logit_sigma=1.0,
             normalise_quats=True) -> GaussianSet:
    """Means uniform in a box centred ``depth`` along +z, log-uniform scales,
    uniform rotations, opacity = sigmoid(N(mu, sigma)), SH colour as in the
    paper's 3DGS setting (degree-0 colour U[0,1], higher bands N(0, 0.1))."""
    rng = np.random.default_rng(seed)
    ex = np.asarray(extent, dtype=np.float64)[:, None]
    means = rng.uniform(-1.0, 1.0, size=(3, n)) * ex
    means[2] += depth
    log_scales = rng.uniform(math.log(scale_range[0]), math.log(scale_range[1]), size=(3, n))
    quats = random_unit_quats(rng, n)
    if not normalise_quats:
        quats = quats * rng.uniform(0.5, 2.0, size=(1, n))
    logits = rng.normal(logit_mu, logit_sigma, size=n)
    sh = sh_coefficients(rng, n, sh_degree)
    return GaussianSet(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), sh_degree)


def config1(seed=1) -> Scene:
    """10k Gaussians, 256x256, SH degree 0, full mask, 16x16 tiles."""
    s = cube_set(seed, 10_000, sh_degree=0)
    cam = pinhole(256, 256, 256.0, 256.0)
    return Scene([s], [Render(0, cam, None)], name="cfg1-10k-256x256-sh0-full")


def config2(seed=2, n=1_000_000) -> Scene:
    """1M Gaussians, 1920x1080, SH degree 3, ~40% rectangle-union mask."""
    s = cube_set(seed, n, sh_degree=3, extent=(4.0, 2.25, 1.0))
    cam = pinhole(1920, 1080, 960.0, 960.0)
    mask = rect_union_mask(np.random.default_rng(seed + 1), 1920, 1080)
    return Scene([s], [Render(0, cam, mask)], name="cfg2-1M-1920x1080-sh3-mask40")


def small_scene(seed, n=64, width=70, height=50, sh_degree=1, mask_kind="rects",
                n_views=1, depth=4.0, logit_mu=0.0, normalise_quats=False) -> Scene:
    """Tiny random scenes for parity and edge cases (ragged image sizes)."""
    rng = np.random.default_rng(seed + 7)
    ext = (1.2 * width / max(width, height), 1.2 * height / max(width, height), 1.0)
    s = cube_set(seed, n, sh_degree=sh_degree, extent=ext, depth=depth,
                 scale_range=(0.02, 0.15), logit_mu=logit_mu,
                 normalise_quats=normalise_quats)
    f = 0.9 * max(width, height)
    renders = []
    for v in range(n_views):
        if v == 0:
            R, t = np.eye(3), np.zeros(3)
        else:
            ang = 0.25 * v
            c, si = math.cos(ang), math.sin(ang)
            R = np.array([[c, 0, -si], [0, 1, 0], [si, 0, c]])
            # keep the scene centre (0,0,depth) in front of the camera
            centre = np.array([0.0, 0.0, depth])
            t = np.array([0.0, 0.0, depth]) - R @ centre
        cam = pinhole(width, height, f, f * rng.uniform(0.9, 1.1),
                      width / 2 + rng.uniform(-3, 3), height / 2 + rng.uniform(-3, 3), R, t)
        if mask_kind == "full":
            mask = None
        elif mask_kind == "empty":
            mask = np.zeros((height, width), np.uint8)
        elif mask_kind == "random":
            mask = (rng.uniform(size=(height, width)) < 0.5).astype(np.uint8)
        else:
            mask = np.zeros((height, width), np.uint8)
            for _ in range(4):
                x0 = rng.integers(0, width)
                y0 = rng.integers(0, height)
                mask[y0:y0 + rng.integers(4, max(5, height // 2)),
                     x0:x0 + rng.integers(4, max(5, width // 2))] = 1
        renders.append(Render(0, cam, mask))
    return Scene([s], renders, name=f"small-{seed}-{n}-{width}x{height}")


# ------------------------------------------------------- facade scenes

def _boxes(rng, n_boxes, half_extent, foot=(10.0, 60.0), height=(10.0, 120.0)):
    cx = rng.uniform(-half_extent, half_extent, n_boxes)
    cy = rng.uniform(-half_extent, half_extent, n_boxes)
    w = rng.uniform(foot[0], foot[1], n_boxes)
    d = rng.uniform(foot[0], foot[1], n_boxes)
    h = rng.uniform(height[0], height[1], n_boxes)
    return np.stack([cx, cy, w, d, h], axis=1)


def _faces(boxes):
    """Per face: corner, e1, e2 (e1 x e2 = outward normal), extents (L1, L2)."""
    X, Y, Z = np.eye(3)
    out = []
    for cx, cy, w, d, h in boxes:
        x0, x1, y0, y1 = cx - w / 2, cx + w / 2, cy - d / 2, cy + d / 2
        out.append(((x0, y0, h), X, Y, w, d))   # roof, +z
        out.append(((x1, y0, 0), Y, Z, d, h))   # +x wall
        out.append(((x0, y0, 0), Z, Y, h, d))   # -x wall
        out.append(((x0, y1, 0), Z, X, h, w))   # +y wall
        out.append(((x0, y0, 0), X, Z, w, h))   # -y wall
    corner = np.array([f[0] for f in out], dtype=np.float64)
    e1 = np.array([f[1] for f in out])
    e2 = np.array([f[2] for f in out])
    L = np.array([[f[3], f[4]] for f in out], dtype=np.float64)
    return corner, e1, e2, L


def facade_set(rng, boxes, n, sh_degree=3, chunk=2_000_000) -> GaussianSet:
    corner, e1, e2, L = _faces(boxes)
    area = L[:, 0] * L[:, 1]
    face = rng.choice(len(area), size=n, p=area / area.sum())
    means = np.empty((3, n))
    log_scales = np.empty((3, n))
    quats = np.empty((4, n))
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        f = face[a:b]
        m = b - a
        u = rng.uniform(0, 1, m)
        v = rng.uniform(0, 1, m)
        means[:, a:b] = (corner[f] + (u * L[f, 0])[:, None] * e1[f]
                         + (v * L[f, 1])[:, None] * e2[f]).T
        s12 = np.exp(rng.uniform(math.log(0.15), math.log(0.6), size=(2, m)))
        s3 = 0.01 * np.minimum(s12[0], s12[1])
        log_scales[:, a:b] = np.log(np.concatenate([s12, s3[None]], axis=0))
        th = rng.uniform(0, 2 * math.pi, m)
        c, s = np.cos(th)[:, None], np.sin(th)[:, None]
        a1 = c * e1[f] + s * e2[f]
        a2 = -s * e1[f] + c * e2[f]
        a3 = np.cross(e1[f], e2[f])
        Rm = np.stack([a1, a2, a3], axis=2)  # columns are the local axes
        quats[:, a:b] = _rot_to_quat(Rm)
    logits = rng.normal(1.0, 1.0, size=n)
    sh = sh_coefficients(rng, n, sh_degree)
    return GaussianSet(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), sh_degree)


def _box_corners(box):
    cx, cy, w, d, h = box
    xs = (cx - w / 2, cx + w / 2)
    ys = (cy - d / 2, cy + d / 2)
    zs = (0.0, h)
    return np.array([(x, y, z) for x in xs for y in ys for z in zs])


def _hull2d(p):
    """Convex hull (counter-clockwise in image coordinates) by monotone chain."""
    pts = sorted(map(tuple, p))
    if len(pts) <= 2:
        return np.array(pts)

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])
    lower, upper = [], []
    for q in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], q) <= 0:
            lower.pop()
        lower.append(q)
    for q in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], q) <= 0:
            upper.pop()
        upper.append(q)
    return np.array(lower[:-1] + upper[:-1])


def box_mask(boxes, cam: Camera):
    """Union of the convex hulls of each box's 8 corners projected by a
    pinhole camera, sampled at pixel centres (u+0.5, v+0.5)."""
    W, H = cam.width, cam.height
    m = np.zeros((H, W), dtype=np.uint8)
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    for box in boxes:
        pc = _box_corners(box) @ R.T + t
        if np.any(pc[:, 2] <= 0.2):
            continue
        uv = np.stack([cam.fx * pc[:, 0] / pc[:, 2] + cam.cx,
                       cam.fy * pc[:, 1] / pc[:, 2] + cam.cy], axis=1)
        hull = _hull2d(uv)
        if len(hull) < 3:
            continue
        x0 = max(0, int(math.floor(hull[:, 0].min() - 0.5)))
        x1 = min(W, int(math.ceil(hull[:, 0].max() + 0.5)))
        y0 = max(0, int(math.floor(hull[:, 1].min() - 0.5)))
        y1 = min(H, int(math.ceil(hull[:, 1].max() + 0.5)))
        if x0 >= x1 or y0 >= y1:
            continue
        px = np.arange(x0, x1) + 0.5
        py = np.arange(y0, y1) + 0.5
        gx, gy = np.meshgrid(px, py)
        inside = np.ones_like(gx, dtype=bool)
        k = len(hull)
        for i in range(k):
            a, b = hull[i], hull[(i + 1) % k]
            inside &= ((b[0] - a[0]) * (gy - a[1]) - (b[1] - a[1]) * (gx - a[0])) >= 0
        m[y0:y1, x0:x1] |= inside.astype(np.uint8)
    return m


def facade_scene(seed, n, n_boxes=200, half_extent=500.0, views=None, sh_degree=3,
                 name="facade") -> Scene:
    rng = np.random.default_rng(seed)
    boxes = _boxes(rng, n_boxes, half_extent)
    s = facade_set(rng, boxes, n, sh_degree)
    renders = []
    for (W, H, f, eye) in views:
        R, t = look_at(eye, (0.0, 0.0, 0.0))
        cam = pinhole(W, H, f, f, W / 2, H / 2, R, t)
        renders.append(Render(0, cam, box_mask(boxes, cam)))
    return Scene([s], renders, name=name, info=dict(boxes=boxes))


def config3(seed=3, n=6_000_000) -> Scene:
    """200 boxes, 6M facade Gaussians, one 45-degree oblique 4000x3000 view."""
    return facade_scene(seed, n, views=[(4000, 3000, 3500.0, (0.0, -500.0, 500.0))],
                        name="cfg3-6M-4000x3000-facade")


def config5(seed=5, n=10_000_000) -> Scene:
    """10M facade Gaussians, two oblique 5472x3648 views (cfg3's field of view)."""
    f = 3500.0 * 5472 / 4000
    return facade_scene(seed, n, views=[(5472, 3648, f, (0.0, -500.0, 500.0)),
                                        (5472, 3648, f, (500.0, 0.0, 500.0))],
                        name="cfg5-10M-2x5472x3648-facade")


def config4(seed=4, n_regions=16, n_min=50_000, n_max=2_000_000, width=1600,
            height=1200, f=1400.0, n_views=4, coverage=(0.3, 0.7), scale=1.0) -> Scene:
    """Batched semantic groups: 16 sub-regions of log-uniform size, 4 views
    each (yaw 0/90/180/270, pitch 45 deg), per-view building masks."""
    sets, renders = [], []
    sizes = []
    for r in range(n_regions):
        rng = np.random.default_rng(400 + r + 1000 * (seed - 4))
        nr = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max))) * scale))
        nr = max(nr, 1)
        for _ in range(1000):
            boxes = _boxes(rng, 8, 100.0)
            cams, masks = [], []
            for v in range(n_views):
                yaw = 2 * math.pi * v / n_views
                eye = (140.0 * math.sin(yaw), -140.0 * math.cos(yaw), 140.0)
                R, t = look_at(eye, (0.0, 0.0, 0.0))
                cam = pinhole(width, height, f, f, width / 2, height / 2, R, t)
                cams.append(cam)
                masks.append(box_mask(boxes, cam))
            cov = [mm.mean() for mm in masks]
            if all(coverage[0] <= c <= coverage[1] for c in cov):
                break
        else:
            raise RuntimeError("no layout met the coverage bounds")
        sets.append(facade_set(rng, boxes, nr))
        for cam, mm in zip(cams, masks):
            renders.append(Render(r, cam, mm))
        sizes.append(nr)
    return Scene(sets, renders, name="cfg4-16x4-1600x1200-facade", info=dict(sizes=sizes))


# ---------------------------------------------------- upstream gradients

# upstream-gradient planes: the rendered outputs, then the soft contributor
# count (drawn last, so the other planes keep their draws)
OUTPUT_CHANNELS = (("rgb", 3), ("normal", 3), ("dist", 1), ("depth", 1), ("alpha", 1), ("count", 1))


def grad_outputs(seed, render: Render, channels=None, scale=None):
    """dL/d(output) planes drawn N(0,1) on masked pixels, zero elsewhere.

    Returns a dict name -> float32 [c][H][W] ([H][W] for 1-channel outputs).
    """
    rng = np.random.default_rng(seed)
    H, W = render.camera.height, render.camera.width
    m = np.ones((H, W), np.float64) if render.mask is None else render.mask.astype(np.float64)
    out = {}
    for name, c in OUTPUT_CHANNELS:
        if channels is not None and name not in channels:
            continue
        g = rng.normal(size=(c, H, W)) * m
        if scale is not None and name in scale:
            g = g * scale[name]
        out[name] = _f32(g if c > 1 else g[0])
    return out


def sample_pixels(seed, render: Render, count):
    """Fixed random sample of masked pixel coordinates (v, u), sorted row-major."""
    rng = np.random.default_rng(seed)
    H, W = render.camera.height, render.camera.width
    m = np.ones((H, W), bool) if render.mask is None else render.mask.astype(bool)
    idx = np.flatnonzero(m.ravel())
    if len(idx) > count:
        idx = np.sort(rng.choice(idx, size=count, replace=False))
    return np.stack([idx // W, idx % W], axis=1)


def crop_windows(seed, render: Render, count=4, size=64):
    """Crops (v0, u0, size) whose centre pixel is masked."""
    rng = np.random.default_rng(seed)
    H, W = render.camera.height, render.camera.width
    m = np.ones((H, W), bool) if render.mask is None else render.mask.astype(bool)
    out = []
    for _ in range(100000):
        v0 = int(rng.integers(0, max(1, H - size)))
        u0 = int(rng.integers(0, max(1, W - size)))
        if m[min(H - 1, v0 + size // 2), min(W - 1, u0 + size // 2)]:
            out.append((v0, u0, size))
            if len(out) == count:
                return out
    return out


def loss_inputs(seed, render: Render):
    """Seeded stand-ins for the rendered planes and a ground-truth image of
    one render (float32): a smooth positive depth surface on masked pixels
    with ~2% holes (depth 0), normals N(0, 1) per component with ~1% exact
    zeros, colours U[0, 1] and a ground truth equal to the colour on ~1% of
    the pixels.  Unmasked pixels hold 0 in rgb, normal and depth."""
    cam = render.camera
    H, W = cam.height, cam.width
    rng = np.random.default_rng(seed)
    m = np.ones((H, W), bool) if render.mask is None else np.asarray(render.mask).astype(bool)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    surf = 4.0 + 0.6 * np.sin(xx / 23.0) * np.cos(yy / 17.0) + 0.002 * xx + rng.uniform(-0.01, 0.01, (H, W))
    depth = np.where(m & (rng.uniform(size=(H, W)) > 0.02), surf, 0.0)
    normal = rng.normal(size=(3, H, W))
    normal[:, rng.uniform(size=(H, W)) < 0.01] = 0.0
    normal *= m[None]
    rgb = rng.uniform(size=(3, H, W)) * m[None]
    gt = rng.uniform(size=(3, H, W))
    same = rng.uniform(size=(H, W)) < 0.01
    gt[:, same] = rgb[:, same]
    return dict(rgb=_f32(rgb), normal=_f32(normal), depth=_f32(depth), gt=_f32(gt))


def load_inputs(seed, render: Render, max_count=60):
    """Seeded stand-ins for a render's per-pixel blended counts (int32) and
    Eq. 9 pixel weights (float32, in [0.1, 3])."""
    cam = render.camera
    rng = np.random.default_rng(seed)
    g = rng.integers(0, max_count, (cam.height, cam.width)).astype(np.int32)
    w = _f32(rng.uniform(0.1, 3.0, (cam.height, cam.width)))
    return g, w


def perturbed(seed, gs: GaussianSet) -> GaussianSet:
    """The set a training run starts from: the generating set plus noise --
    means N(0, 0.1 s) with s the Gaussian's mean axis scale, opacity logits
    N(0, 0.1), SH coefficients N(0, 0.01)."""
    rng = np.random.default_rng(seed)
    s = np.exp(gs.log_scales.astype(np.float64)).mean(0)
    means = gs.means + rng.normal(size=gs.means.shape) * (0.1 * s)[None]
    logits = gs.opacity_logits + rng.normal(scale=0.1, size=gs.opacity_logits.shape)
    sh = gs.sh + rng.normal(scale=0.01, size=gs.sh.shape)
    return GaussianSet(_f32(means), gs.log_scales.copy(), gs.quats.copy(), _f32(logits), _f32(sh), gs.sh_degree)
