"""Seeded synthetic stand-ins for the aerial survey that feeds the building
pipeline around the rasterizer: SfM-like sparse points, oblique views with
coarse building masks, and the per-view depth maps of several rendered
groups.

Like the rest of ``scenes`` this module only draws inputs.  It holds none of
the arithmetic of the steps it feeds (no projection of points into views, no
voting, no clustering, no fusion or volume integration), so the GPU path and
the FP64 oracle can both consume it without sharing any of the method.

The stand-ins follow the paper's setting (Sec. 4.1, Sec. 5.1): a square
kilometre of box buildings photographed by oblique aerial views at the
original 5472 x 3648 resolution; sparse points on roofs and walls (building
points), on the ground and on low clutter (non-building points); coarse
text-prompted building masks that hold every building silhouette but also
view-dependent false detections and a few holes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
from typing import List

import numpy as np

from . import Camera, _boxes, _box_corners, _f32, _faces, _hull2d, look_at, pinhole


@dataclass
class Survey:
    points: np.ndarray          # float32 [3][M] world positions (metres)
    kind: np.ndarray            # int8 [M]: 0 building, 1 ground, 2 clutter (generator truth)
    cameras: List[Camera]
    masks: List[np.ndarray]     # uint8 [H][W] per view, 1 = coarse building pixel
    boxes: np.ndarray           # float64 [n_boxes][5] (cx, cy, w, d, h)
    info: dict = field(default_factory=dict)


def polygon_mask(polys, width, height):
    """Union of convex polygons (vertices counter-clockwise in image
    coordinates, y down) sampled at pixel centres (u+0.5, v+0.5), by row
    spans: O(rows) per polygon instead of O(area)."""
    rows_all, lo_all, hi_all = [], [], []
    for hull in polys:
        if len(hull) < 3:
            continue
        y0 = max(0, int(math.floor(hull[:, 1].min() - 0.5)))
        y1 = min(height, int(math.ceil(hull[:, 1].max() + 0.5)))
        if y0 >= y1:
            continue
        py = np.arange(y0, y1) + 0.5
        lo = np.full(len(py), -np.inf)
        hi = np.full(len(py), np.inf)
        ok = np.ones(len(py), bool)
        k = len(hull)
        for i in range(k):
            a, b = hull[i], hull[(i + 1) % k]
            dx, dy = b[0] - a[0], b[1] - a[1]
            # inside: dx (py - a1) - dy (px - a0) >= 0
            if dy == 0.0:
                ok &= dx * (py - a[1]) >= 0
            else:
                bound = a[0] + dx * (py - a[1]) / dy
                if dy > 0:
                    hi = np.minimum(hi, bound)
                else:
                    lo = np.maximum(lo, bound)
        u0 = np.maximum(np.ceil(lo - 0.5), 0)
        u1 = np.minimum(np.floor(hi - 0.5), width - 1)
        ok &= u0 <= u1
        rows_all.append(np.arange(y0, y1)[ok])
        lo_all.append(u0[ok].astype(np.int64))
        hi_all.append(u1[ok].astype(np.int64))
    diff = np.zeros((height, width + 1), np.int16)
    if rows_all:
        r = np.concatenate(rows_all)
        np.add.at(diff, (r, np.concatenate(lo_all)), 1)
        np.add.at(diff, (r, np.concatenate(hi_all) + 1), -1)
    return (np.cumsum(diff[:, :width], axis=1, dtype=np.int16) > 0).view(np.uint8)


def box_silhouettes(boxes, cam: Camera):
    """Convex hulls of each box's projected corners (boxes wholly in front
    of the camera only), for polygon_mask."""
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    polys = []
    for box in boxes:
        pc = _box_corners(box) @ R.T + t
        if np.any(pc[:, 2] <= 0.2):
            continue
        uv = np.stack([cam.fx * pc[:, 0] / pc[:, 2] + cam.cx, cam.fy * pc[:, 1] / pc[:, 2] + cam.cy], axis=1)
        polys.append(_hull2d(uv))
    return polys


def flight_views(n_views, width, height, f, half_extent, distance):
    """Oblique views on a square grid of ground targets, pitch 45 degrees,
    yaw cycling 0/90/180/270 degrees, camera `distance` metres back and up."""
    k = int(math.ceil(math.sqrt(n_views)))
    g = np.linspace(-half_extent, half_extent, k) if k > 1 else np.zeros(1)
    cams = []
    for i in range(n_views):
        tx, ty = g[i % k], g[(i // k) % k]
        yaw = 0.5 * math.pi * (i % 4)
        eye = (tx + distance * math.sin(yaw), ty - distance * math.cos(yaw), distance)
        R, t = look_at(eye, (tx, ty, 0.0))
        cams.append(pinhole(width, height, f, f, width / 2, height / 2, R, t))
    return cams


def survey(seed, n_points, n_views, width=5472, height=3648, f=4788.0, n_boxes=200, half_extent=500.0,
           distance=300.0, building_share=0.6, ground_share=0.3, false_rects=12, holes=6):
    """Sparse points and coarse masks of an aerial survey.

    Points: `building_share` of them uniform on the roofs and walls of the
    boxes (area-weighted), `ground_share` uniform on the ground outside the
    footprints, the rest low clutter (z in [0, 12] m) over the ground; then
    shuffled (no spatial order).  Masks: union of every box silhouette,
    plus `false_rects` random rectangles per view (1-6% of each image side
    squared: false detections, different in every view), minus `holes`
    small rectangles per view (missed building pixels)."""
    rng = np.random.default_rng(seed)
    boxes = _boxes(rng, n_boxes, half_extent)
    nb = int(round(building_share * n_points))
    ng = int(round(ground_share * n_points))
    nc = n_points - nb - ng
    corner, e1, e2, L = _faces(boxes)
    area = L[:, 0] * L[:, 1]
    face = rng.choice(len(area), size=nb, p=area / area.sum())
    u = rng.uniform(0, 1, nb)
    v = rng.uniform(0, 1, nb)
    pb = corner[face] + (u * L[face, 0])[:, None] * e1[face] + (v * L[face, 1])[:, None] * e2[face]

    def outside_footprints(p):
        keep = np.ones(len(p), bool)
        for cx, cy, w, d, _ in boxes:
            keep &= ~((np.abs(p[:, 0] - cx) < w / 2) & (np.abs(p[:, 1] - cy) < d / 2))
        return keep

    def ground_like(n, zlo, zhi):
        out = np.zeros((0, 3))
        while len(out) < n:
            m = 2 * (n - len(out)) + 16
            p = np.stack([rng.uniform(-1.1 * half_extent, 1.1 * half_extent, m),
                          rng.uniform(-1.1 * half_extent, 1.1 * half_extent, m),
                          rng.uniform(zlo, zhi, m)], axis=1)
            out = np.concatenate([out, p[outside_footprints(p)]])
        return out[:n]

    pg = ground_like(ng, 0.0, 0.0)
    pcl = ground_like(nc, 0.0, 12.0)
    pts = np.concatenate([pb, pg, pcl])
    kind = np.concatenate([np.zeros(nb, np.int8), np.ones(ng, np.int8), np.full(nc, 2, np.int8)])
    perm = rng.permutation(n_points)
    pts, kind = pts[perm], kind[perm]

    cams = flight_views(n_views, width, height, f, 0.8 * half_extent, distance)
    masks = []
    for cam in cams:
        m = polygon_mask(box_silhouettes(boxes, cam), width, height)
        for _ in range(false_rects):
            w = int(width * rng.uniform(0.01, 0.06))
            h = int(height * rng.uniform(0.01, 0.06))
            x0 = int(rng.integers(0, width - w))
            y0 = int(rng.integers(0, height - h))
            m[y0:y0 + h, x0:x0 + w] = 1
        for _ in range(holes):
            w = int(width * rng.uniform(0.002, 0.01))
            h = int(height * rng.uniform(0.002, 0.01))
            x0 = int(rng.integers(0, width - w))
            y0 = int(rng.integers(0, height - h))
            m[y0:y0 + h, x0:x0 + w] = 0
        masks.append(m)
    return Survey(_f32(pts.T), kind, cams, masks, boxes, info=dict(seed=seed))


def vote_small(seed=61, n_points=30_000, n_views=8, width=640, height=427):
    """Small voting workload (seconds on the oracle, several workgroups and
    a ragged tail on the GPU): 30k points, 8 views at 640x427 with the full
    survey's field of view."""
    return survey(seed, n_points, n_views, width, height, f=4788.0 * width / 5472, n_boxes=40,
                  half_extent=200.0, distance=250.0)


def vote_full(seed=62, n_points=2_000_000, n_views=64):
    """Full voting workload: 2M sparse points of a 1 km^2 scene of 200
    buildings, 64 oblique views at 5472x3648 (the paper's image size)."""
    return survey(seed, n_points, n_views)


@dataclass
class DepthStack:
    cameras: List[Camera]
    depths: List[List[np.ndarray]]  # [view][group] float32 [H][W], 0 = no depth
    boxes: np.ndarray
    volume: dict                    # origin (3), voxel, dims (nx, ny, nz), trunc
    info: dict = field(default_factory=dict)


def _ray_box_depth(cam: Camera, boxes, ground=False, which=False):
    """Camera-frame depth of the nearest hit of each pixel-centre ray with a
    set of axis-aligned boxes (and the ground plane z = 0 if `ground`);
    0 where nothing is hit.  With `which`, also the index of the box hit
    (-1 for the ground or nothing).  The generator of the stand-in depth
    maps."""
    W, H = cam.width, cam.height
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    C = -R.T @ t
    u = (np.arange(W) + 0.5 - cam.cx) / cam.fx
    v = (np.arange(H) + 0.5 - cam.cy) / cam.fy
    # world direction with camera-frame z = 1, so the ray parameter is the depth
    dw = [R[0, a] * u[None, :] + R[1, a] * v[:, None] + R[2, a] for a in range(3)]
    inv = [np.divide(1.0, d, out=np.full_like(d, np.inf), where=d != 0) for d in dw]
    best = np.full((H, W), np.inf)
    idx = np.full((H, W), -1)
    for b, (cx, cy, w, d, h) in enumerate(boxes):
        lo = (cx - w / 2, cy - d / 2, 0.0)
        hi = (cx + w / 2, cy + d / 2, h)
        tn = np.full((H, W), -np.inf)
        tf = np.full((H, W), np.inf)
        for a in range(3):
            t0 = (lo[a] - C[a]) * inv[a]
            t1 = (hi[a] - C[a]) * inv[a]
            tn = np.maximum(tn, np.minimum(t0, t1))
            tf = np.minimum(tf, np.maximum(t0, t1))
        hit = (tn <= tf) & (tn > 0) & (tn < best)
        best[hit] = tn[hit]
        idx[hit] = b
    if ground:
        tg = -C[2] * inv[2]
        g = (tg > 0) & (tg < best)
        best[g] = tg[g]
        idx[g] = -1
    depth = np.where(np.isfinite(best), best, 0.0)
    return (depth, idx) if which else depth


def depth_stack(seed, n_views=8, width=1600, height=1200, f=1400.0, n_groups=3, n_boxes=8,
                half_extent=100.0, distance=140.0, noise=0.05, holes=0.02, voxel=0.5, trunc=1.5):
    """Depth maps of one sub-region seen by `n_views` oblique views (pitch 45
    degrees, yaw every 360/n_views degrees, as the batched groups of the
    rasterizer).  The boxes are split into `n_groups` building groups (by x)
    plus one background block (the ground); each group's map holds the
    depth of the visible surfaces of its own boxes (its building mask) and
    the background's map the visible ground, each with its own N(0, noise %)
    relative noise and `holes` of missing pixels.  Neighbouring groups share
    their boundary boxes, so their maps overlap there.  The volume covers the sub-region
    at `voxel` metres."""
    rng = np.random.default_rng(seed)
    boxes = _boxes(rng, n_boxes, half_extent)
    order = np.argsort(boxes[:, 0])
    split = np.array_split(order, n_groups)
    # neighbouring groups share the boxes on their boundary (the last of one
    # split and the first of the next)
    members = [np.union1d(np.union1d(split[g], split[g + 1][:1] if g + 1 < n_groups else []),
                          split[g - 1][-1:] if g > 0 else []).astype(np.int64) for g in range(n_groups)]
    cams, depths = [], []
    for vi in range(n_views):
        yaw = 2 * math.pi * vi / n_views
        eye = (distance * math.sin(yaw), -distance * math.cos(yaw), distance)
        R, t = look_at(eye, (0.0, 0.0, 0.0))
        cam = pinhole(width, height, f, f, width / 2, height / 2, R, t)
        d_all, which = _ray_box_depth(cam, boxes, ground=True, which=True)
        maps = []
        for g in range(n_groups + 1):
            own = np.isin(which, members[g]) if g < n_groups else (which < 0)
            d = np.where(own, d_all, 0.0)
            d = d * (1.0 + noise * 0.01 * rng.normal(size=d.shape))
            d[rng.uniform(size=d.shape) < holes] = 0.0
            maps.append(_f32(d))
        cams.append(cam)
        depths.append(maps)
    ext = half_extent + 10.0
    top = float(boxes[:, 4].max()) + 5.0
    dims = (int(math.ceil(2 * ext / voxel)), int(math.ceil(2 * ext / voxel)), int(math.ceil(top / voxel)))
    vol = dict(origin=_f32([-ext, -ext, -2.0]), voxel=float(np.float32(voxel)), dims=dims,
               trunc=float(np.float32(trunc)))
    return DepthStack(cams, depths, boxes, vol, info=dict(seed=seed, members=members))


def depth_small(seed=81):
    """Small fusion/TSDF workload: 4 views at 256x192, 2 groups, 2 m voxels."""
    return depth_stack(seed, n_views=4, width=256, height=192, f=1400.0 * 256 / 1600, n_groups=2, voxel=2.0,
                       trunc=5.0)


def depth_full(seed=82):
    """Full fusion/TSDF workload: one sub-region, 8 views at 1600x1200 with 3
    building groups and the background block each, volume at 0.5 m voxels
    (440 x 440 x ~250)."""
    return depth_stack(seed)
