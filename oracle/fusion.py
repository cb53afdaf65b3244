"""Multi-view depth fusion and TSDF volume integration (Sec. 4.4, "Mesh
Extraction and Merge"), written as their plain definitions.  TEST
INFRASTRUCTURE ONLY.

Mean fusion: the depth maps that several groups (building groups and
background blocks) render from the same view are merged pixel by pixel;
where they overlap the fused depth is their mean:

  fused(p) = (sum over maps k with depth_k(p) > 0 of depth_k(p)) / (their number),
             0 where no map has a depth.

The fused map is stored in FP32 and decides integers downstream (which
voxels a view updates), so it is defined in FP32: the sum runs over the maps
in their given order, every addition rounded, then one rounded division.

TSDF integration (the truncated signed distance method the paper cites,
the running weighted average of Curless and Levoy with unit weights): for
every voxel centre c = origin + (i + 0.5, j + 0.5, k + 0.5) * voxel and
every view with fused depth D and camera (R, t, K):

  xc, yc, zc = R c + t                   (the voting filter's FP32 order)
  the view sees c if zc > z_near, its projection (u, v) lies inside the
  image, D(floor u, floor v) > 0 and sdf = D - zc >= -trunc;
  then it adds tsdf = min(1, sdf / trunc) with weight 1.

  TSDF(c) = (sum of the added tsdf values) / W(c),  W(c) = number of views
  that saw c;  TSDF = 1 and W = 0 where no view saw it.

Readings (where the paper is silent): the signed distance is measured
along the optical axis (projective TSDF: depth of the surface minus depth of
the voxel), positive in front of the surface; unit weights; views with no
depth at the pixel leave the voxel alone.  The geometric decisions (which
pixel, in front, inside, within the truncation) are taken in FP32 on both
sides, the centre computed as ((i + 0.5) * voxel) + origin with each
operation rounded; the values are summed here in FP64.
"""
import numpy as np

F32 = np.float32


def fuse_depth(depths):
    """FP32 mean of the positive depths of a list of float32 [H][W] maps."""
    s = np.zeros_like(np.asarray(depths[0], F32))
    n = np.zeros(s.shape, np.int64)
    for d in depths:
        d = np.asarray(d, F32)
        v = d > F32(0)
        s = np.where(v, s + d, s)
        n += v
    assert s.dtype == F32
    with np.errstate(invalid="ignore", divide="ignore"):
        out = np.where(n > 0, s / n.astype(F32), F32(0))
    return out.astype(F32), n


def voxel_centres(origin, voxel, dims, index=None):
    """FP32 centres [3][m] of the voxels with flat indices `index` (x fastest;
    all voxels if None)."""
    nx, ny, nz = dims
    idx = np.arange(nx * ny * nz) if index is None else np.asarray(index)
    i = (idx % nx).astype(F32)
    j = ((idx // nx) % ny).astype(F32)
    k = (idx // (nx * ny)).astype(F32)
    o = np.asarray(origin, F32)
    h = F32(0.5)
    vx = F32(voxel)
    return np.stack([(i + h) * vx + o[0], (j + h) * vx + o[1], (k + h) * vx + o[2]])


def integrate(origin, voxel, dims, cams, depths, trunc, z_near=0.2, index=None):
    """TSDF and weight of the voxels `index` (all if None) after every view.
    Returns (tsdf float64 [m], weight int64 [m])."""
    c = voxel_centres(origin, voxel, dims, index)
    x, y, z = c[0], c[1], c[2]
    acc = np.zeros(c.shape[1], np.float64)
    w = np.zeros(c.shape[1], np.int64)
    tr = F32(trunc)
    for cam, D in zip(cams, depths):
        D = np.asarray(D, F32)
        R = np.asarray(cam.R, F32)
        t = np.asarray(cam.t, F32)
        xc = ((R[0, 0] * x + R[0, 1] * y) + R[0, 2] * z) + t[0]
        yc = ((R[1, 0] * x + R[1, 1] * y) + R[1, 2] * z) + t[1]
        zc = ((R[2, 0] * x + R[2, 1] * y) + R[2, 2] * z) + t[2]
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            u = F32(cam.fx) * (xc / zc) + F32(cam.cx)
            v = F32(cam.fy) * (yc / zc) + F32(cam.cy)
        ok = (zc > F32(z_near)) & (u >= 0) & (u < F32(cam.width)) & (v >= 0) & (v < F32(cam.height))
        sel = np.flatnonzero(ok)
        d = D[np.floor(v[sel]).astype(np.int64), np.floor(u[sel]).astype(np.int64)]
        sdf = d - zc[sel]
        assert sdf.dtype == F32
        seen = (d > F32(0)) & (sdf >= -tr)
        sel = sel[seen]
        acc[sel] += np.minimum(1.0, sdf[seen].astype(np.float64) / float(tr))
        w[sel] += 1
    tsdf = np.where(w > 0, acc / np.maximum(w, 1), 1.0)
    return tsdf, w
