"""Reliability-scored multi-view voting filter (Sec. 4.1, Eq. 6-7), written
as its plain definition.  TEST INFRASTRUCTURE ONLY.

For every sparse point p and every view j (camera R_j, t_j, K_j; coarse
building mask M_j of W_j x H_j pixels):

  p is in Image_j   when its camera-frame depth is above z_near and its
                    projection falls inside the image;
  p is in M_j       when it is in Image_j and the mask pixel under the
                    projection is non-zero.

  votes(p) = sum_j I(p in M_j)                    Eq. 6 (p is a potential
                                                  building point iff > 0)
  US(p)    = sum_j I(p in Image_j minus M_j)      Eq. 7 (unreliability score)
  reliable = votes(p) > 0 and US(p) < tau         (tau: the tolerance the
                                                  paper chooses from the
                                                  image overlap)

Readings (where the paper is silent):
  - "appears in the image" is geometric: in front of the camera (depth >
    z_near, 0.2 m as for the rasterizer) and inside the image; there is no
    occlusion test (the paper re-projects the points without one).
  - Pixel (u, v) covers [u, u+1) x [v, v+1) of the image plane, so the
    projection (x, y) lands in pixel (floor x, floor y), inside the image
    iff 0 <= x < W and 0 <= y < H.
  - These are integer decisions taken on floating-point positions, so they
    are taken in FP32 with one fixed operation order, every operation
    rounded on its own (no fused multiply-add), on both sides:
        xc = ((R00 x + R01 y) + R02 z) + t0      (likewise yc, zc)
        front = zc > z_near
        x = fx (xc / zc) + cx ;  y = fy (yc / zc) + cy
    NumPy float32 arithmetic rounds every operation (and its division is
    the correctly rounded one), which is the order written out below.

Flags: bit 0 potential building point (Eq. 6), bit 1 reliable.
"""
import numpy as np

F32 = np.float32


def project(points, cam, z_near=0.2):
    """FP32 projection of float32 points [3][M] into one camera: returns
    (inside, iu, iv) with inside = in front and inside the image, and the
    pixel indices of the inside points (arrays over the inside points)."""
    x, y, z = (np.asarray(points[k], F32) for k in range(3))
    R = np.asarray(cam.R, F32)
    t = np.asarray(cam.t, F32)
    xc = ((R[0, 0] * x + R[0, 1] * y) + R[0, 2] * z) + t[0]
    yc = ((R[1, 0] * x + R[1, 1] * y) + R[1, 2] * z) + t[1]
    zc = ((R[2, 0] * x + R[2, 1] * y) + R[2, 2] * z) + t[2]
    front = zc > F32(z_near)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        px = F32(cam.fx) * (xc / zc) + F32(cam.cx)
        py = F32(cam.fy) * (yc / zc) + F32(cam.cy)
    assert px.dtype == F32 and py.dtype == F32
    inside = front & (px >= F32(0)) & (px < F32(cam.width)) & (py >= F32(0)) & (py < F32(cam.height))
    iu = np.floor(px[inside]).astype(np.int64)
    iv = np.floor(py[inside]).astype(np.int64)
    return inside, iu, iv


def vote(points, cams, masks, tau, z_near=0.2):
    """Eq. 6-7 over every view.  masks[j] is uint8 [H][W] or None (every
    pixel a building pixel).  Returns dict(votes, us, flags) with int64
    votes and US and uint8 flags."""
    m = np.asarray(points).shape[1]
    votes = np.zeros(m, np.int64)
    us = np.zeros(m, np.int64)
    for cam, mask in zip(cams, masks):
        inside, iu, iv = project(points, cam, z_near)
        if mask is None:
            hit = np.ones(len(iu), bool)
        else:
            hit = np.asarray(mask)[iv, iu] != 0
        idx = np.flatnonzero(inside)
        votes[idx[hit]] += 1
        us[idx[~hit]] += 1
    potential = votes > 0
    reliable = potential & (us < tau)
    flags = potential.astype(np.uint8) | (reliable.astype(np.uint8) << 1)
    return dict(votes=votes, us=us, flags=flags)
