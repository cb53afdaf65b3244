"""Per-Gaussian projection (Sec. 3.1): activations, EWA 2D covariance,
SH colour, camera-frame Gaussian normal (Eq. 2) and plane distance (Eq. 3).

Two passes:
  decide(...)   the discrete decisions, taken once on the FP32 inputs
                (culling, depth-order key, smallest-scale axis) or in FP64
                (normal flip, clamps), together with their margins;
  project(...)  the FP64 differentiable map from raw parameters to the
                per-Gaussian 2D quantities, with those decisions frozen.
"""
from dataclasses import dataclass

import numpy as np
import torch

from .sh import sh_basis

F64 = torch.float64


def canonical_depth32(means32, R32, t32):
    """FP32 camera depth of each mean, every product and sum rounded to FP32
    in the fixed order ((r20*x + r21*y) + r22*z) + t2 (no fused multiply-add).
    This value is both the depth-order key and the near-plane test input."""
    m = np.asarray(means32, dtype=np.float32)
    R = np.asarray(R32, dtype=np.float32)
    t = np.asarray(t32, dtype=np.float32)
    a = np.multiply(R[2, 0], m[0], dtype=np.float32)
    b = np.multiply(R[2, 1], m[1], dtype=np.float32)
    c = np.multiply(R[2, 2], m[2], dtype=np.float32)
    s = np.add(np.add(a, b, dtype=np.float32), c, dtype=np.float32)
    tz = np.add(s, t[2], dtype=np.float32)
    assert tz.dtype == np.float32
    return tz


def quat_to_rotmat(q):
    """Unit quaternions (w, x, y, z) [..., 4] -> rotation matrices [..., 3, 3]
    (the textbook Hamilton map)."""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r00 = 1 - 2 * (y * y + z * z)
    r01 = 2 * (x * y - w * z)
    r02 = 2 * (x * z + w * y)
    r10 = 2 * (x * y + w * z)
    r11 = 1 - 2 * (x * x + z * z)
    r12 = 2 * (y * z - w * x)
    r20 = 2 * (x * z - w * y)
    r21 = 2 * (y * z + w * x)
    r22 = 1 - 2 * (x * x + y * y)
    return torch.stack([torch.stack([r00, r01, r02], -1),
                        torch.stack([r10, r11, r12], -1),
                        torch.stack([r20, r21, r22], -1)], -2)


@dataclass
class Decisions:
    visible: np.ndarray      # bool [n]
    tz32: np.ndarray         # float32 [n], the depth key
    order: np.ndarray        # int64 [n_visible], visible ids sorted by (tz32, id)
    jstar: np.ndarray        # int64 [n], axis of the smallest log-scale
    flip: np.ndarray         # bool [n], normal flipped to face the camera
    flip_margin: np.ndarray  # float64 [n], |n_c . t| / |t|
    clamp_margin: np.ndarray  # float64 [n], min relative distance to the J clamp
    colour_min: np.ndarray   # float64 [n], min |unclamped colour| over channels


def camera64(cam):
    R = torch.tensor(np.asarray(cam.R, dtype=np.float64), dtype=F64)
    t = torch.tensor(np.asarray(cam.t, dtype=np.float64), dtype=F64)
    return R, t


def _activations(p):
    scales = torch.exp(p["log_scales"])                      # [3, n]
    q = p["quats"] / torch.linalg.norm(p["quats"], dim=0, keepdim=True)
    opacity = torch.sigmoid(p["opacity_logits"])
    return scales, q, opacity


def _camera_space(p, R, t):
    return (R @ p["means"]).T + t                              # [n, 3]


def decide(gs, cam, cfg):
    """Discrete decisions of the projection, with margins for the allowance
    protocol (decisions within a hair of their threshold are flagged)."""
    n = gs.n
    tz32 = canonical_depth32(gs.means, cam.R, cam.t)
    logit32 = np.asarray(gs.opacity_logits, dtype=np.float32)
    visible = (tz32 > np.float32(cfg.z_near)) & (logit32 >= np.float32(cfg.logit_min))
    ids = np.flatnonzero(visible)
    order = ids[np.lexsort((ids, tz32[ids]))]
    jstar = np.argmin(np.asarray(gs.log_scales, dtype=np.float32), axis=0)
    with torch.no_grad():
        p = {k: torch.tensor(np.asarray(v, dtype=np.float64)) for k, v in gs.arrays().items()}
        R, t = camera64(cam)
        tc = _camera_space(p, R, t)
        _, q, _ = _activations(p)
        Rq = quat_to_rotmat(q.T)                               # [n, 3, 3]
        axis = Rq[torch.arange(n), :, torch.as_tensor(jstar)]  # column j*  [n, 3]
        n_c = axis @ R.T
        dot = (n_c * tc).sum(-1)
        flip = (dot > 0).numpy()
        flip_margin = (dot.abs() / torch.linalg.norm(tc, dim=-1).clamp_min(1e-300)).numpy()
        limx = cfg.fov_clamp * (cam.width / 2.0) / cam.fx
        limy = cfg.fov_clamp * (cam.height / 2.0) / cam.fy
        tz = tc[:, 2].clamp_min(1e-300)
        mx = (tc[:, 0] / tz).abs() / limx
        my = (tc[:, 1] / tz).abs() / limy
        clamp_margin = torch.minimum((mx - 1).abs(), (my - 1).abs()).numpy()
        C = -(R.T @ t)
        d = p["means"].T - C
        d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
        Y = sh_basis(gs.sh_degree, d)                          # [K, n]
        col = torch.einsum("kn,kcn->nc", Y, p["sh"]) + 0.5
        colour_min = col.abs().min(dim=1).values.numpy()
    return Decisions(visible, tz32, order, jstar, flip, flip_margin, clamp_margin, colour_min)


def project(p, cam, dec, cfg, ids=None):
    """Differentiable FP64 per-Gaussian quantities for the Gaussians ``ids``
    (default: the visible ones in depth order).

    ``p`` holds FP64 tensors of the raw parameters (may require grad).
    Returns a dict of tensors indexed like ``ids``:
      mean2d [g,2], cov2d [g,3] (xx, xy, yy), conic [g,3] (a, b, c) with
      q = a dx^2 + 2 b dx dy + c dy^2, opacity [g], colour [g,3],
      normal [g,3] (camera frame), dist [g], tz [g] (FP64 depth).
    """
    if ids is None:
        ids = dec.order
    ids_t = torch.as_tensor(np.asarray(ids, dtype=np.int64))
    sub = {k: v[..., ids_t] for k, v in p.items()}
    R, t = camera64(cam)
    scales, q, opacity = _activations(sub)
    tc = _camera_space(sub, R, t)                              # [g, 3]
    tx, ty, tz = tc[:, 0], tc[:, 1], tc[:, 2]

    # 3D covariance, rotated into the camera frame
    Rq = quat_to_rotmat(q.T)                                   # [g, 3, 3]
    S2 = torch.diag_embed((scales * scales).T)                 # [g, 3, 3]
    Sigma = Rq @ S2 @ Rq.transpose(1, 2)
    Sigma_c = R @ Sigma @ R.T

    # EWA: Jacobian of the perspective map at the (clamped) mean
    limx = cfg.fov_clamp * (cam.width / 2.0) / cam.fx
    limy = cfg.fov_clamp * (cam.height / 2.0) / cam.fy
    xt = torch.clamp(tx / tz, -limx, limx) * tz
    yt = torch.clamp(ty / tz, -limy, limy) * tz
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([cam.fx / tz, zero, -cam.fx * xt / (tz * tz)], -1),
                     torch.stack([zero, cam.fy / tz, -cam.fy * yt / (tz * tz)], -1)], -2)
    cov = J @ Sigma_c @ J.transpose(1, 2)
    cxx = cov[:, 0, 0] + cfg.dilation
    cxy = cov[:, 0, 1]
    cyy = cov[:, 1, 1] + cfg.dilation
    det = cxx * cyy - cxy * cxy
    conic = torch.stack([cyy / det, -cxy / det, cxx / det], -1)
    mean2d = torch.stack([cam.fx * tx / tz + cam.cx, cam.fy * ty / tz + cam.cy], -1)

    # colour from SH on the world-frame view direction
    C = -(R.T @ t)
    d = sub["means"].T - C
    d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
    Y = sh_basis(int(round((sub["sh"].shape[0]) ** 0.5)) - 1, d)
    col = torch.einsum("kn,kcn->nc", Y, sub["sh"]) + 0.5
    colour = torch.clamp(col, min=0.0)

    # Gaussian normal: rotation axis of the smallest scale, into the camera
    # frame (Eq. 2), flipped to face the camera; plane distance (Eq. 3)
    js = torch.as_tensor(dec.jstar[np.asarray(ids)])
    axis = Rq[torch.arange(len(ids_t)), :, js]
    sign = torch.where(torch.as_tensor(dec.flip[np.asarray(ids)]), -1.0, 1.0).to(F64)
    normal = (axis @ R.T) * sign[:, None]
    dist = (normal * tc).sum(-1)
    return dict(mean2d=mean2d, cov2d=torch.stack([cxx, cxy, cyy], -1), conic=conic,
                opacity=opacity, colour=colour, normal=normal, dist=dist, tz=tz)


def params64(gs, requires_grad=False):
    return {k: torch.tensor(np.asarray(v, dtype=np.float64), requires_grad=requires_grad)
            for k, v in gs.arrays().items()}


def support_rect(proj, cam, cfg, tile):
    """Exact FP64 support of every projected Gaussian (the set where its
    unclamped alpha reaches the cut-off, q <= 2 ln(o / alpha_min)), as
    inclusive pixel ranges and as a half-open tile rectangle.

    Returns (px0, px1, py0, py1, tx0, tx1, ty0, ty1, nonempty) as numpy.
    """
    with torch.no_grad():
        o = proj["opacity"].numpy()
        cov = proj["cov2d"].numpy()
        m = proj["mean2d"].numpy()
        qmax = 2.0 * np.log(np.maximum(o, 1e-300) / cfg.alpha_min)
        ok = qmax > 0
        qm = np.where(ok, qmax, 0.0)
        rx = np.sqrt(qm * cov[:, 0])
        ry = np.sqrt(qm * cov[:, 2])
        px0 = np.ceil(m[:, 0] - rx - 0.5)
        px1 = np.floor(m[:, 0] + rx - 0.5)
        py0 = np.ceil(m[:, 1] - ry - 0.5)
        py1 = np.floor(m[:, 1] + ry - 0.5)
        px0 = np.clip(px0, 0, cam.width - 1)
        px1 = np.clip(px1, -1, cam.width - 1)
        py0 = np.clip(py0, 0, cam.height - 1)
        py1 = np.clip(py1, -1, cam.height - 1)
        nonempty = ok & (px0 <= px1) & (py0 <= py1)
        px0, px1, py0, py1 = (a.astype(np.int64) for a in (px0, px1, py0, py1))
        tx0, tx1 = px0 // tile, px1 // tile + 1
        ty0, ty1 = py0 // tile, py1 // tile + 1
    return px0, px1, py0, py1, tx0, tx1, ty0, ty1, nonempty
