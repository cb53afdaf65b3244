"""Training losses on the rendered outputs (Sec. 4.2 Eq. 8, Sec. 4.3 Eq. 9-11),
written as plain FP64 definitions.  TEST INFRASTRUCTURE ONLY.

Per render, with M the number of masked pixels:

  L_rgb  = (1 / 3M) sum over masked pixels and channels |rgb - gt|
  L_ban  = (1 / M)  sum over masked pixels p where both normals exist
           w_p * || n_depth(p) - N(p) / |N(p)| ||      (Eq. 8)
           with ||.|| the L1 norm (the training configuration) or the
           squared L2 norm (Eq. 8 as printed), w_p = boundary_weight (0.1)
           on the mask boundary MB and 1 elsewhere in the mask
  L_geo  = lambda_rgb L_rgb + lambda_normal L_ban    (the PG-geo terms this
           path renders; the multi-view terms of Eq. 10 need other views'
           images and are not part of it)
  L      = (1 - lambda_load) L_geo + lambda_load L_load       (Eq. 11)
  L_load = load_term 0: Var_t(pairs per active tile), a value only (a
           count has zero gradient almost everywhere);
           load_term 1: the GC-load of Eq. 9, std over masked pixels of
           x_i = g_i / w_i with g_i = n_contrib, taken with a gradient
           through the soft count s_i = sum of alpha over the fragments
           blended at pixel i: the value uses the integer g_i, and
           dL/ds_i = dL/dg_i = lambda_load (x_i - mean x) / (M std x w_i)
           (straight through; 0 when std x = 0)

Readings (where the paper is silent):
  - MB: masked pixels with at least one unmasked 4-neighbour inside the
    image (the image border is not a mask boundary).
  - n_depth (the depth-derived normal of Sec. 4.2): every pixel with a
    positive rendered depth inside the mask is back-projected to
    P = depth * ((u + 0.5 - cx) / fx, (v + 0.5 - cy) / fy, 1).  Along x the
    difference is P(u+1) - P(u-1), each neighbour replaced by the pixel
    itself when it is not such a valid pixel (one-sided at the mask
    boundary); likewise along y.  n_depth = normalize(dPy x dPx), which
    faces the camera.  It exists when the pixel is valid and has at least
    one valid neighbour along each axis.
  - The rendered normal N is used only where |N| > normal_eps (decided in
    FP32, as the kernel decides it).
  - The Eq. 9 weight w_i ("gradient-dependent", not fixed by the paper):
    0.1 + |grad Y| / mean over masked pixels of |grad Y|, Y the Rec. 601
    luminance of the ground-truth image, grad by numpy.gradient (central
    differences inside, one-sided at the image border, zero along an axis
    one pixel long); 1 where the mean is 0.  Parity unpinned against the paper (it prints no constants for
    it); pinned only by closed forms of this reading.
"""
from dataclasses import dataclass

import numpy as np
import torch

F64 = torch.float64


@dataclass
class LossConfig:
    lambda_rgb: float = 1.0
    lambda_normal: float = 0.01
    boundary_weight: float = 0.1
    lambda_load: float = 0.0
    normal_norm: int = 1          # 1 = L1, 2 = squared L2
    normal_eps: float = 1e-6
    load_term: int = 0            # 0 = tile-count variance (value), 1 = Eq. 9 GC-load


def as_mask(mask, shape):
    """Boolean mask; None means every pixel is masked."""
    return np.ones(shape, bool) if mask is None else np.asarray(mask).astype(bool)


def mask_boundary(mask, shape=None):
    """MB: masked pixels with an unmasked 4-neighbour inside the image."""
    m = as_mask(mask, shape)
    out = np.zeros_like(m)
    for du, dv in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        # neighbour (u + du, v + dv) masked?  outside the image counts as masked
        out |= m & ~_shift(m, du, dv, True)
    return out


def _shift(a, du, dv, fill):
    """b[v, u] = a[v + dv, u + du] (fill outside the image)."""
    b = torch.full_like(a, fill) if torch.is_tensor(a) else np.full_like(a, fill)
    H, W = a.shape[-2], a.shape[-1]
    ys = slice(max(0, -dv), H - max(0, dv))
    xs = slice(max(0, -du), W - max(0, du))
    ys2 = slice(max(0, dv), H - max(0, -dv))
    xs2 = slice(max(0, du), W - max(0, -du))
    b[..., ys, xs] = a[..., ys2, xs2]
    return b


def pixel_rays(cam):
    """K^-1 p~ at every pixel centre, [3][H][W] float64."""
    H, W = cam.height, cam.width
    u = (np.arange(W) + 0.5 - float(cam.cx)) / float(cam.fx)
    v = (np.arange(H) + 0.5 - float(cam.cy)) / float(cam.fy)
    r = np.empty((3, H, W))
    r[0] = u[None, :]
    r[1] = v[:, None]
    r[2] = 1.0
    return r


def depth_normals(depth, mask, cam):
    """Depth-derived normals (torch, differentiable in depth) and where they
    exist.  depth: float64 tensor [H][W]; mask: bool array [H][W]."""
    valid = torch.from_numpy(as_mask(mask, tuple(depth.shape))) & (depth.detach() > 0)
    P = depth[None] * torch.from_numpy(pixel_rays(cam))
    vxp, vxm = _shift(valid, 1, 0, False), _shift(valid, -1, 0, False)
    vyp, vym = _shift(valid, 0, 1, False), _shift(valid, 0, -1, False)
    a = torch.where(vxp[None], _shift(P, 1, 0, 0.0), P)
    b = torch.where(vxm[None], _shift(P, -1, 0, 0.0), P)
    c = torch.where(vyp[None], _shift(P, 0, 1, 0.0), P)
    d = torch.where(vym[None], _shift(P, 0, -1, 0.0), P)
    dPx, dPy = a - b, c - d
    cr = torch.linalg.cross(dPy, dPx, dim=0)
    exists = valid & (vxp | vxm) & (vyp | vym)
    sq = (cr * cr).sum(0)
    nrm = torch.sqrt(torch.where(exists, sq, torch.ones_like(sq)))
    return cr / nrm[None], exists


def normal_usable(normal32, eps):
    """|N| > eps decided in FP32 from the FP32 rendered normal [3][H][W]."""
    n = np.asarray(normal32, np.float32)
    s = n[0] * n[0] + n[1] * n[1] + n[2] * n[2]
    return np.sqrt(s, dtype=np.float32) > np.float32(eps)


def geo_terms(rgb, normal, depth, gt, mask, cam, lc: LossConfig, normal32=None):
    """(L_rgb, L_ban) as torch scalars, differentiable in rgb, normal, depth
    (float64 tensors [3][H][W], [3][H][W], [H][W])."""
    shape = tuple(depth.shape)
    m = torch.from_numpy(as_mask(mask, shape))
    M = max(int(m.sum()), 1)
    l_rgb = (torch.abs(rgb - torch.as_tensor(gt, dtype=F64)) * m[None]).sum() / (3.0 * M)
    nd, exists = depth_normals(depth, mask, cam)
    n32 = normal.detach().numpy() if normal32 is None else normal32
    use = exists & torch.from_numpy(normal_usable(n32, lc.normal_eps)) & m
    sq = (normal * normal).sum(0)
    nr = normal / torch.sqrt(torch.where(use, sq, torch.ones_like(sq)))[None]
    diff = nd - nr
    e = torch.abs(diff).sum(0) if lc.normal_norm == 1 else (diff * diff).sum(0)
    w = torch.where(torch.from_numpy(mask_boundary(mask, shape)), lc.boundary_weight, 1.0).to(F64)
    l_ban = (torch.where(use, w * e, torch.zeros_like(e))).sum() / M
    return l_rgb, l_ban


def tile_load_variance(tile_pairs, tile_active):
    """Population variance of the pair counts over active tiles (the
    balance-load term's value)."""
    c = np.asarray(tile_pairs, np.float64)[np.asarray(tile_active, bool)]
    return float(c.var()) if c.size else 0.0


def loss_and_grads(rgb32, normal32, depth32, gt32, mask, cam, lc: LossConfig, load_var=0.0, n_contrib=None,
                   weight=None):
    """Total loss and dL/d(rgb, normal, depth) at FP32 inputs (upcast), and
    dL/d(soft count) (zero unless lc.load_term is 1; then n_contrib [H][W]
    and the Eq. 9 weights (None = 1) are needed, and load_var is not used)."""
    rgb = torch.tensor(np.asarray(rgb32, np.float64), requires_grad=True)
    nrm = torch.tensor(np.asarray(normal32, np.float64), requires_grad=True)
    dep = torch.tensor(np.asarray(depth32, np.float64), requires_grad=True)
    l_rgb, l_ban = geo_terms(rgb, nrm, dep, np.asarray(gt32, np.float64), mask, cam, lc,
                             normal32=np.asarray(normal32, np.float32))
    geo = lc.lambda_rgb * l_rgb + lc.lambda_normal * l_ban
    g_count = np.zeros(np.shape(depth32))
    load = float(load_var)
    if lc.load_term == 1:
        w = np.ones(np.shape(depth32)) if weight is None else weight
        load, dg = gc_load_and_grad(n_contrib, w, mask)
        g_count = lc.lambda_load * dg
    total = (1.0 - lc.lambda_load) * geo + lc.lambda_load * load
    g = torch.autograd.grad(total, [rgb, nrm, dep], allow_unused=True)
    grads = [np.zeros(t.shape) if gi is None else gi.numpy() for gi, t in zip(g, (rgb, nrm, dep))]
    return dict(total=float(total.detach()), rgb=float(l_rgb.detach()), normal=float(l_ban.detach()),
                load=load, g_rgb=grads[0], g_normal=grads[1], g_depth=grads[2], g_count=g_count)


def sign_margins(rgb32, normal32, depth32, gt32, mask, cam, lc: LossConfig):
    """Per pixel, the smallest |n_depth - n_rendered| component (where the L1
    sign decides the gradient); +inf where no normal term is taken."""
    dep = torch.tensor(np.asarray(depth32, np.float64))
    nd, exists = depth_normals(dep, mask, cam)
    n = torch.tensor(np.asarray(normal32, np.float64))
    use = exists & torch.from_numpy(normal_usable(normal32, lc.normal_eps)) & torch.from_numpy(
        as_mask(mask, tuple(dep.shape)))
    nr = n / torch.sqrt((n * n).sum(0)).clamp_min(1e-300)[None]
    mg = torch.abs(nd - nr).min(0).values
    return torch.where(use, mg, torch.full_like(mg, float("inf"))).numpy()


def luminance_weights(gt, mask):
    """Eq. 9 per-pixel weights w = 0.1 + |grad Y| / mean_mask |grad Y|."""
    g = np.asarray(gt, np.float64)
    Y = 0.299 * g[0] + 0.587 * g[1] + 0.114 * g[2]
    # a one-pixel axis carries no gradient
    gy = np.gradient(Y, axis=0) if Y.shape[0] > 1 else np.zeros_like(Y)
    gx = np.gradient(Y, axis=1) if Y.shape[1] > 1 else np.zeros_like(Y)
    mag = np.sqrt(gx * gx + gy * gy)
    m = as_mask(mask, Y.shape)
    mean = mag[m].mean() if m.any() else 0.0
    if mean > 0:
        return 0.1 + mag / mean
    return np.ones_like(mag)


def gc_load(n_contrib, weight, mask):
    """Eq. 9: population standard deviation over masked pixels of g_i / w_i."""
    m = as_mask(mask, np.shape(n_contrib))
    x = np.asarray(n_contrib, np.float64)[m] / np.asarray(weight, np.float64)[m]
    return float(x.std()) if x.size else 0.0


def gc_load_and_grad(n_contrib, weight, mask):
    """Eq. 9 GC-load and its gradient with respect to the per-pixel counts:
    sigma = population std over the M masked pixels of x_i = g_i / w_i, and
    d sigma / d g_i = (x_i - mean x) / (M sigma w_i) at masked pixels (0
    elsewhere, and everywhere when sigma = 0).  The gradient is the one the
    soft count carries (straight through the integer count)."""
    shape = np.shape(n_contrib)
    m = as_mask(mask, shape)
    g = np.asarray(n_contrib, np.float64)
    w = np.asarray(weight, np.float64)
    grad = np.zeros(shape)
    M = int(m.sum())
    if M == 0:
        return 0.0, grad
    x = g[m] / w[m]
    mu = x.mean()
    sigma = float(np.sqrt(((x - mu) ** 2).mean()))
    if sigma > 0:
        grad[m] = (x - mu) / (M * sigma * w[m])
    return sigma, grad
