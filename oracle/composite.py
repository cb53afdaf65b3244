"""Per-pixel compositing (Sec. 3.1, Eq. 1-4), written as the plain definition.

For a masked pixel p = (u + 0.5, v + 0.5) and the surviving Gaussians in
depth order (FP32 depth key, ties by index):

    q_i     = d_i^T conic_i d_i,   d_i = p - mean2d_i
    alpha_i = min(0.99, o_i exp(-q_i / 2));  skipped if alpha_i < 1/255
    T_i     = prod_{j < i, not skipped} (1 - alpha_j)          (Eq. 1)
    blending stops before the first fragment whose T_i (1 - alpha_i) < 1e-4
    C = sum c_i alpha_i T_i + T_final bg,  N = sum n_i alpha_i T_i  (Eq. 2)
    D = sum d_i alpha_i T_i (Eq. 3),       depth = D / (N . K^-1 p~)  (Eq. 4)
    alpha_out = 1 - T_final,   n_contrib = number of blended fragments
    count = sum of alpha_i over the blended fragments (a soft n_contrib:
            the differentiable stand-in for the contributor count g_i of
            Eq. 9, whose own gradient is zero almost everywhere)

Here the products over j are taken with a cumulative product along the
depth order (a library step), the stop is the set of fragments whose
inclusive product is still >= 1e-4, and the sums are a matrix product of the
per-fragment weights with the per-Gaussian features.  The gradient is the
vector-Jacobian product of this FP64 forward with every discrete decision
(skip, stop, clamps, flip, cull, order) frozen.

Near-threshold allowance: a decision the FP32 kernel may legitimately take
the other way (relative margin below 1e-3 for the cut-off and the stop, 1e-5
for the normal flip) adds to the pixel's allowance the largest change that
flipping it can cause.  Pixels with a non-zero allowance are also marked
unsafe for gradient comparison.
"""
from dataclasses import dataclass

import numpy as np
import torch

from .project import decide, project, params64, support_rect

F64 = torch.float64
CUT_MARGIN = 1e-3
STOP_MARGIN = 1e-3
FLIP_MARGIN = 1e-5
AMAX_MARGIN = 1e-4
# Outputs: rgb 0-2, normal 3-5, dist 6, alpha 7 (allowance channel layout)


@dataclass
class Geo:
    mx: torch.Tensor
    my: torch.Tensor
    a: torch.Tensor
    b: torch.Tensor
    c: torch.Tensor
    o: torch.Tensor
    feat: torch.Tensor      # [g, 7] colour(3), normal(3), dist(1)
    flip_near: torch.Tensor  # bool [g]


def _geo(proj, dec, pos=None):
    sl = slice(None) if pos is None else torch.as_tensor(pos)
    feat = torch.cat([proj["colour"], proj["normal"], proj["dist"][:, None]], dim=1)
    flip_near = torch.as_tensor(dec.flip_margin[dec.order] < FLIP_MARGIN)
    return Geo(proj["mean2d"][sl, 0], proj["mean2d"][sl, 1], proj["conic"][sl, 0],
               proj["conic"][sl, 1], proj["conic"][sl, 2], proj["opacity"][sl], feat[sl],
               flip_near[sl])


def composite_block(px, py, g: Geo, cfg, want_allow=True):
    """Composite pixel centres (px, py) [P] against candidates ``g`` (already
    in depth order).  Returns (F [P,7], T_final [P], n [P], allow [P,8],
    grad_unsafe [P], count [P])."""
    P, G = px.shape[0], g.mx.shape[0]
    if G == 0:
        F = torch.zeros((P, 7), dtype=F64)
        return F, torch.ones(P, dtype=F64), torch.zeros(P, dtype=torch.int64), \
            torch.zeros((P, 8), dtype=F64), torch.zeros(P, dtype=torch.bool), torch.zeros(P, dtype=F64)
    dx = px[:, None] - g.mx[None, :]
    dy = py[:, None] - g.my[None, :]
    q = g.a[None] * dx * dx + 2.0 * g.b[None] * dx * dy + g.c[None] * dy * dy
    raw = g.o[None] * torch.exp(-0.5 * q)
    alpha = torch.clamp(raw, max=cfg.alpha_max)
    with torch.no_grad():
        keep = alpha >= cfg.alpha_min
        a0 = torch.where(keep, alpha, torch.zeros_like(alpha))
        tin0 = torch.cumprod(1.0 - a0, dim=1)
        contrib = keep & (tin0 >= cfg.t_min)
        tex0 = torch.cat([torch.ones((P, 1), dtype=F64), tin0[:, :-1]], dim=1)
        live = tex0 >= cfg.t_min
    a_c = torch.where(contrib, alpha, torch.zeros_like(alpha))
    tin = torch.cumprod(1.0 - a_c, dim=1)
    tex = torch.cat([torch.ones((P, 1), dtype=F64), tin[:, :-1]], dim=1)
    w = a_c * tex
    F = w @ g.feat
    T = tin[:, -1]
    n = contrib.sum(dim=1)
    count = a_c.sum(dim=1)
    allow = torch.zeros((P, 8), dtype=F64)
    unsafe = torch.zeros(P, dtype=torch.bool)
    if want_allow:
        with torch.no_grad():
            fa = g.feat.detach().abs()
            maxabs = fa.max(dim=0).values
            alpha_d = alpha.detach()
            near_cut = live & ((alpha_d / cfg.alpha_min - 1.0).abs() < CUT_MARGIN)
            wc = cfg.alpha_min * tex0 * near_cut
            allow[:, :7] += wc @ fa + wc.sum(1, keepdim=True) * maxabs[None]
            allow[:, 7] += 2.0 * wc.sum(1)
            near_stop = live & keep & ((tin0 / cfg.t_min - 1.0).abs() < STOP_MARGIN)
            ws = ((alpha_d * tex0 + cfg.t_min) * near_stop).sum(1)
            allow[:, :7] += ws[:, None] * maxabs[None]
            allow[:, 7] += ws
            wf = 2.0 * alpha_d * tex0 * (contrib & g.flip_near[None])
            allow[:, 3:6] += wf.sum(1, keepdim=True)
            allow[:, 6] += wf @ fa[:, 6]
            near_amax = live & keep & ((raw.detach() / cfg.alpha_max - 1.0).abs() < AMAX_MARGIN)
            unsafe = (allow.sum(1) > 0) | near_amax.any(1)
    return F, T, n, allow, unsafe, count


def _candidates_by_cell(proj, cam, cfg, cell):
    """For every cell of ``cell`` x ``cell`` pixels, the depth-ordered
    positions of the Gaussians whose exact support box meets the cell."""
    px0, px1, py0, py1, *_ , nonempty = support_rect(proj, cam, cfg, 1)
    # a hair of outward margin so rounding in the support bound never drops
    # a pixel where alpha reaches the cut-off exactly
    ncx = (cam.width + cell - 1) // cell
    k = np.flatnonzero(nonempty)
    cx0 = np.maximum(px0[k] - 1, 0) // cell
    cx1 = np.minimum(px1[k] + 1, cam.width - 1) // cell
    cy0 = np.maximum(py0[k] - 1, 0) // cell
    cy1 = np.minimum(py1[k] + 1, cam.height - 1) // cell
    wx = cx1 - cx0 + 1
    wy = cy1 - cy0 + 1
    cnt = wx * wy
    tot = int(cnt.sum())
    owner = np.repeat(np.arange(len(k)), cnt)
    local = np.arange(tot) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    cx = cx0[owner] + local % wx[owner]
    cy = cy0[owner] + local // wx[owner]
    cell_id = cy * ncx + cx
    pos = k[owner]
    srt = np.lexsort((pos, cell_id))
    cell_id, pos = cell_id[srt], pos[srt]
    starts = np.searchsorted(cell_id, np.arange(ncx * ((cam.height + cell - 1) // cell) + 1))
    return pos, starts, ncx


def _pixel_list(cam, mask, pixels):
    if pixels is not None:
        pix = np.asarray(pixels, dtype=np.int64).reshape(-1, 2)
    else:
        m = np.ones((cam.height, cam.width), bool) if mask is None else np.asarray(mask).astype(bool)
        idx = np.flatnonzero(m.ravel())
        pix = np.stack([idx // cam.width, idx % cam.width], axis=1)
    return pix


def _groups(pix, proj, cam, cfg, mode, cell, chunk_elems=4_000_000):
    """Yield (pixel rows, candidate positions) groups."""
    G = proj["mean2d"].shape[0]
    if mode == "brute":
        step = max(1, chunk_elems // max(G, 1))
        allpos = np.arange(G)
        for s in range(0, len(pix), step):
            yield np.arange(s, min(len(pix), s + step)), allpos
        return
    pos, starts, ncx = _candidates_by_cell(proj, cam, cfg, cell)
    cid = (pix[:, 0] // cell) * ncx + pix[:, 1] // cell
    order = np.argsort(cid, kind="stable")
    cs = cid[order]
    bounds = np.flatnonzero(np.diff(cs)) + 1
    for grp in np.split(order, bounds):
        if len(grp) == 0:
            continue
        c = cid[grp[0]]
        yield grp, pos[starts[c]:starts[c + 1]]


def _pixel_outputs(F, T, pixf, cam, cfg):
    bg = torch.tensor(cfg.bg, dtype=F64)
    rgb = F[:, 0:3] + T[:, None] * bg[None]
    nrm = F[:, 3:6]
    dist = F[:, 6]
    r = torch.stack([(pixf[:, 0] - cam.cx) / cam.fx, (pixf[:, 1] - cam.cy) / cam.fy,
                     torch.ones_like(pixf[:, 0])], dim=1)
    den = (nrm * r).sum(1)
    with torch.no_grad():
        ok = den < -cfg.depth_guard
    safe = torch.where(ok, den, -torch.ones_like(den))
    depth = torch.where(ok, dist / safe, torch.zeros_like(dist))
    return rgb, nrm, dist, depth, 1.0 - T, den, r


@dataclass
class Prepared:
    gs: object
    cam: object
    mask: object
    cfg: object
    dec: object
    proj: dict


def prepare(gs, cam, mask, cfg):
    dec = decide(gs, cam, cfg)
    with torch.no_grad():
        proj = project(params64(gs), cam, dec, cfg)
    return Prepared(gs, cam, mask, cfg, dec, proj)


def render(gs, cam, mask, cfg, mode="culled", pixels=None, cell=16, prep=None):
    """Forward render at the masked pixels (default: every masked pixel) or
    at the given (v, u) pixels.

    Returns a dict with per-pixel arrays (shape [P] / [P,3]) and, when
    ``pixels`` is None, full images: rgb [3,H,W], normal [3,H,W], dist, depth,
    alpha [H,W] (float64) and n_contrib [H,W] (int64); plus ``allow``
    (float64 [P,8]), ``unsafe`` (bool [P]), ``depth_unreliable`` (bool [P]).
    """
    if prep is None:
        prep = prepare(gs, cam, mask, cfg)
    proj, dec = prep.proj, prep.dec
    pix = _pixel_list(cam, mask, pixels)
    Pn = len(pix)
    res = dict(pix=pix, rgb=np.zeros((Pn, 3)), normal=np.zeros((Pn, 3)), dist=np.zeros(Pn),
               depth=np.zeros(Pn), alpha=np.zeros(Pn), n_contrib=np.zeros(Pn, np.int64),
               allow=np.zeros((Pn, 8)), unsafe=np.zeros(Pn, bool),
               depth_unreliable=np.zeros(Pn, bool), T=np.ones(Pn), den=np.zeros(Pn), count=np.zeros(Pn))
    with torch.no_grad():
        g_all = _geo(proj, dec)
        for rows, cand in _groups(pix, proj, cam, cfg, mode, cell):
            g = Geo(*(getattr(g_all, f)[torch.as_tensor(cand)] for f in
                      ("mx", "my", "a", "b", "c", "o", "feat", "flip_near")))
            pixf = torch.tensor(pix[rows][:, ::-1] + 0.5, dtype=F64)  # (x, y)
            F, T, n, allow, unsafe, count = composite_block(pixf[:, 0], pixf[:, 1], g, cfg)
            rgb, nrm, dist, depth, alpha, den, r = _pixel_outputs(F, T, pixf, cam, cfg)
            res["rgb"][rows] = rgb.numpy()
            res["normal"][rows] = nrm.numpy()
            res["dist"][rows] = dist.numpy()
            res["depth"][rows] = depth.numpy()
            res["alpha"][rows] = alpha.numpy()
            res["T"][rows] = T.numpy()
            res["n_contrib"][rows] = n.numpy()
            res["count"][rows] = count.numpy()
            res["den"][rows] = den.numpy()
            res["allow"][rows] = allow.numpy()
            nr = torch.linalg.norm(nrm, dim=1) * torch.linalg.norm(r, dim=1)
            near_guard = (den + cfg.depth_guard).abs() <= 1e-3 * nr + 1e-12
            res["depth_unreliable"][rows] = ((allow[:, 3:7].sum(1) > 0) | near_guard).numpy()
            res["unsafe"][rows] = (unsafe | near_guard).numpy()
    if pixels is None:
        H, W = cam.height, cam.width
        v, u = pix[:, 0], pix[:, 1]
        img = {}
        for name, c in (("rgb", 3), ("normal", 3)):
            a = np.zeros((c, H, W))
            a[:, v, u] = res[name].T
            img[name] = a
        for name in ("dist", "depth", "alpha", "count"):
            a = np.zeros((H, W))
            a[v, u] = res[name]
            img[name] = a
        a = np.zeros((H, W), np.int64)
        a[v, u] = res["n_contrib"]
        img["n_contrib"] = a
        res["images"] = img
    res["prep"] = prep
    return res


def render_grad(gs, cam, mask, cfg, gout, pixels=None, mode="culled", cell=16):
    """Gradient of L = sum_p sum_ch gout_ch(p) out_ch(p) over the masked
    pixels (or the given (v, u) pixels) with respect to the raw parameters.

    ``gout`` maps output name (rgb, normal, dist, depth, alpha, count) ->
    array [c][H][W] / [H][W] (missing = 0).
    Returns dict of float64 arrays shaped like the inputs.
    """
    dec = decide(gs, cam, cfg)
    p = params64(gs, requires_grad=True)
    proj = project(p, cam, dec, cfg)
    keys = ("mean2d", "conic", "opacity", "colour", "normal", "dist")
    leaves = {k: proj[k].detach().clone().requires_grad_(True) for k in keys}
    proj_l = dict(proj)
    proj_l.update(leaves)
    pix = _pixel_list(cam, mask, pixels)
    H, W = cam.height, cam.width

    def plane(name, c):
        g = gout.get(name)
        if g is None:
            return None
        g = np.asarray(g, dtype=np.float64).reshape(c, H, W)
        return g

    gplanes = {n: plane(n, c) for n, c in (("rgb", 3), ("normal", 3), ("dist", 1),
                                            ("depth", 1), ("alpha", 1), ("count", 1))}
    with torch.no_grad():
        proj_nd = {k: v.detach() for k, v in proj.items()}
    for rows, cand in _groups(pix, proj_nd, cam, cfg, mode, cell):
        ct = torch.as_tensor(cand)
        feat = torch.cat([leaves["colour"], leaves["normal"], leaves["dist"][:, None]], 1)[ct]
        flip_near = torch.zeros(len(cand), dtype=torch.bool)
        g = Geo(leaves["mean2d"][ct, 0], leaves["mean2d"][ct, 1], leaves["conic"][ct, 0],
                leaves["conic"][ct, 1], leaves["conic"][ct, 2], leaves["opacity"][ct], feat,
                flip_near)
        pr = pix[rows]
        pixf = torch.tensor(pr[:, ::-1] + 0.5, dtype=F64)
        F, T, n, _, _, count = composite_block(pixf[:, 0], pixf[:, 1], g, cfg, want_allow=False)
        rgb, nrm, dist, depth, alpha, _, _ = _pixel_outputs(F, T, pixf, cam, cfg)
        loss = torch.zeros((), dtype=F64)
        for name, val in (("rgb", rgb), ("normal", nrm), ("dist", dist), ("depth", depth),
                          ("alpha", alpha), ("count", count)):
            gp = gplanes[name]
            if gp is None:
                continue
            gv = torch.tensor(gp[:, pr[:, 0], pr[:, 1]].T, dtype=F64)
            loss = loss + (gv.reshape(val.shape) * val).sum()
        if loss.requires_grad:
            loss.backward()
    outs, grads = [], []
    for k in keys:
        if leaves[k].grad is not None:
            outs.append(proj[k])
            grads.append(leaves[k].grad)
    if outs:
        torch.autograd.backward(outs, grads)
    res = {}
    for k, v in p.items():
        res[k] = np.zeros(v.shape) if v.grad is None else v.grad.numpy().copy()
    return res


def loss_value(gs, cam, mask, cfg, gout, pixels=None, mode="culled"):
    """L = sum_p sum_ch gout_ch(p) out_ch(p), re-deciding everything (for
    finite differences)."""
    r = render(gs, cam, mask, cfg, mode=mode, pixels=pixels)
    pix = r["pix"]
    H, W = cam.height, cam.width
    tot = 0.0
    for name, c in (("rgb", 3), ("normal", 3), ("dist", 1), ("depth", 1), ("alpha", 1), ("count", 1)):
        g = gout.get(name)
        if g is None:
            continue
        g = np.asarray(g, dtype=np.float64).reshape(c, H, W)[:, pix[:, 0], pix[:, 1]].T
        tot += float((g.reshape(r[name].shape) * r[name]).sum())
    return tot
