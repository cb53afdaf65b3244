"""GPU parity of the training losses (Sec. 4.2 Eq. 8, Sec. 4.3 Eq. 9-11)
and of the balance-load statistics against the FP64 oracle.

The rendered planes the losses read are seeded synthetic stand-ins written
into the batch's output buffers (both sides see the same FP32 values); the
per-tile pair counts come from a binning of seeded synthetic rectangles,
which the GPU reproduces bit-exactly (checked again here).

Tolerances: loss values relative 1e-5; dL/drgb relative 1e-6 (a sign times
a constant); dL/dnormal and dL/ddepth |g - g_ref| <= 1e-3 |g_ref| + 1e-4
max|g_ref|, leaving out pixels where an L1 sign is within 2e-3 of its kink
(FP32 depth-normal error at 1080p is ~1e-4), and for the depth gradient also
their 4-neighbours, whose gradients gather the excluded pixel's terms.
"""
import numpy as np
import pytest
import torch

import scenes
from oracle import binning as ob
from oracle import losses as ol
from paper_2501_01677_amd.raster import LossConfig, RenderConfig
from gpu_common import device_scene, grad_tolerance_check

pytestmark = pytest.mark.gpu

SIGN_MARGIN = 2e-3


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _synthetic_binning(b, sc, tile, seed):
    """Seeded rectangles and depth keys binned on the GPU; returns the
    oracle's per-tile ranges and active flags (checked bit-exact)."""
    rng = np.random.default_rng(seed)
    nrec = int(b.info.n_records)
    grids, offs, active = [], [], []
    off = 0
    rr = []
    for r, rd in enumerate(sc.renders):
        tx, ty = ob.tile_grid(rd.camera.width, rd.camera.height, tile)
        grids.append((tx, ty))
        offs.append(off)
        active.append(ob.tile_mask_counts(rd.mask, rd.camera.width, rd.camera.height, tile) > 0)
        off += tx * ty
        rr.append(np.full(sc.sets[rd.set_index].n, r))
    active = np.concatenate(active)
    rr = np.concatenate(rr)
    rects = np.zeros((nrec, 4), np.int64)
    for r, (tx, ty) in enumerate(grids):
        m = rr == r
        k = int(m.sum())
        x0, y0 = rng.integers(0, tx, k), rng.integers(0, ty, k)
        rects[m] = np.stack([x0, y0, np.minimum(tx, x0 + rng.integers(0, 6, k)),
                             np.minimum(ty, y0 + rng.integers(0, 5, k))], 1)
    depth = rng.integers(0, 2 ** 32, nrec, dtype=np.uint64).astype(np.uint32)
    valid = rng.uniform(size=nrec) < 0.9
    b.view("rect", torch.int16, nrec, 4).copy_(torch.from_numpy(rects.astype(np.uint16).view(np.int16)))
    b.view("depth_key", torch.int32, nrec).copy_(torch.from_numpy(depth.view(np.int32)))
    b.view("n_active", torch.int32, nrec).copy_(torch.from_numpy(valid.astype(np.int32)))
    b.binning()
    _, _, ranges = ob.emit_and_sort_fast(rects, depth, valid, rr, grids, offs, active)
    assert np.array_equal(_u32(b.view("ranges", torch.int32, int(b.info.n_tiles), 2)), ranges)
    per_render = []
    for r, (tx, ty) in enumerate(grids):
        sl = slice(offs[r], offs[r] + tx * ty)
        per_render.append((ranges[sl, 1].astype(np.int64) - ranges[sl, 0], active[sl]))
    return per_render


def _unsafe(margin):
    u = margin < SIGN_MARGIN
    nb = u.copy()
    nb[1:, :] |= u[:-1, :]
    nb[:-1, :] |= u[1:, :]
    nb[:, 1:] |= u[:, :-1]
    nb[:, :-1] |= u[:, 1:]
    return u, nb


def _check_loss(sc, lc, tile=16, seed=0, expect_depth_grad=True, unit_weights=False):
    b = device_scene(sc, RenderConfig(tile=tile), pair_capacity=1 << 20)
    loads = _synthetic_binning(b, sc, tile, seed + 7)
    ins = [scenes.loss_inputs(seed + 100 + r, rd) for r, rd in enumerate(sc.renders)]
    # counts and Eq. 9 weights for the GC-load term
    cw = [scenes.load_inputs(seed + 200 + r, rd) for r, rd in enumerate(sc.renders)]
    for r, x in enumerate(ins):
        for k in ("rgb", "normal", "depth"):
            b.out[r][k].copy_(torch.from_numpy(x[k]))
        b.out[r]["n_contrib"].copy_(torch.from_numpy(cw[r][0]))
        for k in b.gout[r]:
            b.gout[r][k].fill_(float("nan"))       # the loss must write every masked pixel
    gt = [torch.from_numpy(x["gt"]).cuda() for x in ins]
    weights = None if unit_weights else [torch.from_numpy(w).cuda() for _, w in cw]
    vals = b.loss(gt, lc, weights=weights).cpu().numpy()
    olc = ol.LossConfig(lc.lambda_rgb, lc.lambda_normal, lc.boundary_weight, lc.lambda_load, lc.normal_norm,
                        lc.normal_eps, lc.load_term)
    for r, rd in enumerate(sc.renders):
        x = ins[r]
        var = ol.tile_load_variance(*loads[r])
        g_in, w_in = cw[r]
        ref = ol.loss_and_grads(x["rgb"], x["normal"], x["depth"], x["gt"], rd.mask, rd.camera, olc, load_var=var,
                                n_contrib=g_in, weight=None if unit_weights else w_in)
        want = np.array([ref["total"], ref["rgb"], ref["normal"], ref["load"]])
        np.testing.assert_allclose(vals[r], want, rtol=1e-5, atol=1e-7, err_msg=f"render {r} loss values")
        m = ol.as_mask(rd.mask, (rd.camera.height, rd.camera.width))
        g = {k: b.gout[r][k].cpu().numpy() for k in b.gout[r]}
        np.testing.assert_allclose(g["rgb"][:, m], ref["g_rgb"][:, m], rtol=1e-6, atol=0)
        assert np.all(g["dist"][m] == 0) and np.all(g["alpha"][m] == 0)
        if lc.load_term == 1:
            ok, ratio, rel = grad_tolerance_check(g["count"][m], ref["g_count"][m])
            assert ok, ("count", r, ratio, rel)
            assert np.abs(ref["g_count"][m]).max() > 0
        else:
            assert np.all(g["count"][m] == 0)
        margin = ol.sign_margins(x["rgb"], x["normal"], x["depth"], x["gt"], rd.mask, rd.camera, olc)
        u, nb = _unsafe(margin) if lc.normal_norm == 1 else (np.zeros_like(m), np.zeros_like(m))
        assert u[m].mean() < 0.02, u[m].mean()
        ok, ratio, rel = grad_tolerance_check(g["normal"][:, m & ~u], ref["g_normal"][:, m & ~u])
        assert ok, ("normal", r, ratio, rel)
        ok, ratio, rel = grad_tolerance_check(g["depth"][m & ~nb], ref["g_depth"][m & ~nb])
        assert ok, ("depth", r, ratio, rel)
        if expect_depth_grad:
            assert np.abs(ref["g_depth"][m]).max() > 0
    return b


@pytest.mark.parametrize("norm", [1, 2])
def test_loss_matches_oracle_two_renders(norm):
    print(f"[case] loss norm={norm}", flush=True)
    subs = [scenes.small_scene(300 + k, n=200, width=70 + 23 * k, height=50 + 9 * k, sh_degree=0) for k in range(2)]
    sc = scenes.Scene([s.sets[0] for s in subs], [scenes.Render(k, s.renders[0].camera, s.renders[0].mask)
                                                  for k, s in enumerate(subs)])
    _check_loss(sc, LossConfig(normal_norm=norm, lambda_normal=0.3, lambda_load=0.41), seed=norm)


@pytest.mark.parametrize("unit_weights", [False, True])
def test_gc_load_term_matches_oracle(unit_weights):
    """Eq. 9 GC-load as the balance-load term of Eq. 11: its value (the std
    of n_contrib / w over masked pixels) and its gradient to the soft count,
    with luminance-style weights and with unit weights."""
    print(f"[case] GC-load term unit_weights={unit_weights}", flush=True)
    subs = [scenes.small_scene(310 + k, n=200, width=64 + 30 * k, height=48 + 7 * k, sh_degree=0) for k in range(2)]
    sc = scenes.Scene([s.sets[0] for s in subs], [scenes.Render(k, s.renders[0].camera, s.renders[0].mask)
                                                  for k, s in enumerate(subs)])
    _check_loss(sc, LossConfig(lambda_load=0.41, load_term=1), seed=21, unit_weights=unit_weights)


def test_loss_matches_oracle_full_frame_1080p():
    print("[case] loss 1080p", flush=True)
    sc = scenes.config2(n=4096)
    _check_loss(sc, LossConfig(), seed=11)


def test_loss_full_mask_and_degenerate_sizes():
    print("[case] loss full mask / tiny images", flush=True)
    for (W, H) in ((1, 1), (2, 3), (17, 1), (33, 31)):
        sc = scenes.small_scene(320 + W, n=20, width=W, height=H, sh_degree=0, mask_kind="full")
        _check_loss(sc, LossConfig(lambda_normal=0.5), seed=W, expect_depth_grad=min(W, H) >= 3)


def test_luminance_weights_match_oracle():
    print("[case] luminance weights", flush=True)
    for (W, H, kind) in ((70, 50, "rects"), (1, 9, "full"), (40, 33, "empty")):
        sc = scenes.small_scene(340 + W, n=20, width=W, height=H, sh_degree=0, mask_kind=kind)
        b = device_scene(sc)
        gt = scenes.loss_inputs(5, sc.renders[0])["gt"]
        w = b.luminance_weights(0, torch.from_numpy(gt).cuda()).cpu().numpy()
        ref = ol.luminance_weights(gt, sc.renders[0].mask)
        np.testing.assert_allclose(w, ref, rtol=2e-5, atol=1e-6)


def test_load_stats_match_oracle():
    print("[case] load stats", flush=True)
    subs = [scenes.small_scene(360 + k, n=3000, width=120 + 40 * k, height=90, sh_degree=0) for k in range(2)]
    sc = scenes.Scene([s.sets[0] for s in subs], [scenes.Render(k, s.renders[0].camera, s.renders[0].mask)
                                                  for k, s in enumerate(subs)])
    tile = 16
    b = device_scene(sc, RenderConfig(tile=tile), pair_capacity=1 << 20)
    loads = _synthetic_binning(b, sc, tile, 9)
    ws = []
    for r, rd in enumerate(sc.renders):
        g, w = scenes.load_inputs(50 + r, rd)
        b.out[r]["n_contrib"].copy_(torch.from_numpy(g))
        ws.append((g, w))
    got = b.load_stats([torch.from_numpy(w).cuda() for _, w in ws]).cpu().numpy()
    got1 = b.load_stats().cpu().numpy()
    for r, rd in enumerate(sc.renders):
        counts, active = loads[r]
        c = counts[active].astype(np.float64)
        g, w = ws[r]
        m = ol.as_mask(rd.mask, g.shape)
        want = [c.mean(), ol.tile_load_variance(counts, active), (g[m] / w[m].astype(np.float64)).mean(),
                ol.gc_load(g, w, m)]
        np.testing.assert_allclose(got[r], want, rtol=2e-6)
        want1 = [c.mean(), c.var(), g[m].mean(), ol.gc_load(g, np.ones_like(w), m)]
        np.testing.assert_allclose(got1[r], want1, rtol=2e-6)
