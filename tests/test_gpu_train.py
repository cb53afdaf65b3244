"""GPU training step: forward, loss (Sec. 4.2 Eq. 8, Sec. 4.3 Eq. 11),
backward and the fused Adam update, end to end.

The parameter gradient of the whole step is checked against the oracle's
chain: its FP64 render, its loss gradients at the FP32-rounded rendered
planes, and its render vector-Jacobian product with those gradients.  The
ground truth is the oracle's rendered colour moved by 0.02-0.1 per channel,
so no L1 sign sits near its kink; the normal term uses the squared L2 norm
(smooth); pixels with a near-threshold rendering decision are taken out of
the mask on both sides (every pixel is rendered independently, so the rest
is unchanged).
"""
import numpy as np
import pytest
import torch

import scenes
from oracle import adam as oa
from oracle import composite as oc
from oracle import losses as ol
from oracle import project as op
from paper_2501_01677_amd.raster import (LossConfig, RenderConfig, Trainer, adam_step, adam_step_device,
                                         gaussians_to_device)
from gpu_common import CFG, grad_tolerance_check

pytestmark = pytest.mark.gpu

PARAMS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _prepared_scene(seed, sh_degree=2):
    sc = scenes.small_scene(seed, n=160, width=52, height=44, sh_degree=sh_degree, n_views=2)
    rng = np.random.default_rng(seed + 1)
    renders, gts, refs = [], [], []
    for rd in sc.renders:
        full = oc.render(sc.sets[0], rd.camera, rd.mask, CFG)
        unsafe = np.zeros((rd.camera.height, rd.camera.width), bool)
        unsafe[full["pix"][:, 0], full["pix"][:, 1]] = full["unsafe"] | full["depth_unreliable"]
        m1 = (np.asarray(rd.mask).astype(bool) & ~unsafe).astype(np.uint8)
        rd1 = scenes.Render(rd.set_index, rd.camera, m1)
        ref = oc.render(sc.sets[0], rd.camera, m1, CFG)
        off = rng.choice([-1.0, 1.0], (3,) + unsafe.shape) * rng.uniform(0.02, 0.1, (3,) + unsafe.shape)
        gt = (ref["images"]["rgb"] + off).astype(np.float32)
        renders.append(rd1)
        gts.append(gt)
        refs.append(ref)
    return scenes.Scene(sc.sets, renders), gts, refs


def _oracle_step_grads(sc, gts, refs, olc, weights=None):
    gs = sc.sets[0]
    total = {k: np.zeros(getattr(gs, k).shape) for k in PARAMS}
    losses = []
    for r, (rd, gt, ref) in enumerate(zip(sc.renders, gts, refs)):
        im = ref["images"]
        planes = {k: im[k].astype(np.float32) for k in ("rgb", "normal", "depth")}
        lg = ol.loss_and_grads(planes["rgb"], planes["normal"], planes["depth"], gt, rd.mask, rd.camera, olc,
                               n_contrib=im["n_contrib"], weight=None if weights is None else weights[r])
        losses.append(lg)
        g = oc.render_grad(gs, rd.camera, rd.mask, CFG, {"rgb": lg["g_rgb"], "normal": lg["g_normal"],
                                                        "depth": lg["g_depth"], "count": lg["g_count"]})
        for k in PARAMS:
            total[k] += g[k]
    return total, losses


def _trainer(sc, gts, lc, lr=1e-3, cfg=None, **kw):
    dev = [gaussians_to_device(s) for s in sc.sets]
    renders = [dict(set=rd.set_index, camera=rd.camera, mask=torch.from_numpy(np.ascontiguousarray(rd.mask)).cuda())
               for rd in sc.renders]
    gt = [torch.from_numpy(g).cuda() for g in gts]
    t = Trainer(dev, renders, gt, cfg or RenderConfig(tile=16), lc, lr=lr, **kw)
    t.fit()
    return t


@pytest.mark.parametrize("reduce", [0, 1])
def test_training_step_gradient_matches_oracle_chain(reduce):
    """Loss, backward and the raw-parameter gradients of one training step
    against the oracle's chain, under both backward reductions."""
    print(f"[case] train step gradient reduce={reduce}", flush=True)
    sc, gts, refs = _prepared_scene(401)
    lc = LossConfig(lambda_normal=0.2, normal_norm=2, lambda_load=0.41)
    olc = ol.LossConfig(lambda_normal=0.2, normal_norm=2, lambda_load=0.41)
    ref, lgs = _oracle_step_grads(sc, gts, refs, olc)
    t = _trainer(sc, gts, lc, lr=0.0, cfg=RenderConfig(tile=16, bwd_reduce=reduce), keep_grads=True)
    out = t.step().cpu().numpy()
    torch.cuda.synchronize()
    # the geometric terms (the load term is a value of the binning only)
    geo_gpu = (1 - 0.41) * (out[:, 1].astype(np.float64) + 0.2 * out[:, 2])
    np.testing.assert_allclose(geo_gpu, [lg["total"] for lg in lgs], rtol=1e-4)
    ex = np.zeros(sc.sets[0].n, bool)
    for rd in sc.renders:
        dec = op.decide(sc.sets[0], rd.camera, CFG)
        ex |= (dec.colour_min < 1e-5) | (dec.clamp_margin < 1e-5) | (dec.flip_margin < 1e-5)
    for k in PARAMS:
        got = t.batch.grads[0][k].cpu().numpy()
        ok, ratio, rel = grad_tolerance_check(got, ref[k], exclude=ex)
        assert ok, (k, ratio, rel)
    # lr = 0: the parameters are unchanged, the step counter advanced
    np.testing.assert_array_equal(t.params[0]["means"].cpu().numpy(), sc.sets[0].means)
    assert int(t.state[0]) == 1


@pytest.mark.parametrize("reduce", [0, 1])
def test_training_step_with_gc_load_matches_oracle_chain(reduce):
    """The GC-load of Eq. 9 as the balance-load term (lambda 0.41) with
    luminance weights: its value from the integer counts, its gradient
    through the soft count into every blended fragment's alpha, against the
    oracle's chain."""
    print(f"[case] train step with GC-load reduce={reduce}", flush=True)
    sc, gts, refs = _prepared_scene(403)
    ws = [ol.luminance_weights(gt, rd.mask).astype(np.float32) for gt, rd in zip(gts, sc.renders)]
    lc = LossConfig(lambda_normal=0.2, normal_norm=2, lambda_load=0.41, load_term=1)
    olc = ol.LossConfig(lambda_normal=0.2, normal_norm=2, lambda_load=0.41, load_term=1)
    ref, lgs = _oracle_step_grads(sc, gts, refs, olc, weights=ws)
    ref0, _ = _oracle_step_grads(sc, gts, refs, ol.LossConfig(lambda_normal=0.2, normal_norm=2, lambda_load=0.41))
    t = _trainer(sc, gts, lc, lr=0.0, cfg=RenderConfig(tile=16, bwd_reduce=reduce), keep_grads=True,
                 weights=[torch.from_numpy(w).cuda() for w in ws])
    out = t.step().cpu().numpy()
    torch.cuda.synchronize()
    np.testing.assert_allclose(out[:, 3], [lg["load"] for lg in lgs], rtol=1e-5)
    np.testing.assert_allclose(out[:, 0], [lg["total"] for lg in lgs], rtol=1e-4)
    ex = np.zeros(sc.sets[0].n, bool)
    for rd in sc.renders:
        dec = op.decide(sc.sets[0], rd.camera, CFG)
        ex |= (dec.colour_min < 1e-5) | (dec.clamp_margin < 1e-5) | (dec.flip_margin < 1e-5)
    for k in PARAMS:
        got = t.batch.grads[0][k].cpu().numpy()
        ok, ratio, rel = grad_tolerance_check(got, ref[k], exclude=ex)
        assert ok, (k, ratio, rel)
    # the term does steer the counts: the opacity gradient differs from the
    # value-only (tile-variance) term's
    d = np.abs(ref["opacity_logits"] - ref0["opacity_logits"]).max()
    assert d > 1e-3 * np.abs(ref0["opacity_logits"]).max()


@pytest.mark.parametrize("det", [False, True])
def test_captured_training_step_replays_like_eager_steps(det):
    """Three replays of a captured training step against three eager steps:
    bit-identical parameters with the deterministic backward; with float
    atomics the gradients differ by addition order only."""
    print(f"[case] train graph replay det={det}", flush=True)
    sc, gts, _ = _prepared_scene(402)
    lc = LossConfig(lambda_load=0.41)
    cfg = RenderConfig(tile=16, deterministic=det)
    a = _trainer(sc, gts, lc, cfg=cfg)
    b = _trainer(sc, gts, lc, cfg=cfg)
    la = [a.step().clone() for _ in range(3)]
    b.capture()          # capture records without running: the step counter is untouched
    assert int(b.state[0]) == 0
    lb = [b.replay().clone() for _ in range(3)]
    torch.cuda.synchronize()
    assert int(a.state[0]) == 3 and int(b.state[0]) == 3
    for x, y in zip(la, lb):
        np.testing.assert_allclose(y.cpu().numpy(), x.cpu().numpy(), rtol=1e-5, atol=1e-7)
    assert not a.overflowed() and not b.overflowed()
    pa, pb = a.P.cpu().numpy(), b.P.cpu().numpy()
    if det:
        np.testing.assert_array_equal(pb, pa)
        np.testing.assert_array_equal(b.m.cpu().numpy(), a.m.cpu().numpy())
        np.testing.assert_array_equal(b.v.cpu().numpy(), a.v.cpu().numpy())
    d = np.abs(pa - pb)
    # gradients differ only by the order of float atomics; Adam's first steps
    # move every coordinate by about lr, so compare the bulk tightly
    assert d.max() <= 6 * 1e-3
    assert np.mean(d <= 1e-6) > 0.999
    assert np.any(a.params[0]["means"].cpu().numpy() != sc.sets[0].means)


def test_device_step_adam_matches_host_step():
    rng = np.random.default_rng(3)
    n = 10_001
    p0, g1, g2 = (rng.normal(size=n).astype(np.float32) for _ in range(3))
    P = [torch.from_numpy(p0.copy()).cuda() for _ in range(2)]
    M = [torch.zeros(n, device="cuda") for _ in range(2)]
    V = [torch.zeros(n, device="cuda") for _ in range(2)]
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    for step, g in ((1, g1), (2, g2)):
        gt = torch.from_numpy(g).cuda()
        adam_step(P[0], gt, M[0], V[0], lr=1e-2, step=step)
        adam_step_device(P[1], gt, M[1], V[1], lr=1e-2, state=st)
    assert int(st[0]) == 2
    for x, y in ((P[0], P[1]), (M[0], M[1]), (V[0], V[1])):
        np.testing.assert_allclose(y.cpu().numpy(), x.cpu().numpy(), rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("sh_degree", [2, 3])
@pytest.mark.parametrize("keep_grads", [False, True])
def test_adam_folded_into_backward_matches_separate_update(keep_grads, sh_degree):
    """Three training steps with Adam folded into the backward projection
    against three with the separate Adam launch, both with the deterministic
    backward (so the gradients agree bit for bit while the parameters do):
    parameters and both moments elementwise; the separate run's update
    against the definition (FP64 Adam on the gradients it stored); with
    keep_grads the stored gradients of the folded run equal the separate
    run's.  Degree 2 updates the SH coefficients in groups of 3, degree 3 in
    groups of 8."""
    print(f"[case] fused backward+Adam keep_grads={keep_grads} sh_degree={sh_degree}", flush=True)
    sc, gts, _ = _prepared_scene(403, sh_degree)
    lc = LossConfig(lambda_load=0.41)
    cfg = RenderConfig(tile=16, deterministic=True)
    lr = 1e-3
    a = _trainer(sc, gts, lc, lr=lr, cfg=cfg, fused=False)
    b = _trainer(sc, gts, lc, lr=lr, cfg=cfg, fused=True, keep_grads=keep_grads)
    p_ref = a.P.cpu().numpy().astype(np.float64)
    m_ref = np.zeros_like(p_ref)
    v_ref = np.zeros_like(p_ref)
    f = lambda x: float(np.float32(x))
    for t in range(1, 4):
        la = a.step().clone()
        lb = b.step().clone()
        np.testing.assert_allclose(lb.cpu().numpy(), la.cpu().numpy(), rtol=1e-5, atol=1e-7)
        ga = a.G.cpu().numpy()
        if keep_grads:
            gb = b.G.cpu().numpy()
            if t == 1:   # same parameters, deterministic backward: the same bits
                np.testing.assert_array_equal(gb, ga)
            else:
                np.testing.assert_allclose(gb, ga, rtol=1e-4, atol=1e-6 * np.abs(ga).max())
        p_ref, m_ref, v_ref = oa.adam_step(p_ref, ga.astype(np.float64), m_ref, v_ref, f(lr), f(0.9), f(0.999),
                                           f(1e-8), t)
    torch.cuda.synchronize()
    assert int(a.state[0]) == 3 and int(b.state[0]) == 3
    for name, x, y, ref in (("P", a.P, b.P, p_ref), ("m", a.m, b.m, m_ref), ("v", a.v, b.v, v_ref)):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        scale = np.abs(x).max()
        # folded vs separate: the same FP32 update on (nearly) the same gradients
        np.testing.assert_allclose(y, x, rtol=1e-5, atol=1e-6 * scale, err_msg=name)
        # the separate update against the definition, on its own gradients
        np.testing.assert_allclose(x, ref, rtol=1e-5, atol=1e-7 * scale, err_msg=name)
    assert np.any(b.params[0]["means"].cpu().numpy() != sc.sets[0].means)
    gb = b.G.cpu().numpy()
    if not keep_grads:
        assert not np.any(gb), "gradients must not be stored without keep_grads"
