"""Parity at full size, in the launch configurations the benchmark times
(16x16 tiles), on outputs the oracle can compute one by one:

  * headline workload (1M Gaussians, SH degree 3, 1920x1080, rectangle-union
    mask): 1024 seeded masked pixels under the image tolerance protocol (the
    share of pixels carrying an allowance is reported and bounded), and a
    loss restricted to two 32x32 crops (dL/dout = 0 outside them and at the
    crops' near-threshold pixels, on both sides); every Gaussian whose
    oracle gradient is zero must get exactly zero;
  * 6M-Gaussian facade view at 4000x3000: 512 sampled pixels;
  * 16 sub-regions x 4 views at 1600x1200 in one persistent launch;
  * the training step at scale (10M facade Gaussians, two 5472x3648 views):
    256 sampled pixels per view, and the whole step -- forward, the loss of
    Sec. 4.2-4.3 (squared-L2 normal term, balance-load share 0.41), backward
    with the Adam update folded in at lr = 0 -- with the building mask cut to
    one 32x32 crop per view, each stage against the oracle on the same
    inputs (planes, loss gradients at the GPU's planes, parameter gradients
    of those loss gradients).
"""
import numpy as np
import pytest
import torch

import scenes
from oracle import composite as oc
from oracle import losses as ol
from oracle import project as op
from paper_2501_01677_amd.raster import LossConfig, RenderConfig, Trainer, gaussians_to_device
from gpu_common import CFG, check_unmasked_zero, compare_images, device_scene, grad_tolerance_check, outputs_numpy

pytestmark = pytest.mark.gpu

PARAMS = ("means", "log_scales", "quats", "opacity_logits", "sh")


@pytest.fixture(scope="module")
def headline():
    sc = scenes.config2()
    b = device_scene(sc, RenderConfig(tile=16))
    b.forward()
    b.fit_capacity(1.1)
    b.forward(check_overflow=False)
    torch.cuda.synchronize()
    return sc, b


def test_headline_forward_sampled_pixels(headline):
    print("[case] 1080p forward sample", flush=True)
    sc, b = headline
    rd = sc.renders[0]
    pix = scenes.sample_pixels(17, rd, 1024)
    ref = oc.render(sc.sets[0], rd.camera, rd.mask, CFG, pixels=pix)
    gpu = outputs_numpy(b, 0)
    rep = {}
    bad = compare_images(gpu, ref, rd, rep)
    assert not bad, bad
    # About 260 fragments are evaluated per pixel here, so a few percent of
    # the pixels hold some decision within the oracle's margins (alpha within
    # 1e-3 relative of the cut-off, T' within 1e-3 of the stop, a near edge-on
    # normal flip).  That share is a property of the workload and the oracle
    # alone (42 of these 1024 seeded pixels, 4.10%); those pixels are still
    # checked within tolerance + allowance above.  What the GPU's FP32
    # decisions actually change is the share of pixels whose error exceeds
    # the plain tolerance, i.e. that need their allowance at all.
    frac = rep["allow_pixels"] / rep["pixels"]
    used = rep["used_allowance"] / rep["pixels"]
    print(f"[info] 1080p sample: {rep['allow_pixels']} of {rep['pixels']} pixels carry an allowance "
          f"({100 * frac:.2f}%), {rep['used_allowance']} need it ({100 * used:.2f}%), "
          f"{rep['depth_excluded']} excluded from the depth check", flush=True)
    assert frac <= 0.045
    assert used <= 0.005
    assert check_unmasked_zero(gpu, rd.mask)
    assert int(b.status().overflow) == 0


def test_headline_gradients_on_crops(headline):
    print("[case] 1080p gradient crops", flush=True)
    sc, b = headline
    rd = sc.renders[0]
    gs = sc.sets[0]
    H, W = rd.camera.height, rd.camera.width
    crops = scenes.crop_windows(21, rd, count=2, size=32)
    sel = np.zeros((H, W), bool)
    for v0, u0, s in crops:
        sel[v0:v0 + s, u0:u0 + s] = True
    sel &= rd.mask.astype(bool)
    cp = np.argwhere(sel)
    fw = oc.render(gs, rd.camera, rd.mask, CFG, pixels=cp)
    sel[cp[fw["unsafe"], 0], cp[fw["unsafe"], 1]] = False
    g = scenes.grad_outputs(5, rd, scale={"depth": 0.05})
    g = {k: (v * sel).astype(np.float32) for k, v in g.items()}
    ref = oc.render_grad(gs, rd.camera, rd.mask, CFG, g, pixels=np.argwhere(sel))
    b.backward([{k: torch.from_numpy(v).cuda() for k, v in g.items()}])
    torch.cuda.synchronize()
    dec = op.decide(gs, rd.camera, CFG)
    ex = (dec.colour_min < 1e-5) | (dec.clamp_margin < 1e-5) | (dec.flip_margin < 1e-5)
    touched = np.zeros(gs.n, bool)
    for k in PARAMS:
        got = b.grads[0][k].cpu().numpy()
        ok, ratio, rel = grad_tolerance_check(got, ref[k], exclude=ex)
        assert ok, (k, ratio, rel)
        touched |= np.abs(ref[k]).reshape(-1, gs.n).max(0) > 0
    assert touched.sum() > 100
    silent = ~touched & ~ex
    for k in PARAMS:
        got = b.grads[0][k].cpu().numpy().reshape(-1, gs.n)
        assert np.all(got[:, silent] == 0), k


def test_facade_forward_sampled_pixels():
    """The 6M-Gaussian aerial facade workload at 4000x3000 with the
    box-silhouette mask: 512 seeded masked pixels against the oracle."""
    print("[case] facade 4000x3000 forward sample", flush=True)
    sc = scenes.config3()
    b = device_scene(sc, RenderConfig(tile=16), want_grads=False)
    b.forward()
    torch.cuda.synchronize()
    rd = sc.renders[0]
    pix = scenes.sample_pixels(19, rd, 512)
    ref = oc.render(sc.sets[0], rd.camera, rd.mask, CFG, pixels=pix)
    gpu = outputs_numpy(b, 0)
    bad = compare_images(gpu, ref, rd)
    assert not bad, bad
    assert check_unmasked_zero(gpu, rd.mask)
    assert ref["n_contrib"].mean() > 5


@pytest.mark.parametrize("reduce", [1, 0])
def test_batched_subregions_sampled_pixels_and_crop_gradients(reduce):
    """The 16 sub-region x 4 view batch (5.4M Gaussians, 1600x1200) in one
    persistent launch with 8-tile queue chunks and the lane-exchange backward
    reduction (the configuration the autotuner picks for it), and with the
    matrix-core reduction: 256 seeded pixels of six renders against the
    oracle, and the gradient of a loss on one 32x32 crop of the largest
    sub-region's render (every other render gets dL/dout = 0)."""
    print(f"[case] batched 16x4 samples + crop gradient reduce={reduce}", flush=True)
    sc = scenes.config4()
    b = device_scene(sc, RenderConfig(tile=16, persistent=True, queue_chunk=8, workgroups_per_cu=8,
                                      bwd_reduce=reduce))
    b.forward()
    b.fit_capacity(1.1)
    b.forward(check_overflow=False)
    torch.cuda.synchronize()
    big = int(np.argmax([s.n for s in sc.sets]))
    rds = [r for r, rd in enumerate(sc.renders) if rd.set_index == big][:2] + [0, 13, 38, 63]
    for r in rds:
        rd = sc.renders[r]
        pix = scenes.sample_pixels(23 + r, rd, 256)
        ref = oc.render(sc.sets[rd.set_index], rd.camera, rd.mask, CFG, pixels=pix)
        gpu = outputs_numpy(b, r)
        bad = compare_images(gpu, ref, rd)
        assert not bad, (r, bad)
    r = rds[0]
    rd = sc.renders[r]
    gs = sc.sets[rd.set_index]
    H, W = rd.camera.height, rd.camera.width
    (v0, u0, s), = scenes.crop_windows(29, rd, count=1, size=32)
    sel = np.zeros((H, W), bool)
    sel[v0:v0 + s, u0:u0 + s] = True
    sel &= rd.mask.astype(bool)
    cp = np.argwhere(sel)
    fw = oc.render(gs, rd.camera, rd.mask, CFG, pixels=cp)
    sel[cp[fw["unsafe"], 0], cp[fw["unsafe"], 1]] = False
    gouts = []
    for q, rq in enumerate(sc.renders):
        if q == r:
            g = scenes.grad_outputs(6, rq, scale={"depth": 0.05})
            g = {k: (v * sel).astype(np.float32) for k, v in g.items()}
            gsel = g
        else:
            g = {k: np.zeros_like(v) for k, v in scenes.grad_outputs(0, rq).items()}
        gouts.append({k: torch.from_numpy(v).cuda() for k, v in g.items()})
    b.backward(gouts)
    torch.cuda.synchronize()
    ref = oc.render_grad(gs, rd.camera, rd.mask, CFG, gsel, pixels=np.argwhere(sel))
    dec = op.decide(gs, rd.camera, CFG)
    ex = (dec.colour_min < 1e-5) | (dec.clamp_margin < 1e-5) | (dec.flip_margin < 1e-5)
    touched = np.zeros(gs.n, bool)
    for k in PARAMS:
        got = b.grads[rd.set_index][k].cpu().numpy()
        ok, ratio, rel = grad_tolerance_check(got, ref[k], exclude=ex)
        assert ok, (k, ratio, rel)
        touched |= np.abs(ref[k]).reshape(-1, gs.n).max(0) > 0
    assert touched.sum() > 20
    for k in PARAMS:
        got = b.grads[rd.set_index][k].cpu().numpy().reshape(-1, gs.n)
        assert np.all(got[:, ~touched & ~ex] == 0), k
    # the other sub-regions received no upstream gradient at all
    for s_idx in range(len(sc.sets)):
        if s_idx != rd.set_index:
            assert not torch.any(b.grads[s_idx]["means"]), s_idx


# ------------------------------------------------- training step at scale

@pytest.fixture(scope="module")
def training_scale():
    sc = scenes.config5()
    preps = [oc.prepare(sc.sets[0], rd.camera, None, CFG) for rd in sc.renders]
    return sc, preps


@pytest.mark.timeout(900)
def test_training_scale_forward_sampled_pixels(training_scale):
    """Both 5472x3648 views of the 10M-Gaussian facade workload in one batch:
    256 seeded masked pixels per view against the oracle."""
    print("[case] 10M facade 2x5472x3648 forward samples", flush=True)
    sc, preps = training_scale
    b = device_scene(sc, RenderConfig(tile=16), want_grads=False)
    b.forward()
    torch.cuda.synchronize()
    for r, rd in enumerate(sc.renders):
        pix = scenes.sample_pixels(31 + r, rd, 256)
        ref = oc.render(sc.sets[0], rd.camera, rd.mask, CFG, pixels=pix, prep=preps[r])
        gpu = outputs_numpy(b, r)
        rep = {}
        bad = compare_images(gpu, ref, rd, rep)
        assert not bad, (r, bad)
        assert check_unmasked_zero(gpu, rd.mask)
        assert ref["n_contrib"].mean() > 5
        print(f"[info] view {r}: {rep['allow_pixels']} of {rep['pixels']} pixels carry an allowance, "
              f"{rep['used_allowance']} need it", flush=True)
        assert rep["used_allowance"] <= 0.01 * rep["pixels"]
    assert int(b.status().overflow) == 0
    del b
    torch.cuda.empty_cache()


def _subset(gs, ids):
    """The Gaussians ``ids`` (ascending, so ties in depth keep their order)."""
    a = gs.arrays()
    return scenes.GaussianSet(*(np.ascontiguousarray(a[k][..., ids]) for k in
                                ("means", "log_scales", "quats", "opacity_logits", "sh")), gs.sh_degree)


@pytest.mark.timeout(900)
def test_training_scale_step_stages_match_oracle(training_scale):
    """The captured-size training step on the 10M-Gaussian two-view batch
    with each view's building mask cut to one 32x32 crop (less its
    near-threshold pixels): forward, the loss (squared-L2 normal term,
    balance-load share 0.41) and the backward with Adam folded in at lr = 0
    storing the gradients.  Each stage is compared with the oracle on the
    same inputs: the loss values and the loss gradients at the GPU's FP32
    planes, and the parameter gradients as the oracle's vector-Jacobian
    product of those loss gradients.  The oracle works on the Gaussians
    whose exact support meets a crop; every other Gaussian must get exactly
    zero gradient.

    The stages are not chained through the oracle's own planes: at these
    distances (about 770 m, 0.16 m per pixel) the depth-derived normal of
    Sec. 4.2 differentiates the depth over a two-pixel baseline, which
    multiplies the relative rounding of an FP32 depth (about 2e-6) some
    2400-fold.  The chained comparison is printed for reference."""
    print("[case] 10M facade training step, crop masks", flush=True)
    sc, preps = training_scale
    gs = sc.sets[0]
    crops = [scenes.crop_windows(37 + r, rd, count=1, size=32)[0] for r, rd in enumerate(sc.renders)]
    union = np.zeros(gs.n, bool)
    for (v0, u0, s), prep, rd in zip(crops, preps, sc.renders):
        px0, px1, py0, py1, *_, ne = op.support_rect(prep.proj, rd.camera, CFG, 1)
        hit = ne & (px1 >= u0 - 1) & (px0 <= u0 + s) & (py1 >= v0 - 1) & (py0 <= v0 + s)
        union[prep.dec.order[hit]] = True
    ids = np.flatnonzero(union)
    sub = _subset(gs, ids)
    olc = ol.LossConfig(lambda_normal=0.2, normal_norm=2, lambda_load=0.41)
    rng = np.random.default_rng(41)
    masks, gts, chain = [], [], []
    ex = np.zeros(sub.n, bool)
    for (v0, u0, s), rd in zip(crops, sc.renders):
        H, W = rd.camera.height, rd.camera.width
        sel = np.zeros((H, W), bool)
        sel[v0:v0 + s, u0:u0 + s] = True
        sel &= rd.mask.astype(bool)
        cp = np.argwhere(sel)
        fw = oc.render(sub, rd.camera, sel.astype(np.uint8), CFG, pixels=cp)
        bad = fw["unsafe"] | fw["depth_unreliable"]
        sel[cp[bad, 0], cp[bad, 1]] = False
        m1 = sel.astype(np.uint8)
        im = oc.render(sub, rd.camera, m1, CFG)["images"]
        off = rng.choice([-1.0, 1.0], (3, H, W)) * rng.uniform(0.02, 0.1, (3, H, W))
        gt = (im["rgb"] + off).astype(np.float32)
        chain.append(ol.loss_and_grads(*(im[k].astype(np.float32) for k in ("rgb", "normal", "depth")), gt, m1,
                                       rd.camera, olc))
        dec = op.decide(sub, rd.camera, CFG)
        ex |= (dec.colour_min < 1e-5) | (dec.clamp_margin < 1e-5) | (dec.flip_margin < 1e-5)
        masks.append(m1)
        gts.append(gt)
        print(f"[info] crop ({v0}, {u0}): {int(m1.sum())} masked pixels, {len(ids)} candidate Gaussians", flush=True)
    dev = [gaussians_to_device(gs)]
    renders = [dict(set=0, camera=rd.camera, mask=torch.from_numpy(m).cuda()) for rd, m in zip(sc.renders, masks)]
    t = Trainer(dev, renders, [torch.from_numpy(g).cuda() for g in gts], RenderConfig(tile=16),
                LossConfig(lambda_normal=0.2, normal_norm=2, lambda_load=0.41), lr=0.0, keep_grads=True)
    del dev
    t.fit()
    out = t.step().cpu().numpy()
    torch.cuda.synchronize()
    assert not t.overflowed()
    ref = {k: np.zeros(getattr(sub, k).shape) for k in PARAMS}
    ref_chain = {k: np.zeros(getattr(sub, k).shape) for k in PARAMS}
    for r, rd in enumerate(sc.renders):
        m = masks[r].astype(bool)
        planes = {k: t.batch.out[r][k].cpu().numpy() for k in ("rgb", "normal", "depth")}
        gout = {k: t.batch.gout[r][k].cpu().numpy() for k in ("rgb", "normal", "depth")}
        # the rendered planes at the crop pixels, under the image tolerances
        ref_px = oc.render(sub, rd.camera, masks[r], CFG, pixels=np.argwhere(m))
        rep = {}
        assert not compare_images({k: t.batch.out[r][k].cpu().numpy() for k in t.batch.out[r]}, ref_px, rd, rep)
        # loss values and gradients at the GPU's planes
        lg = ol.loss_and_grads(planes["rgb"], planes["normal"], planes["depth"], gts[r], masks[r], rd.camera, olc)
        np.testing.assert_allclose((1 - 0.41) * (out[r, 1].astype(np.float64) + 0.2 * out[r, 2]), lg["total"],
                                   rtol=1e-4)
        np.testing.assert_allclose(gout["rgb"][:, m], lg["g_rgb"][:, m], rtol=1e-6, atol=0)
        for ch in ("normal", "depth"):
            ok, ratio, rel = grad_tolerance_check(gout[ch][..., m], lg["g_" + ch][..., m])
            assert ok, ("loss gradient", ch, r, ratio, rel)
        g = oc.render_grad(sub, rd.camera, masks[r], CFG, gout)
        gc = oc.render_grad(sub, rd.camera, masks[r], CFG, {k: chain[r]["g_" + k] for k in ("rgb", "normal", "depth")})
        for k in PARAMS:
            ref[k] += g[k]
            ref_chain[k] += gc[k]
    for k in PARAMS:
        got = t.batch.grads[0][k].cpu().numpy()
        ok, ratio, rel = grad_tolerance_check(got[..., ids], ref[k], exclude=ex)
        _, cratio, crel = grad_tolerance_check(got[..., ids], ref_chain[k], exclude=ex)
        print(f"[info] {k}: worst ratio {ratio:.3f}, relative L2 {rel:.2e} "
              f"(chained through the oracle's planes: {cratio:.3f}, {crel:.2e})", flush=True)
        assert ok, (k, ratio, rel)
        # outside the crops' supports: exactly zero
        rest = np.ones(gs.n, bool)
        rest[ids] = False
        assert np.all(got.reshape(-1, gs.n)[:, rest] == 0), k
    # lr = 0: the parameters are unchanged, the step counter advanced
    np.testing.assert_array_equal(t.params[0]["means"].cpu().numpy(), gs.means)
    assert int(t.state[0]) == 1
