"""GPU backward parity: gradients of sum(gout * outputs) with respect to the
raw parameters against the FP64 oracle's vector-Jacobian product, plus the
autograd wrapper, batched-vs-loop gradients and the fused Adam update."""
import numpy as np
import pytest
import torch

import scenes
from oracle import adam as oa
from oracle import composite as oc
from oracle import project as op
from paper_2501_01677_amd.raster import MaskedRasterizer, RenderConfig, adam_step, gaussians_to_device
from gpu_common import CFG, device_scene, grad_tolerance_check

pytestmark = pytest.mark.gpu

PARAMS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _gouts(sc, seed, depth_scale=0.05):
    """Upstream gradients N(0,1) on masked pixels; unsafe pixels (a decision
    near its threshold) are zeroed for both implementations."""
    out = []
    for r, rd in enumerate(sc.renders):
        g = scenes.grad_outputs(seed + r, rd, scale={"depth": depth_scale})
        fw = oc.render(sc.sets[rd.set_index], rd.camera, rd.mask, CFG)
        unsafe = np.zeros((rd.camera.height, rd.camera.width), bool)
        unsafe[fw["pix"][:, 0], fw["pix"][:, 1]] = fw["unsafe"]
        for k in g:
            g[k] = (g[k] * ~unsafe).astype(np.float32)
        out.append(g)
    return out


def _excluded(gs, cams):
    """Gaussians whose gradient has a kink within FP32 reach in some view
    (colour clamp, Jacobian clamp, normal flip)."""
    ex = np.zeros(gs.n, bool)
    for cam in cams:
        dec = op.decide(gs, cam, CFG)
        ex |= (dec.colour_min < 1e-5) | (dec.clamp_margin < 1e-5) | (dec.flip_margin < 1e-5)
    return ex


def _check_grads(sc, b, gouts, label):
    for s, gs in enumerate(sc.sets):
        ref = {k: np.zeros(getattr(gs, k).shape) for k in PARAMS}
        cams = []
        for r, rd in enumerate(sc.renders):
            if rd.set_index != s:
                continue
            cams.append(rd.camera)
            g = oc.render_grad(gs, rd.camera, rd.mask, CFG, gouts[r])
            for k in PARAMS:
                ref[k] += g[k]
        ex = _excluded(gs, cams)
        for k in PARAMS:
            got = b.grads[s][k].cpu().numpy()
            ok, ratio, rel = grad_tolerance_check(got, ref[k], exclude=ex)
            assert ok, (label, s, k, ratio, rel)
            # Gaussians that touch no masked pixel get exactly zero
            touched = np.abs(ref[k]).reshape(-1, gs.n).max(0) > 0
            silent = ~touched & ~ex
            assert np.all(got.reshape(-1, gs.n)[:, silent] == 0), (label, k)


GRAD_SCENES = {
    "rects-sh1": lambda: scenes.small_scene(131, n=120, width=48, height=40, sh_degree=1),
    "full-sh3": lambda: scenes.small_scene(132, n=150, width=40, height=36, sh_degree=3, mask_kind="full"),
    "two-views-sh2": lambda: scenes.small_scene(133, n=150, width=44, height=38, sh_degree=2, n_views=2),
    "opaque-sh0": lambda: scenes.small_scene(134, n=200, width=40, height=40, sh_degree=0, logit_mu=3.0,
                                             mask_kind="full"),
}


@pytest.mark.parametrize("reduce", [0, 1])
@pytest.mark.parametrize("tile", [8, 16, 32])
@pytest.mark.parametrize("name", sorted(GRAD_SCENES))
def test_gradients_match_oracle(name, tile, reduce):
    """Both backward reductions (matrix cores, lane exchanges) against the oracle."""
    print(f"[case] backward {name} tile={tile} reduce={reduce}", flush=True)
    sc = GRAD_SCENES[name]()
    b = device_scene(sc, RenderConfig(tile=tile, bwd_reduce=reduce))
    b.forward()
    gouts = _gouts(sc, 1000)
    b.backward([{k: torch.from_numpy(v).cuda() for k, v in g.items()} for g in gouts])
    torch.cuda.synchronize()
    _check_grads(sc, b, gouts, (name, tile, reduce))


@pytest.mark.parametrize("reduce", [0, 1])
def test_persistent_backward_matches_oracle(reduce):
    print(f"[case] backward persistent reduce={reduce}", flush=True)
    sc = GRAD_SCENES["two-views-sh2"]()
    b = device_scene(sc, RenderConfig(tile=16, persistent=True, queue_chunk=3, bwd_reduce=reduce))
    b.forward()
    gouts = _gouts(sc, 2000)
    b.backward([{k: torch.from_numpy(v).cuda() for k, v in g.items()} for g in gouts])
    _check_grads(sc, b, gouts, "persistent")


def test_autograd_function_matches_direct_backward():
    print("[case] autograd", flush=True)
    sc = scenes.small_scene(141, n=200, width=50, height=40, sh_degree=2)
    dev = gaussians_to_device(sc.sets[0])
    for k in PARAMS:
        dev[k].requires_grad_(True)
    rd = sc.renders[0]
    mask = torch.from_numpy(rd.mask).cuda()
    rz = MaskedRasterizer([dev], [dict(set=0, camera=rd.camera, mask=mask)], RenderConfig(tile=16))
    out = rz()[0]
    g = {k: torch.randn_like(out[k]) for k in ("rgb", "normal", "dist", "alpha")}
    loss = sum((g[k] * out[k]).sum() for k in g)
    got = torch.autograd.grad(loss, [dev[k] for k in PARAMS])
    b = device_scene(sc, RenderConfig(tile=16))
    b.forward()
    gg = {k: g[k].detach() for k in g}
    gg["depth"] = torch.zeros_like(out["depth"])
    b.backward([gg])
    # two runs of the same kernels differ only by the order of float atomics
    for k, t in zip(PARAMS, got):
        scale = float(b.grads[0][k].abs().max())
        torch.testing.assert_close(t, b.grads[0][k], rtol=1e-5, atol=1e-6 * scale)


def test_autograd_function_refuses_a_stale_forward():
    """The backward differentiates the batch's latest forward with the
    parameters as they are: a second forward, or an in-place update of a
    parameter, before the backward is an error, not a silent wrong answer."""
    sc = scenes.small_scene(142, n=100, width=40, height=32, sh_degree=1)
    dev = gaussians_to_device(sc.sets[0])
    for k in PARAMS:
        dev[k].requires_grad_(True)
    rd = sc.renders[0]
    rz = MaskedRasterizer([dev], [dict(set=0, camera=rd.camera, mask=torch.from_numpy(rd.mask).cuda())],
                          RenderConfig(tile=16))
    first = rz()[0]
    second = rz()[0]
    with pytest.raises(RuntimeError, match="another forward"):
        first["rgb"].sum().backward()
    out = rz()[0]
    with torch.no_grad():
        dev["means"].add_(0.0)
    with pytest.raises(RuntimeError, match="modified in place"):
        out["rgb"].sum().backward()
    out = rz()[0]
    out["rgb"].sum().backward()
    assert dev["means"].grad is not None and torch.any(dev["means"].grad != 0)


@pytest.mark.parametrize("det", [False, True])
def test_batched_gradients_equal_loop(det):
    """Three sub-regions x two views in one persistent batched launch against
    each sub-region launched alone (plain launch): bit-identical in the
    deterministic mode; with float atomics the sums differ only by their
    addition order."""
    print(f"[case] batched gradients det={det}", flush=True)
    subs = [scenes.small_scene(150 + k, n=100 + 50 * k, width=40 + 6 * k, height=36, sh_degree=k % 4,
                               n_views=2) for k in range(3)]
    sets = [s.sets[0] for s in subs]
    renders = [scenes.Render(k, rd.camera, rd.mask) for k, s in enumerate(subs) for rd in s.renders]
    big = scenes.Scene(sets, renders)
    bb = device_scene(big, RenderConfig(tile=16, persistent=True, deterministic=det))
    bb.forward()
    rng = np.random.default_rng(0)
    gl = []
    for rd in renders:
        g = scenes.grad_outputs(int(rng.integers(1 << 30)), rd, scale={"depth": 0.05})
        gl.append({k: torch.from_numpy(v).cuda() for k, v in g.items()})
    bb.backward(gl)
    r = 0
    worst = 0.0
    for k, s in enumerate(subs):
        bs = device_scene(s, RenderConfig(tile=16, deterministic=det))
        bs.forward()
        bs.backward(gl[r:r + len(s.renders)])
        r += len(s.renders)
        for name in PARAMS:
            a, b = bb.grads[k][name], bs.grads[0][name]
            if det:
                assert torch.equal(a, b), (k, name)
            else:
                scale = float(b.abs().max())
                torch.testing.assert_close(a, b, rtol=1e-5, atol=1e-6 * scale)
                worst = max(worst, float(((a - b).abs() / (b.abs() + 1e-6 * scale)).max()))
    print(f"[info] batched vs loop worst relative deviation {worst:.3g}", flush=True)


DET_SCENES = {
    # 10k Gaussians on a full 256x256 frame (the small parity workload)
    "config1": lambda: scenes.config1(),
    "two-views-sh2": lambda: scenes.small_scene(133, n=150, width=44, height=38, sh_degree=2, n_views=2),
}


@pytest.mark.parametrize("reduce", [0, 1])
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_deterministic_backward_bit_reproducible_and_matches_oracle(tile, reduce):
    """Deterministic mode: three backward passes give bit-identical
    gradients, the persistent launch gives the same bits as the plain one,
    and the gradients meet the oracle tolerance."""
    print(f"[case] deterministic backward tile={tile} reduce={reduce}", flush=True)
    sc = DET_SCENES["two-views-sh2"]()
    gouts = _gouts(sc, 3000)
    gl = [{k: torch.from_numpy(v).cuda() for k, v in g.items()} for g in gouts]
    runs = []
    for persistent in (False, True):
        b = device_scene(sc, RenderConfig(tile=tile, bwd_reduce=reduce, deterministic=True, persistent=persistent,
                                          queue_chunk=2))
        b.forward()
        for _ in range(2 if persistent else 3):
            b.backward(gl)
            runs.append({k: b.grads[0][k].clone() for k in PARAMS})
    for r in runs[1:]:
        for k in PARAMS:
            assert torch.equal(r[k], runs[0][k]), k
    _check_grads(sc, b, gouts, ("det", tile, reduce))


@pytest.mark.parametrize("reduce", [0, 1])
def test_deterministic_backward_on_the_small_parity_workload(reduce):
    """10k Gaussians, 256x256, 16x16 tiles: repeated backward passes are
    bit-identical in the deterministic mode, and every repeated atomic-mode
    pass agrees with them to its addition-order rounding; how many
    atomic-mode elements change between runs is reported."""
    print(f"[case] deterministic backward config 1 reduce={reduce}", flush=True)
    sc = DET_SCENES["config1"]()
    rd = sc.renders[0]
    g = scenes.grad_outputs(77, rd, scale={"depth": 0.05})
    gl = [{k: torch.from_numpy(v).cuda() for k, v in g.items()}]
    res = {}
    for det in (True, False):
        b = device_scene(sc, RenderConfig(tile=16, bwd_reduce=reduce, deterministic=det))
        b.forward()
        out = []
        for _ in range(3):
            b.backward(gl)
            out.append(torch.cat([b.grads[0][k].reshape(-1) for k in PARAMS]).clone())
        res[det] = out
    for o in res[True][1:]:
        assert torch.equal(o, res[True][0])
    changed = sum(int((o != res[False][0]).sum()) for o in res[False][1:])
    print(f"[info] atomic mode: {changed} gradient elements changed between runs", flush=True)
    d = res[True][0]
    scale = float(d.abs().max())
    # every atomic-mode pass (each one starts from cleared 2D-gradient slots)
    for a in res[False]:
        torch.testing.assert_close(a, d, rtol=1e-5, atol=1e-6 * scale)


def test_empty_mask_gives_zero_gradients():
    sc = scenes.small_scene(161, n=80, width=30, height=30, mask_kind="empty")
    b = device_scene(sc)
    b.forward()
    g = scenes.grad_outputs(1, scenes.Render(0, sc.renders[0].camera, None))
    b.backward([{k: torch.from_numpy(v).cuda() for k, v in g.items()}])
    for k in PARAMS:
        assert not torch.any(b.grads[0][k]), k


@pytest.mark.parametrize("n", [1, 7, 4096, 100_003])
def test_adam_matches_definition(n):
    rng = np.random.default_rng(n)
    p0 = rng.normal(size=n).astype(np.float32)
    m0 = (rng.normal(size=n) * 0.1).astype(np.float32)
    v0 = (rng.uniform(size=n) * 0.01).astype(np.float32)
    g0 = rng.normal(size=n).astype(np.float32)
    p, m, v, g = (torch.from_numpy(x.copy()).cuda() for x in (p0, m0, v0, g0))
    adam_step(p, g, m, v, lr=1e-3, step=3)
    # the kernel receives FP32 hyperparameters; the oracle takes those exact values
    f = lambda x: float(np.float32(x))
    rp, rm, rv = oa.adam_step(p0, g0, m0, v0, f(1e-3), f(0.9), f(0.999), f(1e-8), 3)
    np.testing.assert_allclose(p.cpu().numpy(), rp, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(m.cpu().numpy(), rm, rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(v.cpu().numpy(), rv, rtol=1e-6, atol=1e-9)
    # an unaligned view takes the scalar path
    if n > 8:
        p, m, v, g = (torch.from_numpy(x.copy()).cuda() for x in (p0, m0, v0, g0))
        adam_step(p[1:], g[1:], m[1:], v[1:], lr=1e-3, step=3)
        np.testing.assert_allclose(p[1:].cpu().numpy(), rp[1:], rtol=1e-6, atol=1e-7)
