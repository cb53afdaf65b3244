"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test checks the oracle against something other than itself: closed
forms, brute-force expansions, library routines (scipy, numpy, torch.optim),
numerical Jacobians and finite differences.
"""
import math

import numpy as np
import pytest
import torch

import scenes
from oracle import OracleConfig
from oracle import composite as oc
from oracle import project as op
from oracle import sh as osh
from oracle import binning as ob
from oracle import adam as oa

CFG = OracleConfig()
Y00 = 0.5 / math.sqrt(math.pi)


def make_set(means, log_scales, quats, logits, colours=None, sh=None, deg=0):
    means = np.asarray(means, np.float32).T.copy()
    n = means.shape[1]
    if sh is None:
        colours = np.asarray(colours, np.float64).T  # [3, n]
        sh = ((colours - 0.5) / Y00)[None].astype(np.float32)
    return scenes.GaussianSet(means, np.asarray(log_scales, np.float32).T.copy(),
                              np.asarray(quats, np.float32).T.copy(),
                              np.asarray(logits, np.float32).copy(),
                              np.asarray(sh, np.float32), deg)


def cam_id(W=32, H=32, f=32.0):
    return scenes.pinhole(W, H, f, f)


def at_pixel(cam, u, v, z):
    """World point (camera = identity) projecting onto pixel centre (u, v)."""
    x = (u + 0.5 - cam.cx) * z / cam.fx
    y = (v + 0.5 - cam.cy) * z / cam.fy
    return [x, y, z]


def logit(o):
    return math.log(o / (1 - o))


# ------------------------------------------------------------------ SH

def test_legendre_matches_scipy():
    from scipy.special import lpmv
    z = torch.linspace(-0.99, 0.99, 41, dtype=torch.float64)
    q = osh.legendre_q(3, z)
    s = (1 - z * z).sqrt()
    for l in range(4):
        for m in range(l + 1):
            ours = (q[(l, m)] * s ** m).numpy()
            ref = lpmv(m, l, z.numpy())  # includes the Condon-Shortley phase
            np.testing.assert_allclose(ours, ref, rtol=1e-12, atol=1e-12)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for the degree <= 6
    # polynomials that products of degree <= 3 harmonics are.
    zn, zw = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phi = 2 * np.pi * np.arange(nphi) / nphi
    Z, P = np.meshgrid(zn, phi, indexing="ij")
    W = np.repeat(zw[:, None], nphi, 1) * (2 * np.pi / nphi)
    s = np.sqrt(1 - Z ** 2)
    d = torch.tensor(np.stack([s * np.cos(P), s * np.sin(P), Z], -1).reshape(-1, 3))
    Y = osh.sh_basis(3, d).numpy()
    gram = (Y * W.reshape(-1)[None]) @ Y.T
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_sh_low_degree_closed_form():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = osh.sh_basis(1, torch.tensor(d)).numpy()
    c1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(Y[0], Y00, rtol=1e-14)
    np.testing.assert_allclose(Y[1], -c1 * d[:, 1], rtol=1e-13)
    np.testing.assert_allclose(Y[2], c1 * d[:, 2], rtol=1e-13)
    np.testing.assert_allclose(Y[3], -c1 * d[:, 0], rtol=1e-13)


# ----------------------------------------------------------- projection

def test_canonical_depth_is_fp32_without_fma():
    rng = np.random.default_rng(1)
    m = rng.normal(size=(3, 1000)).astype(np.float32)
    R = rng.normal(size=(3, 3)).astype(np.float32)
    t = rng.normal(size=3).astype(np.float32)
    tz = op.canonical_depth32(m, R, t)
    for i in range(0, 1000, 97):
        a = np.float32(R[2, 0] * m[0, i])
        b = np.float32(R[2, 1] * m[1, i])
        c = np.float32(R[2, 2] * m[2, i])
        ref = np.float32(np.float32(np.float32(a + b) + c) + t[2])
        assert tz[i] == ref


def test_isotropic_ewa_on_axis():
    cam = cam_id(64, 48, 50.0)
    sig, z = 0.05, 3.0
    gs = make_set([[0.0, 0.0, z]], [[math.log(sig)] * 3], [[0.3, -0.2, 0.5, 0.7]], [0.0],
                  colours=[[0.5, 0.5, 0.5]])
    prep = oc.prepare(gs, cam, None, CFG)
    cov = prep.proj["cov2d"].numpy()[0]
    s = np.float64(np.float32(sig))
    np.testing.assert_allclose(cov, [(50 * s / z) ** 2 + 0.3, 0.0, (50 * s / z) ** 2 + 0.3],
                               rtol=1e-6, atol=1e-12)


def test_ewa_matches_numerical_jacobian():
    rng = np.random.default_rng(3)
    cam = scenes.pinhole(80, 60, 70.0, 65.0, 41.0, 29.0)
    n = 20
    means = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.4, 0.4, n), rng.uniform(2, 4, n)], 1)
    ls = rng.uniform(-3, -1, (n, 3))
    q = rng.normal(size=(n, 4))
    gs = make_set(means, ls, q, np.zeros(n), colours=np.full((n, 3), 0.5))
    prep = oc.prepare(gs, cam, None, CFG)
    cov = prep.proj["cov2d"].numpy()
    for k, i in enumerate(prep.dec.order):
        t = gs.means[:, i].astype(np.float64)
        h = 1e-6

        def proj2(tt):
            return np.array([cam.fx * tt[0] / tt[2] + cam.cx, cam.fy * tt[1] / tt[2] + cam.cy])
        J = np.stack([(proj2(t + h * e) - proj2(t - h * e)) / (2 * h) for e in np.eye(3)], 1)
        qq = gs.quats[:, i].astype(np.float64)
        qq /= np.linalg.norm(qq)
        w, x, y, z = qq
        # rotation from Rodrigues' formula (axis-angle), not the quaternion map
        ang = 2 * math.atan2(math.sqrt(x * x + y * y + z * z), w)
        ax = np.array([x, y, z]) / max(1e-300, math.sqrt(x * x + y * y + z * z))
        K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        Rr = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
        S = np.diag(np.exp(2 * gs.log_scales[:, i].astype(np.float64)))
        ref = J @ (Rr @ S @ Rr.T) @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(cov[k], [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-7, atol=1e-9)
        conic = prep.proj["conic"].numpy()[k]
        inv = np.linalg.inv(ref)
        np.testing.assert_allclose(conic, [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-6, atol=1e-9)


def test_culling_decisions():
    cam = cam_id()
    gs = make_set([[0, 0, 0.1], [0, 0, 0.2], [0, 0, 0.2000001], [0, 0, 3], [0, 0, 3]],
                  np.full((5, 3), -3.0), np.tile([1.0, 0, 0, 0], (5, 1)),
                  [0.0, 0.0, 0.0, -6.0, -5.5], colours=np.full((5, 3), 0.5))
    dec = op.decide(gs, cam, CFG)
    # depth <= 0.2 culled, logit below -ln 254 culled (o < 1/255)
    assert dec.visible.tolist() == [False, False, True, False, True]


# ------------------------------------------------------- compositing

def test_single_gaussian_at_pixel_centre():
    cam = cam_id(32, 32, 32.0)
    for o in (0.3, 0.995):
        col = [0.2, 0.7, 0.9]
        gs = make_set([at_pixel(cam, 10, 12, 2.5)], [[-3.0, -3.5, -4.0]], [[1.0, 0, 0, 0]],
                      [logit(o)], colours=[col])
        r = oc.render(gs, cam, None, CFG, mode="brute")
        im = r["images"]
        o32 = 1 / (1 + math.exp(-float(np.float32(logit(o)))))
        a = min(0.99, o32)
        c = np.float32((np.asarray(col, np.float64) - 0.5) / Y00).astype(np.float64) * Y00 + 0.5
        np.testing.assert_allclose(im["rgb"][:, 12, 10], a * c, rtol=1e-9)
        np.testing.assert_allclose(im["alpha"][12, 10], a, rtol=1e-9)
        # identity rotation, smallest scale on z: normal -z (faces the camera)
        np.testing.assert_allclose(im["normal"][:, 12, 10], [0, 0, -a], atol=1e-12)
        z = float(gs.means[2, 0])
        np.testing.assert_allclose(im["dist"][12, 10], -a * z, rtol=1e-9)
        # Eq. 4: depth of a fronto-parallel plane is its z whatever alpha is
        np.testing.assert_allclose(im["depth"][12, 10], z, rtol=1e-12)
        assert im["n_contrib"][12, 10] == 1


def test_two_and_three_gaussians_expansion():
    cam = cam_id(32, 32, 32.0)
    os_ = [0.6, 0.5, 0.7]
    cols = [[0.9, 0.1, 0.2], [0.2, 0.8, 0.3], [0.4, 0.4, 0.9]]
    zs = [2.0, 3.0, 5.0]
    pts = [at_pixel(cam, 15, 15, z) for z in zs]
    # input order scrambled: compositing follows depth, not index
    perm = [2, 0, 1]
    gs = make_set([pts[i] for i in perm], [[-2.5, -2.6, -5.0]] * 3, [[1.0, 0, 0, 0]] * 3,
                  [logit(os_[i]) for i in perm], colours=[cols[i] for i in perm])
    r = oc.render(gs, cam, None, CFG, mode="brute")
    a = [1 / (1 + math.exp(-float(np.float32(logit(o))))) for o in os_]
    c = [np.float32((np.asarray(cc, np.float64) - 0.5) / Y00).astype(np.float64) * Y00 + 0.5
         for cc in cols]
    exp2 = a[0] * c[0] + (1 - a[0]) * a[1] * c[1]
    exp3 = exp2 + (1 - a[0]) * (1 - a[1]) * a[2] * c[2]
    np.testing.assert_allclose(r["images"]["rgb"][:, 15, 15], exp3, rtol=1e-9)
    np.testing.assert_allclose(r["images"]["alpha"][15, 15],
                               1 - (1 - a[0]) * (1 - a[1]) * (1 - a[2]), rtol=1e-12)
    # only the two front ones
    gs2 = make_set(pts[:2], [[-2.5, -2.6, -5.0]] * 2, [[1.0, 0, 0, 0]] * 2,
                   [logit(o) for o in os_[:2]], colours=cols[:2])
    r2 = oc.render(gs2, cam, None, CFG, mode="brute")
    np.testing.assert_allclose(r2["images"]["rgb"][:, 15, 15], exp2, rtol=1e-9)


def test_transmittance_stop_is_exclusive():
    # 0.99-opaque layers: T after k layers = 0.01^k; the second layer would
    # take T to 1e-4 exactly -> 0.01^2 = 1e-4 is not < 1e-4 -> included;
    # the third (1e-6) is not.
    cam = cam_id(32, 32, 32.0)
    pts = [at_pixel(cam, 8, 8, z) for z in (2.0, 2.5, 3.0, 3.5)]
    gs = make_set(pts, [[-2.0, -2.0, -5.0]] * 4, [[1.0, 0, 0, 0]] * 4, [8.0] * 4,
                  colours=[[1, 1, 1]] * 4)
    r = oc.render(gs, cam, None, CFG, mode="brute", pixels=[(8, 8)])
    n = r["n_contrib"][0]
    a = 0.99
    T = 1.0
    k = 0
    for _ in range(4):
        if T * (1 - a) < 1e-4:
            break
        T *= (1 - a)
        k += 1
    assert n == k
    np.testing.assert_allclose(r["alpha"][0], 1 - T, rtol=1e-12)


def test_telescoping_and_monotone_transmittance():
    sc = scenes.small_scene(11, n=120, width=40, height=30, sh_degree=0, mask_kind="full")
    gs = sc.sets[0]
    # colour exactly 1 on every channel: rgb must equal 1 - T = alpha
    gs.sh[:] = np.float32(0.5 / Y00)
    cam = sc.renders[0].camera
    r = oc.render(gs, cam, None, CFG, mode="brute")
    c = float(np.float32(0.5 / Y00)) * Y00 + 0.5
    np.testing.assert_allclose(r["rgb"][:, 0] / c, r["alpha"], atol=1e-12)
    # transmittance along the depth order never increases
    prep = r["prep"]
    g = oc._geo(prep.proj, prep.dec)
    pix = torch.tensor([[7.5, 9.5], [20.5, 15.5], [33.5, 2.5]], dtype=torch.float64)
    dx = pix[:, 0:1] - g.mx[None]
    dy = pix[:, 1:2] - g.my[None]
    qq = g.a * dx * dx + 2 * g.b * dx * dy + g.c * dy * dy
    al = torch.clamp(g.o * torch.exp(-0.5 * qq), max=0.99)
    al = torch.where(al >= CFG.alpha_min, al, torch.zeros_like(al))
    T = torch.cumprod(1 - al, 1)
    assert torch.all(T[:, 1:] <= T[:, :-1])


def test_brute_equals_culled():
    sc = scenes.small_scene(5, n=300, width=70, height=50, sh_degree=2)
    gs, rd = sc.sets[0], sc.renders[0]
    b = oc.render(gs, rd.camera, rd.mask, CFG, mode="brute")
    c = oc.render(gs, rd.camera, rd.mask, CFG, mode="culled")
    for k in ("rgb", "normal", "dist", "depth", "alpha"):
        np.testing.assert_allclose(b[k], c[k], atol=1e-12, rtol=1e-12)
    assert np.array_equal(b["n_contrib"], c["n_contrib"])


def test_sub_cutoff_fragment_changes_nothing():
    sc = scenes.small_scene(6, n=40, width=32, height=32, sh_degree=0, mask_kind="full")
    gs, cam = sc.sets[0], sc.renders[0].camera
    base = oc.render(gs, cam, None, CFG, mode="brute")
    # a tiny Gaussian centred on a pixel corner with o = 0.0045: its alpha at
    # the nearest centres is 0.0045 * exp(-(0.25+0.25)/0.6) < 1/255
    p = at_pixel(cam, 10, 10, 3.0)
    p[0] += 0.5 * 3.0 / cam.fx
    p[1] += 0.5 * 3.0 / cam.fy
    extra = make_set([p], [[-12.0] * 3], [[1.0, 0, 0, 0]], [logit(0.0045)], colours=[[1, 0, 0]])
    gs2 = scenes.GaussianSet(np.concatenate([gs.means, extra.means], 1),
                             np.concatenate([gs.log_scales, extra.log_scales], 1),
                             np.concatenate([gs.quats, extra.quats], 1),
                             np.concatenate([gs.opacity_logits, extra.opacity_logits]),
                             np.concatenate([gs.sh, extra.sh], 2), 0)
    r2 = oc.render(gs2, cam, None, CFG, mode="brute")
    for k in ("rgb", "normal", "dist", "depth", "alpha", "n_contrib"):
        assert np.array_equal(base[k], r2[k])


def test_permutation_invariance():
    sc = scenes.small_scene(8, n=150, width=48, height=40, sh_degree=1)
    gs, rd = sc.sets[0], sc.renders[0]
    perm = np.random.default_rng(0).permutation(gs.n)
    gp = scenes.GaussianSet(gs.means[:, perm], gs.log_scales[:, perm], gs.quats[:, perm],
                            gs.opacity_logits[perm], gs.sh[:, :, perm], gs.sh_degree)
    a = oc.render(gs, rd.camera, rd.mask, CFG)
    b = oc.render(gp, rd.camera, rd.mask, CFG)
    tz = op.canonical_depth32(gs.means, rd.camera.R, rd.camera.t)
    assert len(np.unique(tz)) == gs.n  # distinct depths: order is a function of depth only
    for k in ("rgb", "normal", "dist", "alpha"):
        np.testing.assert_allclose(a[k], b[k], atol=1e-12)


def _plane_set(n0, point, normal, cam, rng, n=400, extent=1.5):
    normal = np.asarray(normal, float) / np.linalg.norm(normal)
    e1 = np.cross(normal, [0.3, 1.0, 0.2])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(normal, e1)
    uv = rng.uniform(-extent, extent, (n, 2))
    means = np.asarray(point) + uv[:, :1] * e1 + uv[:, 1:] * e2
    Rm = np.stack([e1, e2, normal], 1)
    if np.linalg.det(Rm) < 0:
        Rm[:, 0] *= -1
    q = scenes._rot_to_quat(np.repeat(Rm[None], n, 0)).T
    ls = np.tile([math.log(0.25), math.log(0.2), math.log(1e-4)], (n, 1))
    return make_set(means, ls, q, np.full(n, 2.0), colours=np.full((n, 3), 0.5))


def test_fronto_parallel_and_tilted_plane_depth():
    cam = scenes.pinhole(40, 30, 36.0, 36.0)
    rng = np.random.default_rng(2)
    z0 = 3.0
    gs = _plane_set(0, [0, 0, z0], [0, 0, 1], cam, rng)
    r = oc.render(gs, cam, None, CFG)
    cov = r["alpha"] > 0.5
    assert cov.mean() > 0.5
    # the plane is exactly flat only up to the FP32 rounding of the inputs
    np.testing.assert_allclose(r["depth"][cov], z0, rtol=1e-6)
    # tilted plane through P0 with normal n: depth = (n . P0) / (n . r)
    P0, nrm = np.array([0.1, -0.2, 3.5]), np.array([0.3, -0.2, -1.0])
    gs = _plane_set(0, P0, nrm, cam, rng, n=1500, extent=2.5)
    r = oc.render(gs, cam, None, CFG)
    cov = r["alpha"] > 0.5
    assert cov.mean() > 0.5
    pix = r["pix"][cov]
    ray = np.stack([(pix[:, 1] + 0.5 - cam.cx) / cam.fx, (pix[:, 0] + 0.5 - cam.cy) / cam.fy,
                    np.ones(len(pix))], 1)
    nu = nrm / np.linalg.norm(nrm)
    ref = (nu @ P0) / (ray @ nu)
    np.testing.assert_allclose(r["depth"][cov], ref, rtol=2e-5)


# ---------------------------------------------------- gradients (FD)

def _fd_scene(seed):
    sc = scenes.small_scene(seed, n=6, width=24, height=20, sh_degree=2, mask_kind="full",
                            logit_mu=0.5)
    gs, rd = sc.sets[0], sc.renders[0]
    gs.log_scales[:] = np.log(np.float32(0.12)) + np.random.default_rng(seed).uniform(
        -0.3, 0.3, gs.log_scales.shape).astype(np.float32)
    return gs, rd


@pytest.mark.parametrize("seed", [21, 22])
def test_gradient_matches_central_differences(seed):
    gs, rd = _fd_scene(seed)
    cam = rd.camera
    fw = oc.render(gs, cam, None, CFG, mode="brute")
    gout = scenes.grad_outputs(seed + 1000, rd)
    # pixels with a decision near its threshold are excluded from the loss
    unsafe = np.zeros((cam.height, cam.width), bool)
    unsafe[fw["pix"][:, 0], fw["pix"][:, 1]] = fw["unsafe"]
    for k in gout:
        gout[k] = gout[k] * ~unsafe
    # keep the depth loss small: it amplifies grazing pixels
    gout["depth"] = gout["depth"] * 0.05
    g = oc.render_grad(gs, cam, None, CFG, gout, mode="brute")
    rng = np.random.default_rng(seed)
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        arr = getattr(gs, name)
        flat = arr.reshape(-1)
        picks = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in picks:
            base = np.float64(flat[i])
            h = 1e-6 * max(1.0, abs(base))
            vals = []
            for s in (+1, -1):
                p64 = {k: np.asarray(v, np.float64).copy() for k, v in gs.arrays().items()}
                p64[name].reshape(-1)[i] = base + s * h
                vals.append(_loss64(gs, p64, cam, gout))
            fd = (vals[0] - vals[1]) / (2 * h)
            ad = g[name].reshape(-1)[i]
            assert abs(fd - ad) <= 1e-6 * max(1.0, abs(ad)) + 1e-7, (name, i, fd, ad)


def test_soft_count_closed_forms():
    """The soft contributor count (sum of alpha over the blended fragments,
    the differentiable stand-in for g_i of Eq. 9): one Gaussian at a pixel
    centre gives its alpha; three stacked ones give the plain sum of their
    alphas (not weighted by transmittance); behind opaque layers only the
    blended ones count."""
    cam = cam_id(32, 32, 32.0)
    o = 0.45
    gs = make_set([at_pixel(cam, 10, 12, 2.5)], [[-3.0, -3.5, -4.0]], [[1.0, 0, 0, 0]], [logit(o)],
                  colours=[[0.2, 0.7, 0.9]])
    r = oc.render(gs, cam, None, CFG, mode="brute")
    o32 = 1 / (1 + math.exp(-float(np.float32(logit(o)))))
    np.testing.assert_allclose(r["images"]["count"][12, 10], o32, rtol=1e-12)
    os_ = [0.6, 0.5, 0.7]
    pts = [at_pixel(cam, 15, 15, z) for z in (2.0, 3.0, 5.0)]
    gs3 = make_set(pts, [[-2.5, -2.6, -5.0]] * 3, [[1.0, 0, 0, 0]] * 3, [logit(v) for v in os_],
                   colours=[[0.5, 0.5, 0.5]] * 3)
    r3 = oc.render(gs3, cam, None, CFG, mode="brute", pixels=[(15, 15)])
    a = [1 / (1 + math.exp(-float(np.float32(logit(v))))) for v in os_]
    np.testing.assert_allclose(r3["count"][0], sum(a), rtol=1e-12)
    assert r3["n_contrib"][0] == 3
    # 0.99 layers: the stop leaves two blended, each alpha 0.99
    pts4 = [at_pixel(cam, 8, 8, z) for z in (2.0, 2.5, 3.0, 3.5)]
    gs4 = make_set(pts4, [[-2.0, -2.0, -5.0]] * 4, [[1.0, 0, 0, 0]] * 4, [8.0] * 4, colours=[[1, 1, 1]] * 4)
    r4 = oc.render(gs4, cam, None, CFG, mode="brute", pixels=[(8, 8)])
    assert r4["n_contrib"][0] == 2
    np.testing.assert_allclose(r4["count"][0], 2 * 0.99, rtol=1e-12)


def _count64(gs, p64, cam, c):
    """sum_p c_p count_p with perturbed FP64 parameters and the decisions of
    the unperturbed FP32 inputs."""
    dec = op.decide(gs, cam, CFG)
    p = {k: torch.tensor(v) for k, v in p64.items()}
    with torch.no_grad():
        proj = op.project(p, cam, dec, CFG)
        g = oc._geo(proj, dec)
        pix = oc._pixel_list(cam, None, None)
        pixf = torch.tensor(pix[:, ::-1] + 0.5, dtype=torch.float64)
        *_, count = oc.composite_block(pixf[:, 0], pixf[:, 1], g, CFG, want_allow=False)
    return float((torch.tensor(c[pix[:, 0], pix[:, 1]]) * count).sum())


def test_soft_count_gradient_by_central_differences():
    gs, rd = _fd_scene(23)
    cam = rd.camera
    fw = oc.render(gs, cam, None, CFG, mode="brute")
    c = np.random.default_rng(5).normal(size=(cam.height, cam.width))
    unsafe = np.zeros((cam.height, cam.width), bool)
    unsafe[fw["pix"][:, 0], fw["pix"][:, 1]] = fw["unsafe"]
    c = c * ~unsafe
    assert fw["images"]["count"].max() > 0.5
    g = oc.render_grad(gs, cam, None, CFG, {"count": c}, mode="brute")
    assert np.all(g["sh"] == 0)   # the count does not see colour
    rng = np.random.default_rng(23)
    for name in ("means", "log_scales", "quats", "opacity_logits"):
        flat = getattr(gs, name).reshape(-1)
        for i in rng.choice(flat.size, size=min(10, flat.size), replace=False):
            base = np.float64(flat[i])
            h = 1e-6 * max(1.0, abs(base))
            vals = []
            for sgn in (+1, -1):
                p64 = {k: np.asarray(v, np.float64).copy() for k, v in gs.arrays().items()}
                p64[name].reshape(-1)[i] = base + sgn * h
                vals.append(_count64(gs, p64, cam, c))
            fd = (vals[0] - vals[1]) / (2 * h)
            ad = g[name].reshape(-1)[i]
            assert abs(fd - ad) <= 1e-6 * max(1.0, abs(ad)) + 1e-7, (name, i, fd, ad)


def _loss64(gs, p64, cam, gout):
    """FP64 forward with perturbed FP64 parameters, decisions from the
    unperturbed FP32 inputs (they are all far from their thresholds)."""
    dec = op.decide(gs, cam, CFG)
    p = {k: torch.tensor(v) for k, v in p64.items()}
    with torch.no_grad():
        proj = op.project(p, cam, dec, CFG)
        g = oc._geo(proj, dec)
        pix = oc._pixel_list(cam, None, None)
        pixf = torch.tensor(pix[:, ::-1] + 0.5, dtype=torch.float64)
        F, T, n, _, _, count = oc.composite_block(pixf[:, 0], pixf[:, 1], g, CFG, want_allow=False)
        rgb, nrm, dist, depth, alpha, _, _ = oc._pixel_outputs(F, T, pixf, cam, CFG)
    tot = 0.0
    for name, val in (("rgb", rgb), ("normal", nrm), ("dist", dist), ("depth", depth), ("alpha", alpha),
                      ("count", count)):
        if name not in gout:
            continue
        c = 3 if val.dim() == 2 else 1
        gp = np.asarray(gout[name], np.float64).reshape(c, cam.height, cam.width)
        gv = gp[:, pix[:, 0], pix[:, 1]].T.reshape(val.shape)
        tot += float((torch.tensor(gv) * val).sum())
    return tot


def test_clamped_jacobian_gradient_by_fd():
    # a Gaussian far outside the frustum clamp still projects inside the
    # image when large; its gradient is the exact derivative of the clamped map
    cam = scenes.pinhole(24, 20, 20.0, 20.0)
    gs = make_set([[3.0 * 0.78 * 1.15, 0.1, 3.0]], [[math.log(1.2), math.log(0.9), math.log(0.5)]],
                  [[0.9, 0.1, 0.3, -0.2]], [1.0], colours=[[0.6, 0.3, 0.8]])
    dec = op.decide(gs, cam, CFG)
    assert dec.visible[0]
    limx = 1.3 * 12 / 20.0
    assert gs.means[0, 0] / gs.means[2, 0] > limx  # clamped
    rd = scenes.Render(0, cam, None)
    gout = scenes.grad_outputs(5, rd, channels=("rgb", "alpha"))
    fw = oc.render(gs, cam, None, CFG, mode="brute")
    assert fw["alpha"].max() > 0.05
    unsafe = np.zeros((cam.height, cam.width), bool)
    unsafe[fw["pix"][:, 0], fw["pix"][:, 1]] = fw["unsafe"]
    for k in gout:
        gout[k] = gout[k] * ~unsafe
    for k in ("normal", "dist", "depth"):
        gout[k] = np.zeros((cam.height, cam.width) if k != "normal" else (3, cam.height, cam.width), np.float32)
    g = oc.render_grad(gs, cam, None, CFG, gout, mode="brute")
    for name, i in (("means", 0), ("means", 2), ("log_scales", 1), ("quats", 3)):
        base = float(getattr(gs, name).reshape(-1)[i])
        h = 1e-6 * max(1.0, abs(base))
        vals = []
        for s in (+1, -1):
            p64 = {k: np.asarray(v, np.float64).copy() for k, v in gs.arrays().items()}
            p64[name].reshape(-1)[i] = base + s * h
            vals.append(_loss64(gs, p64, cam, gout))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[name].reshape(-1)[i]) <= 1e-6 * max(1, abs(fd)) + 1e-7


# ----------------------------------------------------------- binning

def test_binning_matches_brute_force_per_tile():
    rng = np.random.default_rng(9)
    render_tiles = [(5, 4), (3, 7)]
    offs = [0, 20]
    total = 41
    active = rng.uniform(size=total) < 0.7
    n = 60
    rr = rng.integers(0, 2, n)
    rects = np.zeros((n, 4), np.int64)
    for i in range(n):
        tx, ty = render_tiles[rr[i]]
        x0, x1 = sorted(rng.integers(0, tx + 1, 2))
        y0, y1 = sorted(rng.integers(0, ty + 1, 2))
        rects[i] = (x0, y0, x1, y1)
    depth = rng.integers(0, 50, n).astype(np.uint32)  # many ties
    valid = rng.uniform(size=n) < 0.9
    keys, vals, ranges = ob.emit_and_sort(rects, depth, valid, rr, render_tiles, offs, active)
    k2, v2, r2 = ob.emit_and_sort_fast(rects, depth, valid, rr, render_tiles, offs, active)
    assert np.array_equal(keys, k2) and np.array_equal(vals, v2) and np.array_equal(ranges, r2)
    for r in range(2):
        tx_n, ty_n = render_tiles[r]
        for ty in range(ty_n):
            for tx in range(tx_n):
                gt = offs[r] + ty * tx_n + tx
                members = [i for i in range(n) if valid[i] and rr[i] == r and active[gt]
                           and rects[i, 0] <= tx < rects[i, 2] and rects[i, 1] <= ty < rects[i, 3]]
                members = sorted(members, key=lambda i: (int(depth[i]), i))
                s, e = ranges[gt]
                assert list(vals[s:e]) == members


def test_tile_mask_counts_brute():
    rng = np.random.default_rng(4)
    m = (rng.uniform(size=(37, 53)) < 0.3).astype(np.uint8)
    c = ob.tile_mask_counts(m, 53, 37, 16)
    tx, ty = ob.tile_grid(53, 37, 16)
    for y in range(ty):
        for x in range(tx):
            assert c[y * tx + x] == m[y * 16:(y + 1) * 16, x * 16:(x + 1) * 16].sum()


# -------------------------------------------------------------- Adam

def test_adam_matches_torch_optim():
    rng = np.random.default_rng(0)
    p0 = rng.normal(size=100)
    pt = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(100), np.zeros(100)
    for step in range(1, 6):
        g = rng.normal(size=100)
        pt.grad = torch.tensor(g)
        opt.step()
        p, m, v = oa.adam_step(p, g, m, v, 1e-2, 0.9, 0.999, 1e-8, step)
        np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_off_centre_alpha_is_ewa_gaussian():
    # alpha at an off-centre pixel = o * exp(-1/2 d^T Sigma'^-1 d) with
    # Sigma' built from a numerical Jacobian and Rodrigues' rotation
    cam = scenes.pinhole(40, 40, 40.0, 40.0)
    gs = make_set([[0.05, -0.03, 3.0]], [[math.log(0.08), math.log(0.05), math.log(0.02)]],
                  [[0.8, 0.3, -0.4, 0.2]], [logit(0.7)], colours=[[0.5, 0.5, 0.5]])
    r = oc.render(gs, cam, None, CFG, mode="brute")
    t = gs.means[:, 0].astype(np.float64)
    h = 1e-6

    def proj2(tt):
        return np.array([cam.fx * tt[0] / tt[2] + cam.cx, cam.fy * tt[1] / tt[2] + cam.cy])
    J = np.stack([(proj2(t + h * e) - proj2(t - h * e)) / (2 * h) for e in np.eye(3)], 1)
    qq = gs.quats[:, 0].astype(np.float64)
    qq /= np.linalg.norm(qq)
    ang = 2 * math.atan2(np.linalg.norm(qq[1:]), qq[0])
    ax = qq[1:] / np.linalg.norm(qq[1:])
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    Rr = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K
    S = np.diag(np.exp(2 * gs.log_scales[:, 0].astype(np.float64)))
    cov = J @ Rr @ S @ Rr.T @ J.T + 0.3 * np.eye(2)
    m = proj2(t)
    o = 1 / (1 + math.exp(-float(gs.opacity_logits[0])))
    checked = 0
    for (v, u) in [(v, u) for v in range(16, 24) for u in range(17, 25)]:
        d = np.array([u + 0.5, v + 0.5]) - m
        a = min(0.99, o * math.exp(-0.5 * d @ np.linalg.solve(cov, d)))
        if a < 1 / 255:
            continue
        checked += 1
        np.testing.assert_allclose(r["images"]["alpha"][v, u], a, rtol=1e-7)
    assert checked >= 6


def test_sh_colour_uses_world_view_direction():
    # rotated, translated camera; degree-1 colour depends on the unit vector
    # from the camera centre to the mean, in world coordinates
    R, t = scenes.look_at((1.0, -2.0, 0.5), (0.2, 0.1, 3.0), up=(0.0, -1.0, 0.0))
    cam = scenes.pinhole(40, 40, 40.0, 40.0, R=R, t=t)
    centre = np.array([1.0, -2.0, 0.5])
    mu = np.array([0.2, 0.1, 3.0])
    sh = np.zeros((4, 3, 1), np.float32)
    sh[0, :, 0] = [0.3, 0.1, -0.2]
    sh[1:, :, 0] = [[0.4, -0.3, 0.2], [0.1, 0.5, -0.4], [-0.2, 0.3, 0.6]]
    gs = make_set([mu], [[-2.0, -2.2, -4.0]], [[1.0, 0, 0, 0]], [logit(0.9)], sh=sh, deg=1)
    prep = oc.prepare(gs, cam, None, CFG)
    d = gs.means[:, 0].astype(np.float64) - (-(cam.R.astype(np.float64).T @ cam.t.astype(np.float64)))
    np.testing.assert_allclose(-(cam.R.astype(np.float64).T @ cam.t.astype(np.float64)), centre, atol=1e-6)
    d /= np.linalg.norm(d)
    c1 = math.sqrt(3 / (4 * math.pi))
    basis = np.array([Y00, -c1 * d[1], c1 * d[2], -c1 * d[0]])
    ref = np.maximum(basis @ sh[:, :, 0].astype(np.float64) + 0.5, 0)
    np.testing.assert_allclose(prep.proj["colour"].numpy()[0], ref, rtol=1e-12)


def test_tilted_plane_depth_with_rotated_camera():
    R, t = scenes.look_at((0.5, -0.3, -1.0), (0.0, 0.0, 3.0), up=(0.0, -1.0, 0.0))
    cam = scenes.pinhole(40, 30, 36.0, 36.0, R=R, t=t)
    rng = np.random.default_rng(12)
    P0, nrm = np.array([0.0, 0.1, 3.0]), np.array([0.2, 0.4, -1.0])
    gs = _plane_set(0, P0, nrm, cam, rng, n=2500, extent=3.0)
    r = oc.render(gs, cam, None, CFG)
    cov = r["alpha"] > 0.5
    assert cov.mean() > 0.4
    pix = r["pix"][cov]
    ray_c = np.stack([(pix[:, 1] + 0.5 - cam.cx) / cam.fx, (pix[:, 0] + 0.5 - cam.cy) / cam.fy,
                      np.ones(len(pix))], 1)
    Rc, tc = cam.R.astype(np.float64), cam.t.astype(np.float64)
    n_c = Rc @ (nrm / np.linalg.norm(nrm))
    p0_c = Rc @ P0 + tc
    ref = (n_c @ p0_c) / (ray_c @ n_c)
    np.testing.assert_allclose(r["depth"][cov], ref, rtol=2e-5)
    # rendered normal faces the camera: n . ray < 0
    assert np.all((r["normal"][cov] * ray_c).sum(1) < 0)


# ------------------------------------------- Jacobian clamp (reading R5)

def _rodrigues(qq):
    """Rotation of a unit quaternion (w, x, y, z) from its axis and angle."""
    qq = np.asarray(qq, np.float64) / np.linalg.norm(qq)
    w, x, y, z = qq
    s = math.sqrt(x * x + y * y + z * z)
    ang = 2 * math.atan2(s, w)
    ax = np.array([x, y, z]) / max(s, 1e-300)
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def _numerical_pinhole_jacobian(cam, p):
    """2x3 Jacobian of the pinhole map (x, y, z) -> (fx x/z + cx, fy y/z + cy)
    at camera point p, by FP64 central differences."""
    def proj(tt):
        return np.array([cam.fx * tt[0] / tt[2] + cam.cx, cam.fy * tt[1] / tt[2] + cam.cy])
    h = 1e-6
    return np.stack([(proj(p + h * e) - proj(p - h * e)) / (2 * h) for e in np.eye(3)], 1)


def test_jacobian_clamp_beyond_the_lateral_limit():
    """A Gaussian far off to the side is projected with the Jacobian of the
    pinhole map taken at its mean pulled back to the lateral limit
    1.3 x tan(half field of view) (the half image over the focal length) per
    axis, at the same depth; its 2D mean is not clamped.  Three Gaussians:
    clamped in x, clamped in y, clamped in both, under a rotated camera."""
    W, H, f = 24, 20, 20.0
    R, t = scenes.look_at([0.3, -0.2, -4.0], [0.1, 0.2, 0.0], up=(0.0, -1.0, 0.0))
    cam = scenes.pinhole(W, H, f, f, 11.0, 10.5, R, t)
    Rc, tc = cam.R.astype(np.float64), cam.t.astype(np.float64)
    limx, limy = 1.3 * (W / 2) / cam.fx, 1.3 * (H / 2) / cam.fy
    # camera-frame targets: x/z 1.4 limx; y/z -1.3 limy; both
    cam_pts = np.array([[1.4 * limx * 3.0, 0.1, 3.0],
                        [0.2, -1.3 * limy * 2.5, 2.5],
                        [-1.25 * limx * 4.0, 1.2 * limy * 4.0, 4.0]])
    means = (cam_pts - tc) @ Rc                       # world = R^T (x_c - t)
    rng = np.random.default_rng(8)
    ls = rng.uniform(-1.5, -0.5, (3, 3))
    q = rng.normal(size=(3, 4))
    gs = make_set(means, ls, q, np.zeros(3), colours=np.full((3, 3), 0.5))
    prep = oc.prepare(gs, cam, None, CFG)
    assert len(prep.dec.order) == 3
    cov = prep.proj["cov2d"].numpy()
    m2d = prep.proj["mean2d"].numpy()
    k_of = {int(i): k for k, i in enumerate(prep.dec.order)}
    teeth = []
    for i in range(3):
        k = k_of[i]
        p = Rc @ gs.means[:, i].astype(np.float64) + tc
        xr, yr = p[0] / p[2], p[1] / p[2]
        clamped = np.array([np.clip(xr, -limx, limx) * p[2], np.clip(yr, -limy, limy) * p[2], p[2]])
        J = _numerical_pinhole_jacobian(cam, clamped)
        Rr = _rodrigues(gs.quats[:, i])
        Sig = Rc @ Rr @ np.diag(np.exp(2 * gs.log_scales[:, i].astype(np.float64))) @ Rr.T @ Rc.T
        ref = J @ Sig @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(cov[k], [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-6, atol=1e-9)
        # the 2D mean is the unclamped projection
        np.testing.assert_allclose(m2d[k], [cam.fx * xr + cam.cx, cam.fy * yr + cam.cy], rtol=1e-12)
        # the same covariance without the clamp, and with a limit of the whole
        # image over the focal length, are far from it: the pin has teeth
        for alt in (p, np.array([np.clip(xr, -2 * limx, 2 * limx) * p[2],
                                 np.clip(yr, -2 * limy, 2 * limy) * p[2], p[2]])):
            Ja = _numerical_pinhole_jacobian(cam, alt)
            ra = Ja @ Sig @ Ja.T + 0.3 * np.eye(2)
            teeth.append(np.abs(ra - ref).max() / np.abs(ref).max())
    assert min(teeth) > 1e-3, teeth


# ----------------------------------------------- Eq. 4 depth guard (R16)

def test_depth_guard_on_an_edge_on_plane():
    """Eq. 4 divides the blended distance by N . K^-1 p~; the reading sets the
    depth (and its gradient) to 0 unless that denominator is below -1e-6.
    One flat Gaussian whose plane is parallel to the ray of pixel (20, 16)
    (tilted by eps): the denominator there is alpha (n . r), computed here
    from an axis-angle rotation of the FP32 quaternion, and spans both sides
    of -1e-6 and of 0."""
    cam = scenes.pinhole(32, 32, 32.0, 32.0)
    u, v = 20, 16
    r = np.array([(u + 0.5 - cam.cx) / cam.fx, (v + 0.5 - cam.cy) / cam.fy, 1.0])
    mean = at_pixel(cam, 16, 16, 3.0)
    ls = [math.log(2.0), math.log(1.0), math.log(1e-3)]   # axis 2 is the normal

    def one(eps):
        n = np.array([1.0, 0.0, -r[0] + eps])
        n /= np.linalg.norm(n)
        e1 = np.array([0.0, 1.0, 0.0])
        e0 = np.cross(e1, n)
        Rm = np.stack([e0, e1, n], 1)
        assert np.linalg.det(Rm) > 0
        q = scenes._rot_to_quat(Rm[None])[:, 0]
        return make_set([mean], [ls], [q], [logit(0.8)], colours=[[0.4, 0.5, 0.6]])

    res0 = oc.render(one(0.0), cam, None, CFG, mode="brute", pixels=[[v, u]])
    a0 = float(res0["alpha"][0])
    assert a0 > 0.1
    for target in (5e-7, -5e-7, -3e-6, 3e-6):
        nrm = math.sqrt(1 + r[0] ** 2)
        gs = one(target * nrm / a0)
        res = oc.render(gs, cam, None, CFG, mode="brute", pixels=[[v, u]])
        alpha, den = float(res["alpha"][0]), float(res["den"][0])
        n_ind = _rodrigues(gs.quats[:, 0])[:, 2]
        t_c = gs.means[:, 0].astype(np.float64)
        assert n_ind @ t_c < 0                              # faces the camera: no flip
        np.testing.assert_allclose(den, alpha * (n_ind @ r), rtol=1e-6, atol=1e-12)
        assert abs(den - target) < 0.3 * abs(target)        # the intended band
        depth = float(res["depth"][0])
        gout = {"depth": np.zeros((cam.height, cam.width), np.float32)}
        gout["depth"][v, u] = 1.0
        g = oc.render_grad(gs, cam, None, CFG, gout, mode="brute", pixels=[[v, u]])
        gmax = max(np.abs(x).max() for x in g.values())
        if den < -1e-6:
            # D / den, D = alpha (n . t) from the same independent normal
            np.testing.assert_allclose(depth, alpha * (n_ind @ t_c) / den, rtol=1e-5)
            assert gmax > 0
        else:
            assert depth == 0.0 and gmax == 0.0, (target, den, depth, gmax)
