"""Pins of the loss oracle (Sec. 4.2 Eq. 8, Sec. 4.3 Eq. 9-11) against
closed forms, a library routine and finite differences."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

import scenes
from oracle import losses as ol


def _blob_mask(seed, H, W):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W]
    m = ((xx - W * 0.45) / (W * 0.35)) ** 2 + ((yy - H * 0.5) / (H * 0.38)) ** 2 < 1.0
    for _ in range(4):  # holes
        cx, cy = rng.uniform(0.3, 0.7) * W, rng.uniform(0.3, 0.7) * H
        m &= (xx - cx) ** 2 + (yy - cy) ** 2 > 4.0
    m[rng.integers(0, H, 6), rng.integers(0, W, 6)] = True  # isolated pixels
    m[:, -3:] = True  # touches the image border
    return m


def test_mask_boundary_matches_binary_erosion():
    for seed in range(3):
        m = _blob_mask(seed, 37, 53)
        cross = ndi.generate_binary_structure(2, 1)
        inner = ndi.binary_erosion(m, structure=cross, border_value=1)
        assert np.array_equal(ol.mask_boundary(m), m & ~inner)


def _plane_depth(cam, n, d):
    """Exact depth of the plane n . X = d along every pixel ray."""
    r = ol.pixel_rays(cam)
    return d / (n[0] * r[0] + n[1] * r[1] + n[2] * r[2])


def _cam(W=64, H=48):
    return scenes.pinhole(W, H, fx=300.0, fy=280.0, cx=37.3, cy=21.9)


@pytest.mark.parametrize("tilt", [(0.0, 0.0), (0.35, -0.2), (-0.5, 0.45)])
def test_depth_normals_of_a_plane_are_its_normal(tilt):
    cam = _cam()
    n = np.array([tilt[0], tilt[1], -1.0])
    n /= np.linalg.norm(n)          # faces the camera (n_z < 0)
    d = -5.0                        # the plane lies in front of the camera
    depth = _plane_depth(cam, n, d)
    assert np.all(depth > 0)
    m = _blob_mask(7, cam.height, cam.width)
    nd, exists = ol.depth_normals(torch.from_numpy(depth), m, cam)
    nd, exists = nd.numpy(), exists.numpy()
    # existence: brute force over the definition
    H, W = m.shape
    for v in range(H):
        for u in range(W):
            ok = lambda x, y: 0 <= x < W and 0 <= y < H and m[y, x]
            want = m[v, u] and (ok(u + 1, v) or ok(u - 1, v)) and (ok(u, v + 1) or ok(u, v - 1))
            assert exists[v, u] == want, (u, v)
    assert exists.sum() > 0.5 * m.sum()
    err = np.abs(nd[:, exists] - n[:, None]).max()
    assert err < 1e-10, err
    # one-sided pixels (boundary) are covered by the same check
    assert (exists & ol.mask_boundary(m)).sum() > 10


def test_depth_normal_orientation_fronto_parallel():
    cam = _cam(8, 6)
    depth = np.full((6, 8), 3.0)
    nd, ex = ol.depth_normals(torch.from_numpy(depth), np.ones((6, 8), bool), cam)
    assert ex.all()
    np.testing.assert_allclose(nd.numpy()[:, ex.numpy()], np.array([[0.0], [0.0], [-1.0]]) * np.ones((1, 48)),
                               atol=1e-12)


def _rot(axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


@pytest.mark.parametrize("norm", [1, 2])
def test_loss_closed_form_rotated_normals(norm):
    cam = _cam()
    H, W = cam.height, cam.width
    n = np.array([0.2, -0.1, -1.0])
    n /= np.linalg.norm(n)
    depth = _plane_depth(cam, n, -4.0)
    m = _blob_mask(3, H, W)
    Rr = _rot([0.3, 1.0, 0.2], 0.4)
    nr = Rr @ n
    scale = np.random.default_rng(0).uniform(0.2, 0.9, (H, W))
    normal = nr[:, None, None] * scale[None]             # |N| varies, direction fixed
    delta = np.array([0.25, -0.125, 0.5])
    gt = np.random.default_rng(1).uniform(0, 1, (3, H, W))
    rgb = gt + delta[:, None, None]
    lc = ol.LossConfig(normal_norm=norm, lambda_normal=0.01, boundary_weight=0.1)
    rgb_t, nrm_t, dep_t = (torch.from_numpy(x) for x in (rgb, normal, depth))
    l_rgb, l_ban = ol.geo_terms(rgb_t, nrm_t, dep_t, gt, m, cam, lc, normal32=normal.astype(np.float32))
    M = m.sum()
    assert abs(float(l_rgb) - np.abs(delta).sum() / 3.0) < 1e-12
    e = np.abs(n - nr).sum() if norm == 1 else 2.0 - 2.0 * float(n @ nr)
    _, exists = ol.depth_normals(dep_t, m, cam)
    mb = ol.mask_boundary(m)
    wsum = np.where(mb, 0.1, 1.0)[exists.numpy()].sum()
    assert abs(float(l_ban) - wsum * e / M) < 1e-9 * max(1.0, wsum * e / M)


def test_unmasked_and_zero_normals_take_no_part():
    cam = _cam(20, 16)
    rng = np.random.default_rng(5)
    m = np.zeros((16, 20), bool)
    m[3:12, 4:15] = True
    depth = np.where(m, rng.uniform(2, 3, (16, 20)), 0.0)
    rgb, gt = rng.uniform(0, 1, (3, 16, 20)), rng.uniform(0, 1, (3, 16, 20))
    normal = rng.normal(size=(3, 16, 20))
    normal[:, 5, 6] = 0.0                                  # |N| = 0 inside the mask
    lc = ol.LossConfig()
    r = ol.loss_and_grads(rgb, normal, depth, gt, m, cam, lc)
    assert np.all(r["g_rgb"][:, ~m] == 0) and np.all(r["g_normal"][:, ~m] == 0) and np.all(r["g_depth"][~m] == 0)
    assert np.all(r["g_normal"][:, 5, 6] == 0)
    # changing anything outside the mask leaves the loss unchanged
    rgb2, normal2, depth2 = rgb.copy(), normal.copy(), depth.copy()
    rgb2[:, ~m] += 3.0
    normal2[:, ~m] *= -2.0
    r2 = ol.loss_and_grads(rgb2, normal2, depth2, gt, m, cam, lc)
    assert r2["total"] == r["total"]


def _smooth_inputs(seed, cam, m):
    """Inputs away from every kink: a curved depth surface, rendered normals
    far from the depth normals, colours away from the ground truth."""
    rng = np.random.default_rng(seed)
    H, W = cam.height, cam.width
    yy, xx = np.mgrid[0:H, 0:W] / 10.0
    depth = np.where(m, 3.0 + 0.3 * np.sin(xx) * np.cos(0.7 * yy) + 0.05 * xx, 0.0)
    normal = rng.normal(size=(3, H, W))
    gt = rng.uniform(0.2, 0.8, (3, H, W))
    rgb = gt + rng.choice([-1.0, 1.0], (3, H, W)) * rng.uniform(0.05, 0.2, (3, H, W))
    return rgb, normal, depth, gt


@pytest.mark.parametrize("norm", [1, 2])
def test_loss_gradients_match_finite_differences(norm):
    cam = _cam(14, 11)
    m = np.zeros((11, 14), bool)
    m[1:10, 2:13] = True
    m[4, 5] = False
    rgb, normal, depth, gt = _smooth_inputs(11, cam, m)
    lc = ol.LossConfig(normal_norm=norm, lambda_normal=0.7, lambda_load=0.3)
    mg = ol.sign_margins(rgb, normal, depth, gt, m, cam, lc)
    assert np.isfinite(mg).sum() > 40 and mg[np.isfinite(mg)].min() > 1e-4
    r = ol.loss_and_grads(rgb, normal, depth, gt, m, cam, lc, load_var=5.0)

    def f(rgb_, nrm_, dep_):
        with torch.no_grad():
            l1, l2 = ol.geo_terms(torch.from_numpy(rgb_), torch.from_numpy(nrm_), torch.from_numpy(dep_), gt, m,
                                  cam, lc, normal32=normal.astype(np.float32))
        return (1 - lc.lambda_load) * (lc.lambda_rgb * float(l1) + lc.lambda_normal * float(l2)) + lc.lambda_load * 5.0

    rng = np.random.default_rng(0)
    h = 1e-6
    for name, arr, g in (("rgb", rgb, r["g_rgb"]), ("normal", normal, r["g_normal"]), ("depth", depth, r["g_depth"])):
        flat = np.flatnonzero(np.broadcast_to(m, arr.shape) if arr.ndim == 3 else m)
        for idx in rng.choice(flat, 25, replace=False):
            a1, a2 = arr.copy().ravel(), arr.copy().ravel()
            a1[idx] += h
            a2[idx] -= h
            args1 = [rgb, normal, depth]
            args2 = [rgb, normal, depth]
            k = ("rgb", "normal", "depth").index(name)
            args1[k] = a1.reshape(arr.shape)
            args2[k] = a2.reshape(arr.shape)
            fd = (f(*args1) - f(*args2)) / (2 * h)
            assert abs(fd - g.ravel()[idx]) < 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, idx, fd, g.ravel()[idx])
    assert abs(r["total"] - f(rgb, normal, depth)) < 1e-12


def test_luminance_weights_closed_forms():
    H, W = 9, 12
    m = np.ones((H, W), bool)
    ramp = np.zeros((3, H, W))
    ramp[:] = 0.01 * np.arange(W)[None, None, :] + 0.02 * np.arange(H)[None, :, None]
    w = ol.luminance_weights(ramp, m)        # |grad Y| constant -> 0.1 + 1
    np.testing.assert_allclose(w, 1.1, rtol=0, atol=1e-12)
    # quadratic luminance: central differences are exact inside
    q = np.zeros((3, H, W))
    q[:] = (np.arange(W) ** 2)[None, None, :] * 1e-3
    w = ol.luminance_weights(q, m)
    gx = 2e-3 * np.arange(W).astype(float)
    gx[0], gx[-1] = 1e-3, (W - 1) ** 2 * 1e-3 - (W - 2) ** 2 * 1e-3   # one-sided at the border
    want = 0.1 + gx / gx.mean()
    np.testing.assert_allclose(w, np.broadcast_to(want, (H, W)), rtol=1e-12)
    # flat ground truth: no gradient information, all weights 1
    np.testing.assert_array_equal(ol.luminance_weights(np.ones((3, H, W)), m), 1.0)


def test_gc_load_and_tile_variance_closed_forms():
    m = np.zeros((4, 5), bool)
    m[1:3, 1:4] = True
    g = np.zeros((4, 5))
    g[1, 1:4] = 4
    g[2, 1:4] = 8
    w = np.full((4, 5), 2.0)
    assert abs(ol.gc_load(g, w, m) - 1.0) < 1e-15          # values 2 and 4, half each
    assert ol.gc_load(np.full((4, 5), 7), np.ones((4, 5)), m) == 0.0
    assert abs(ol.tile_load_variance([1, 3, 100, 5], [True, True, False, True]) - 8.0 / 3.0) < 1e-14


def test_gc_load_gradient_against_library_std():
    """Eq. 9's GC-load std(g / w) over masked pixels: its value is numpy's
    population std, its gradient in each g_i agrees with central
    differences of numpy.std, the weighted gradient sums to zero (a shift of
    every x_i leaves the std unchanged), and a constant x has none."""
    rng = np.random.default_rng(9)
    H, W = 6, 7
    m = rng.uniform(size=(H, W)) < 0.7
    g = rng.integers(0, 40, (H, W)).astype(np.float64)
    w = rng.uniform(0.1, 3.0, (H, W))
    val, grad = ol.gc_load_and_grad(g, w, m)
    assert abs(val - np.std(g[m] / w[m])) < 1e-14
    assert abs(val - ol.gc_load(g, w, m)) < 1e-14
    assert np.all(grad[~m] == 0)
    for i in np.flatnonzero(m.ravel())[:12]:
        h = 1e-5
        gp, gm = g.copy(), g.copy()
        gp.ravel()[i] += h
        gm.ravel()[i] -= h
        fd = (np.std(gp[m] / w[m]) - np.std(gm[m] / w[m])) / (2 * h)
        assert abs(fd - grad.ravel()[i]) <= 1e-8 * max(1.0, abs(fd)), (i, fd, grad.ravel()[i])
    assert abs((grad * w)[m].sum()) < 1e-12
    w2 = np.where(rng.uniform(size=(H, W)) < 0.5, 0.5, 2.0)   # x = g / w exactly 3
    v0, g0 = ol.gc_load_and_grad(3.0 * w2, w2, m)
    assert v0 < 1e-12 and np.all(g0 == 0)


def test_loss_with_the_gc_load_term():
    """load_term 1: L = (1 - lambda) L_geo + lambda std(g / w), and the
    soft-count gradient is lambda times that of the std; the geometric
    gradients are scaled by (1 - lambda) only."""
    cam = _cam(20, 16)
    m = _blob_mask(4, 16, 20)
    rng = np.random.default_rng(3)
    rgb = rng.uniform(0, 1, (3, 16, 20)).astype(np.float32)
    gt = rng.uniform(0, 1, (3, 16, 20)).astype(np.float32)
    nrm = np.zeros((3, 16, 20), np.float32)
    nrm[2] = -1
    dep = np.full((16, 20), 3.0, np.float32)
    nc = rng.integers(1, 30, (16, 20))
    w = rng.uniform(0.2, 2.0, (16, 20))
    lam = 0.41
    base = ol.loss_and_grads(rgb, nrm, dep, gt, m, cam, ol.LossConfig())
    lc = ol.LossConfig(lambda_load=lam, load_term=1)
    r = ol.loss_and_grads(rgb, nrm, dep, gt, m, cam, lc, n_contrib=nc, weight=w)
    val, grad = ol.gc_load_and_grad(nc, w, m)
    assert abs(r["load"] - val) < 1e-15
    assert abs(r["total"] - ((1 - lam) * base["total"] + lam * val)) < 1e-12
    np.testing.assert_allclose(r["g_count"], lam * grad, rtol=0, atol=1e-18)
    np.testing.assert_allclose(r["g_rgb"], (1 - lam) * base["g_rgb"], rtol=1e-12, atol=0)
    # the tile-variance term (load_term 0) carries no count gradient
    r0 = ol.loss_and_grads(rgb, nrm, dep, gt, m, cam, ol.LossConfig(lambda_load=lam), load_var=5.0)
    assert np.all(r0["g_count"] == 0) and r0["load"] == 5.0
