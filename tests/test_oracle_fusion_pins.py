"""Pins of the fusion and TSDF oracle (Sec. 4.4) against closed forms and
invariants fixed from outside its code: means of constant and single maps,
the FP64 mean, a fronto-parallel and a tilted plane (the TSDF value of every
voxel in closed form, the zero crossing at the plane), empty and repeated
views, and the generator's depth maps."""
import numpy as np
import pytest

import scenes
from oracle import fusion as of
from scenes import survey as sv


def test_fusion_means():
    rng = np.random.default_rng(0)
    H, W = 20, 30
    a = rng.uniform(1, 50, (H, W)).astype(np.float32)
    # one map: copied; constant maps: unchanged; nothing: zero
    f, n = of.fuse_depth([a])
    assert np.array_equal(f, a) and np.all(n == 1)
    f, n = of.fuse_depth([a, a])
    assert np.array_equal(f, a) and np.all(n == 2)  # a + a and the halving are exact
    f, n = of.fuse_depth([a, a, a])
    assert np.all(np.abs(f - a) <= np.spacing(a)) and np.all(n == 3)  # a + a + a rounds once
    z = np.zeros_like(a)
    f, n = of.fuse_depth([z, z])
    assert not f.any() and not n.any()
    # holes are skipped: a map with a hole contributes nothing there
    b = rng.uniform(1, 50, (H, W)).astype(np.float32)
    b[::3, ::2] = 0
    c = rng.uniform(1, 50, (H, W)).astype(np.float32)
    f, n = of.fuse_depth([a, b, c])
    ref = (a.astype(np.float64) + b + c) / np.where(b > 0, 3, 2)
    assert np.array_equal(n, np.where(b > 0, 3, 2))
    assert np.all(np.abs(f - ref) <= 4 * np.spacing(ref.astype(np.float32)))


def _axis_camera(W=64, H=48, f=40.0):
    return scenes.pinhole(W, H, f, f, W / 2, H / 2)


def test_tsdf_fronto_parallel_plane_closed_form():
    cam = _axis_camera()
    z0, trunc, vox = 10.0, 1.0, 0.25
    D = np.full((cam.height, cam.width), z0, np.float32)
    origin = np.array([-0.5, -0.5, 7.0], np.float32)  # a 4 x 4 x 24 column around the axis
    dims = (4, 4, 24)
    tsdf, w = of.integrate(origin, vox, dims, [cam], [D], trunc)
    zc = 7.0 + (np.arange(24) + 0.5) * vox
    want = np.minimum(1.0, (z0 - zc) / trunc)
    seen = zc <= z0 + trunc
    got = tsdf.reshape(24, 4, 4)
    wg = w.reshape(24, 4, 4)
    assert np.all(wg[seen] == 1) and np.all(wg[~seen] == 0)
    assert np.allclose(got[seen], want[seen][:, None, None], atol=1e-6)
    assert np.all(got[~seen] == 1.0)
    # the zero crossing of the linear interpolation along the axis is the plane
    col = got[:, 1, 1]
    k = np.flatnonzero((col[:-1] > 0) & (col[1:] <= 0))[0]
    zx = zc[k] + vox * col[k] / (col[k] - col[k + 1])
    assert abs(zx - z0) < 1e-5


def test_tsdf_tilted_plane_every_voxel():
    """Camera at the origin looking at the plane z = 12 + 0.3 x; the depth
    of each pixel is the plane's depth along that pixel's centre ray, and
    the TSDF of each voxel is (depth at its pixel - its depth) / trunc,
    clamped at 1, on voxels well inside the truncation band and away from
    pixel edges."""
    cam = _axis_camera(80, 60, 50.0)
    u = (np.arange(cam.width) + 0.5 - cam.cx) / cam.fx
    D = np.repeat((12.0 / (1.0 - 0.3 * u))[None, :], cam.height, 0).astype(np.float32)
    origin = np.array([-3.0, -2.0, 9.0], np.float32)
    vox, dims, trunc = 0.2, (30, 20, 30), 1.2
    tsdf, w = of.integrate(origin, vox, dims, [cam], [D], trunc)
    c = of.voxel_centres(origin, vox, dims).astype(np.float64)
    x, y, z = c
    up = cam.fx * x / z + cam.cx
    vp = cam.fy * y / z + cam.cy
    inside = (up >= 0) & (up < cam.width) & (vp >= 0) & (vp < cam.height) & (z > 0.2)
    iu = np.clip(np.floor(up), 0, cam.width - 1).astype(int)
    iv = np.clip(np.floor(vp), 0, cam.height - 1).astype(int)
    sdf = D[iv, iu].astype(np.float64) - z
    margin = np.minimum(np.abs(up - np.round(up)), np.abs(vp - np.round(vp))) > 1e-3
    band = inside & margin & (np.abs(sdf + trunc) > 1e-3)
    seen = band & (sdf >= -trunc)
    assert seen.sum() > 1000 and (band & ~seen).sum() > 100
    assert np.all(w[seen] == 1) and np.all(w[band & ~seen] == 0)
    assert np.allclose(tsdf[seen], np.minimum(1.0, sdf[seen] / trunc), atol=2e-6)
    assert np.all(w[~inside] == 0)


def test_tsdf_repeated_empty_and_back_views():
    cam = _axis_camera()
    D = np.full((cam.height, cam.width), 10.0, np.float32)
    D[:, : cam.width // 2] = 0  # left half: no depth
    origin = np.array([-2.0, -2.0, 8.0], np.float32)
    dims, vox, trunc = (16, 16, 16), 0.25, 1.0
    t1, w1 = of.integrate(origin, vox, dims, [cam], [D], trunc)
    t2, w2 = of.integrate(origin, vox, dims, [cam, cam], [D, D], trunc)
    assert np.array_equal(w2, 2 * w1) and np.allclose(t1, t2, atol=1e-12)
    t3, w3 = of.integrate(origin, vox, dims, [cam, cam], [D, np.zeros_like(D)], trunc)
    assert np.array_equal(w3, w1) and np.allclose(t3, t1, atol=1e-12)
    # voxels on the no-depth half are never updated
    c = of.voxel_centres(origin, vox, dims)
    left = cam.fx * c[0] / c[2] + cam.cx < cam.width // 2 - 0.01
    assert np.all(w1[left] == 0) and w1[~left].any()
    # a camera turned around sees nothing of the volume
    back = scenes.pinhole(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                          R=np.diag([-1.0, 1.0, -1.0]))
    _, wb = of.integrate(origin, vox, dims, [back], [D], trunc)
    assert not wb.any()


def test_generator_maps_fuse_to_the_box_surfaces():
    """On the stand-in depth stack the fused maps hold the visible surface
    (boxes and ground, rendered without noise) within the noise, overlaps
    (a box two groups share) average two noisy copies of one surface, and
    the fused map covers every pixel some map covers."""
    ds = sv.depth_small()
    overlaps = 0
    for cam, maps in zip(ds.cameras, ds.depths):
        f, n = of.fuse_depth(maps)
        clean = sv._ray_box_depth(cam, ds.boxes, ground=True)
        assert np.array_equal(f > 0, np.any(np.stack(maps) > 0, 0))
        both = (f > 0) & (clean > 0)
        assert both.mean() > 0.9
        overlaps += int((n >= 2).sum())
        rel = np.abs(f[both] - clean[both]) / clean[both]
        assert rel.max() < 5e-3 and np.median(rel) < 1e-3
    assert overlaps > 1000
