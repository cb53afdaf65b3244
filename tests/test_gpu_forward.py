"""GPU forward parity: projection records, binning, compositing and the
depth epilogue against the FP64 oracle, plus invariants and edge cases."""
import math

import numpy as np
import pytest
import torch

import scenes
from oracle import binning as ob
from oracle import composite as oc
from oracle import project as op
from paper_2501_01677_amd.raster import RenderConfig
from gpu_common import (CFG, check_unmasked_zero, compare_images, device_scene, outputs_numpy)

pytestmark = pytest.mark.gpu

SCENES = {
    "ragged-rects-sh1": lambda: scenes.small_scene(31, n=250, width=70, height=50, sh_degree=1),
    "full-sh3": lambda: scenes.small_scene(32, n=300, width=64, height=48, sh_degree=3, mask_kind="full"),
    "random-mask-sh2": lambda: scenes.small_scene(33, n=300, width=45, height=61, sh_degree=2,
                                                  mask_kind="random"),
    "three-views-sh3": lambda: scenes.small_scene(34, n=400, width=83, height=47, sh_degree=3, n_views=3),
    "opaque-sh0": lambda: scenes.small_scene(35, n=500, width=66, height=66, sh_degree=0, logit_mu=3.0,
                                             mask_kind="full"),
}


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("tile", [8, 16, 32])
@pytest.mark.parametrize("name", sorted(SCENES))
def test_forward_matches_oracle(name, tile):
    print(f"[case] forward {name} tile={tile}", flush=True)
    sc = SCENES[name]()
    b = device_scene(sc, RenderConfig(tile=tile))
    b.forward()
    torch.cuda.synchronize()
    for r, rd in enumerate(sc.renders):
        ref = oc.render(sc.sets[rd.set_index], rd.camera, rd.mask, CFG)
        gpu = outputs_numpy(b, r)
        bad = compare_images(gpu, ref, rd)
        assert not bad, (name, tile, r, bad)
        assert check_unmasked_zero(gpu, rd.mask)


def test_config1_full_frame_matches_oracle():
    print("[case] config1 forward", flush=True)
    sc = scenes.config1()
    b = device_scene(sc, RenderConfig(tile=16))
    b.forward()
    rd = sc.renders[0]
    ref = oc.render(sc.sets[0], rd.camera, None, CFG)
    rep = {}
    bad = compare_images(outputs_numpy(b, 0), ref, rd, rep)
    assert not bad, bad
    assert rep["allow_pixels"] < 0.01 * rep["pixels"]


def test_records_depth_keys_and_support_rects():
    print("[case] records", flush=True)
    sc = scenes.small_scene(41, n=600, width=90, height=70, sh_degree=3, n_views=2)
    tile = 16
    b = device_scene(sc, RenderConfig(tile=tile))
    b.forward()
    n = sc.sets[0].n
    nrec = int(b.info.n_records)
    rec = b.view("records", torch.float32, nrec, 16).cpu().numpy().astype(np.float64)
    nact = _u32(b.view("n_active", torch.int32, nrec))
    dkey = _u32(b.view("depth_key", torch.int32, nrec))
    rect = b.view("rect", torch.int16, nrec, 4).cpu().numpy().view(np.uint16).astype(np.int64)
    gs = sc.sets[0]
    p64 = op.params64(gs)
    checked = 0
    for r, rd in enumerate(sc.renders):
        cam = rd.camera
        sl = slice(r * n, (r + 1) * n)
        dec = op.decide(gs, cam, CFG)
        # depth-order key: bit-exact on every record
        assert np.array_equal(dkey[sl], dec.tz32.view(np.uint32))
        ids = np.flatnonzero(dec.visible)
        proj = op.project(p64, cam, dec, CFG, ids=ids)
        proj = {k: v.detach().numpy() for k, v in proj.items()}
        px0, px1, py0, py1, tx0, tx1, ty0, ty1, ne = op.support_rect(
            {k: torch.tensor(v) for k, v in proj.items()}, cam, CFG, tile)
        counts = ob.tile_mask_counts(rd.mask, cam.width, cam.height, tile)
        tiles_x, _ = ob.tile_grid(cam.width, cam.height, tile)
        active = (counts > 0).reshape(-1, tiles_x)
        R = rec[sl][ids]
        live = nact[sl][ids] > 0
        for j, i in enumerate(ids):
            has_active = ne[j] and active[ty0[j]:ty1[j], tx0[j]:tx1[j]].any()
            if has_active:
                assert live[j], ("visible Gaussian with active support not emitted", r, i)
            if not live[j]:
                continue
            checked += 1
            gr = rect[sl][i]
            # GPU tile rect contains the exact support, at most one tile wider per side
            if ne[j]:
                assert gr[0] <= tx0[j] and gr[1] <= ty0[j] and gr[2] >= tx1[j] and gr[3] >= ty1[j]
                assert gr[0] >= tx0[j] - 1 and gr[1] >= ty0[j] - 1 and gr[2] <= tx1[j] + 1 and gr[3] <= ty1[j] + 1
            np.testing.assert_allclose(R[j, 0:2], proj["mean2d"][j], rtol=1e-5, atol=1e-3)
            np.testing.assert_allclose(R[j, 2:5], proj["conic"][j], rtol=2e-4, atol=1e-6)
            np.testing.assert_allclose(R[j, 5], proj["opacity"][j], rtol=1e-5)
            np.testing.assert_allclose(R[j, 6:9], proj["colour"][j], rtol=1e-4, atol=2e-6)
            if dec.flip_margin[i] > 1e-5:
                np.testing.assert_allclose(R[j, 9:12], proj["normal"][j], atol=2e-6)
                np.testing.assert_allclose(R[j, 12], proj["dist"][j], rtol=1e-5, atol=1e-5)
    assert checked > 300


@pytest.mark.parametrize("tile", [8, 16, 32])
@pytest.mark.parametrize("W,H", [(300, 70), (70, 45), (1100, 40)])
def test_tile_counts_and_row_prefixes_bit_exact(W, H, tile):
    """Masked pixels per tile and the per-row prefix of active tiles, against
    the oracle's counts; widths that are multiples of 4 take the word-wise
    span counting, the others the byte-wise one."""
    print(f"[case] tile mask {W}x{H} tile={tile}", flush=True)
    sc = scenes.small_scene(300 + W + tile, n=40, width=W, height=H, sh_degree=0, n_views=2)
    b = device_scene(sc, RenderConfig(tile=tile), want_grads=False)
    b.forward()
    torch.cuda.synchronize()
    tc = _u32(b.view("tile_count", torch.int32, int(b.info.n_tiles)))
    toff = soff = 0
    sat_len = sum((t[0] + 1) * (t[1] + 1) for t in (ob.tile_grid(W, H, tile) for _ in sc.renders))
    sat = _u32(b.view("sat", torch.int32, sat_len))
    for rd in sc.renders:
        tx, ty = ob.tile_grid(W, H, tile)
        want = ob.tile_mask_counts(rd.mask, W, H, tile)
        assert np.array_equal(tc[toff:toff + tx * ty], want)
        act = (want.reshape(ty, tx) > 0).astype(np.uint32)
        rows = np.concatenate([np.zeros((ty, 1), np.uint32), np.cumsum(act, 1, dtype=np.uint32)], 1)
        assert np.array_equal(sat[soff:soff + ty * (tx + 1)].reshape(ty, tx + 1), rows)
        toff += tx * ty
        soff += (tx + 1) * (ty + 1)


def _emit_reference_inputs(b, sc, tile):
    """Per-render tile grids, offsets and active flags from the masks."""
    grids, offs, active = [], [], []
    off = 0
    for rd in sc.renders:
        tx, ty = ob.tile_grid(rd.camera.width, rd.camera.height, tile)
        grids.append((tx, ty))
        offs.append(off)
        active.append(ob.tile_mask_counts(rd.mask, rd.camera.width, rd.camera.height, tile) > 0)
        off += tx * ty
    return grids, offs, np.concatenate(active)


# rectangle kinds: (image size, largest width - 1 and height - 1 in tiles, pair capacity per record)
RECT_KINDS = {"small": ((300, 200), (4, 3), 64), "mid": ((600, 400), (11, 8), 200),
              "wide": ((1100, 300), (48, 14), 700)}


@pytest.mark.parametrize("n,seed,kind,det", [(300, 1, "small", False), (40_000, 2, "small", False),
                                             (20_000, 7, "mid", False), (20_000, 8, "mid", True),
                                             (3_000, 3, "wide", False), (8_000, 4, "wide", False),
                                             (8_000, 4, "wide", True), (60_000, 5, "wide", False),
                                             (60_000, 6, "wide", True), (2_100_000, 9, "small", False)])
def test_binning_bit_exact_on_synthetic_rects(n, seed, kind, det):
    """small: waves of fewer than 256 pairs (emission's balanced form).  mid:
    rectangles up to 8 rows x 11 columns, so waves of several hundred pairs
    whose rows all hold at most 12 active tiles take the row-lane form.
    wide: rectangles up to 48 x 14 tiles, so emission also takes its path for
    rectangles too large to stage (more than 8 rows or 32 columns).  The pair
    capacities select both radix chunk sizes (1024 keys, and 4096 from 2^19
    keys); the 60000-record cases hold tile lists of several thousand pairs.
    The 4.2M-record case takes the depth sort's 4096-key chunks and the
    emission's one-workgroup scan of the per-chunk pair totals (more than
    2048 chunks).  det: the deterministic configuration, whose tile sort
    carries emission indices."""
    print(f"[case] binning n={n} kind={kind} det={det}", flush=True)
    tile = 16
    (W, H), (mw, mh), cap = RECT_KINDS[kind]
    sc = scenes.small_scene(50 + seed, n=n, width=W, height=H, sh_degree=0, n_views=2)
    b = device_scene(sc, RenderConfig(tile=tile, deterministic=det), pair_capacity=cap * n)
    rng = np.random.default_rng(seed)
    nrec = int(b.info.n_records)
    grids, offs, active = _emit_reference_inputs(b, sc, tile)
    rr = np.repeat(np.arange(len(sc.renders)), n)
    rects = np.zeros((nrec, 4), np.int64)
    for r, (tx, ty) in enumerate(grids):
        m = rr == r
        k = int(m.sum())
        x0 = rng.integers(0, tx, k)
        y0 = rng.integers(0, ty, k)
        x1 = np.minimum(tx, x0 + rng.integers(0, mw + 1, k))
        y1 = np.minimum(ty, y0 + rng.integers(0, mh + 1, k))
        rects[m] = np.stack([x0, y0, x1, y1], 1)
    depth = rng.integers(0, 2000, nrec).astype(np.uint32) * np.uint32(1 << 20)  # ties and high bits
    depth[::7] = rng.integers(0, 2 ** 32, len(depth[::7]), dtype=np.uint64).astype(np.uint32)
    valid = rng.uniform(size=nrec) < 0.9
    b.view("rect", torch.int16, nrec, 4).copy_(torch.from_numpy(rects.astype(np.uint16).view(np.int16)))
    b.view("depth_key", torch.int32, nrec).copy_(torch.from_numpy(depth.view(np.int32)))
    b.view("n_active", torch.int32, nrec).copy_(torch.from_numpy(valid.astype(np.int32)))
    b.binning()
    st = b.status()
    keys, vals, ranges = ob.emit_and_sort_fast(rects, depth, valid, rr, grids, offs, active)
    assert st.overflow == 0
    assert st.pairs_needed == len(keys)
    K = len(keys)
    g_tile = _u32(b.view("pair_tile", torch.int32, K))
    g_rec = _u32(b.view("pair_record", torch.int32, K))
    g_rng = _u32(b.view("ranges", torch.int32, int(b.info.n_tiles), 2))
    assert np.array_equal(g_tile, (keys >> np.uint64(32)).astype(np.uint32))
    assert np.array_equal(g_rec, vals)
    assert np.array_equal(g_rng, ranges)


def test_forward_tile_lists_are_the_depth_ordered_support_sets():
    print("[case] tile lists", flush=True)
    tile = 16
    sc = scenes.small_scene(61, n=800, width=120, height=90, sh_degree=1, n_views=2)
    b = device_scene(sc, RenderConfig(tile=tile))
    b.forward()
    nrec = int(b.info.n_records)
    st = b.status()
    K = int(st.pairs_needed)
    rect = b.view("rect", torch.int16, nrec, 4).cpu().numpy().view(np.uint16).astype(np.int64)
    nact = _u32(b.view("n_active", torch.int32, nrec))
    dkey = _u32(b.view("depth_key", torch.int32, nrec))
    grids, offs, active = _emit_reference_inputs(b, sc, tile)
    rr = np.repeat(np.arange(len(sc.renders)), sc.sets[0].n)
    # depth keys are checked bit-exact against the oracle elsewhere; here the
    # per-tile lists must be exactly the records whose rectangle covers the
    # tile, in (depth key, record) order
    keys, vals, ranges = ob.emit_and_sort_fast(rect, dkey, nact > 0, rr, grids, offs, active)
    assert K == len(keys)
    assert np.array_equal(_u32(b.view("pair_record", torch.int32, K)), vals)
    assert np.array_equal(_u32(b.view("ranges", torch.int32, int(b.info.n_tiles), 2)), ranges)


def _all_outputs(b):
    return [outputs_numpy(b, r) for r in range(len(b.renders))]


@pytest.mark.parametrize("tile,reduce", [(8, 0), (16, 0), (16, 1), (32, 0)])
def test_compositing_work_counters_bound_the_blending(tile, reduce):
    """The per-(tile, wave) work counters: a wave evaluates at least as many
    list entries as any of its pixels blends fragments; in the backward the
    entries with a contributing pixel number at least that maximum and at
    most the wave's blended pairs and its evaluated entries; waves of tiles
    without masked pixels count nothing."""
    print(f"[case] work counters tile={tile} reduce={reduce}", flush=True)
    sc = scenes.small_scene(151, n=600, width=90, height=70, sh_degree=1)
    b = device_scene(sc, RenderConfig(tile=tile, bwd_reduce=reduce))
    b.forward()
    b.backward([{k: torch.from_numpy(v).cuda() for k, v in scenes.grad_outputs(3, rd).items()}
                for rd in sc.renders])
    torch.cuda.synchronize()
    rd = sc.renders[0]
    W, H = rd.camera.width, rd.camera.height
    tx, ty = (W + tile - 1) // tile, (H + tile - 1) // tile
    sb = tile // 8
    wpt = sb * sb
    work = b.view("work", torch.int32, tx * ty * wpt, 3).cpu().numpy().astype(np.int64)
    tc = b.view("tile_count", torch.int32, tx * ty).cpu().numpy()
    nc = np.zeros((ty * tile, tx * tile), np.int64)
    nc[:H, :W] = b.out[0]["n_contrib"].cpu().numpy()
    # per wave (8x8 block): max and sum of n_contrib
    blocks = nc.reshape(ty, sb, 8, tx, sb, 8).transpose(0, 3, 1, 4, 2, 5).reshape(ty * tx * wpt, 64)
    mx, sm = blocks.max(1), blocks.sum(1)
    active = np.repeat(tc > 0, wpt)
    assert np.all(work[~active] == 0)
    assert np.all(work[:, 0] >= mx)
    assert np.all(work[:, 2] >= mx) and np.all(work[:, 2] <= sm) and np.all(work[:, 2] <= work[:, 1])
    assert sm.sum() == int(b.out[0]["n_contrib"].sum()) and sm.sum() > 0


def test_invariants_tiles_persistent_mask_determinism():
    print("[case] invariants", flush=True)
    sc = scenes.small_scene(71, n=700, width=97, height=75, sh_degree=2, n_views=2)
    base = None
    for tile in (8, 16, 32):
        for persistent in (False, True):
            b = device_scene(sc, RenderConfig(tile=tile, persistent=persistent, queue_chunk=2))
            b.forward()
            outs = _all_outputs(b)
            if base is None:
                base = outs
                b.forward()
                again = _all_outputs(b)
                for o1, o2 in zip(base, again):
                    for k in o1:
                        assert np.array_equal(o1[k], o2[k]), ("determinism", k)
            else:
                for o1, o2 in zip(base, outs):
                    for k in o1:
                        assert np.array_equal(o1[k], o2[k]), (tile, persistent, k)
    # masked render == full render on the masked pixels, bit for bit
    full = scenes.Scene(sc.sets, [scenes.Render(r.set_index, r.camera, None) for r in sc.renders])
    bf = device_scene(full, RenderConfig(tile=16))
    bf.forward()
    outs_full = _all_outputs(bf)
    for r, rd in enumerate(sc.renders):
        m = rd.mask.astype(bool)
        for k in base[r]:
            a, f = base[r][k], outs_full[r][k]
            if a.ndim == 3:
                assert np.array_equal(a[:, m], f[:, m]), k
            else:
                assert np.array_equal(a[m], f[m]), k


def test_batched_equals_per_region_loop():
    print("[case] batched vs loop", flush=True)
    subs = [scenes.small_scene(80 + k, n=150 + 200 * k, width=60 + 10 * k, height=50, sh_degree=k % 4,
                               n_views=2) for k in range(4)]
    sets = [s.sets[0] for s in subs]
    renders = []
    for k, s in enumerate(subs):
        for rd in s.renders:
            renders.append(scenes.Render(k, rd.camera, rd.mask))
    big = scenes.Scene(sets, renders)
    for persistent in (False, True):
        bb = device_scene(big, RenderConfig(tile=16, persistent=persistent))
        bb.forward()
        r = 0
        for k, s in enumerate(subs):
            bs = device_scene(s, RenderConfig(tile=16))
            bs.forward()
            for v in range(len(s.renders)):
                o1, o2 = outputs_numpy(bb, r), outputs_numpy(bs, v)
                for key in o1:
                    assert np.array_equal(o1[key], o2[key]), (persistent, k, v, key)
                r += 1


def test_edge_cases_empty_mask_behind_camera_no_gaussians_tiny_image():
    print("[case] edge cases", flush=True)
    # empty mask: everything zero
    sc = scenes.small_scene(91, n=100, width=40, height=30, mask_kind="empty")
    b = device_scene(sc)
    b.forward()
    for k, a in outputs_numpy(b, 0).items():
        assert not np.any(a), k
    assert b.status().pairs_needed == 0
    # every Gaussian behind the camera
    sc = scenes.small_scene(92, n=100, width=40, height=30, mask_kind="full", depth=-4.0)
    b = device_scene(sc)
    b.forward()
    o = outputs_numpy(b, 0)
    assert not np.any(o["rgb"]) and not np.any(o["alpha"]) and not np.any(o["n_contrib"])
    # no Gaussians at all
    sc = scenes.small_scene(93, n=0, width=33, height=17, mask_kind="full")
    b = device_scene(sc)
    b.forward()
    assert not np.any(outputs_numpy(b, 0)["alpha"])
    # a 1x1 image
    sc = scenes.small_scene(94, n=50, width=1, height=1, mask_kind="full", depth=2.0)
    b = device_scene(sc)
    b.forward()
    ref = oc.render(sc.sets[0], sc.renders[0].camera, None, CFG)
    assert not compare_images(outputs_numpy(b, 0), ref, sc.renders[0])


def test_capacity_overflow_is_flagged_and_replanned():
    print("[case] capacity", flush=True)
    sc = scenes.small_scene(95, n=500, width=80, height=60, mask_kind="full")
    ref_b = device_scene(sc)
    ref_b.forward()
    need = ref_b.status().pairs_needed
    assert need > 100
    b = device_scene(sc, pair_capacity=64)
    b.forward(check_overflow=False)
    st = b.status()
    assert st.overflow == 1 and st.pairs_needed == need
    b.forward()  # replans and reruns
    assert b.capacity >= need
    o1, o2 = outputs_numpy(ref_b, 0), outputs_numpy(b, 0)
    for k in o1:
        assert np.array_equal(o1[k], o2[k]), k


def test_device_error_word_is_reported_and_raises():
    """A single-pass scan that gives up its bounded wait sets the status
    error word: read_status reports it, the binding raises instead of
    returning invalid outputs, and the next forward starts clean.  (The word
    is planted from the host after a normal forward.)"""
    from paper_2501_01677_amd.raster import DeviceError
    sc = scenes.small_scene(91, n=100, width=40, height=32, sh_degree=1)
    b = device_scene(sc, RenderConfig(tile=16))
    b.forward()
    st = b.status()
    assert st.error == 0 and st.overflow == 0
    words = b.view("status", torch.int32, 16)
    words[9] = 1
    assert b.status().error == 1
    with pytest.raises(DeviceError):
        b.check_status()
    with pytest.raises(DeviceError):
        b.fit_capacity()
    b.forward()
    assert b.status().error == 0

