"""Benchmark of the masked differentiable rasterizer on one MI355X.

Headline: masked forward+backward throughput (Mpixels/s of building-mask
pixels) on the 1M-Gaussian, 1920x1080, SH-degree-3 workload with a ~40%
rectangle-union mask.  One step = the whole hot path over that batch:
tile-mask reduce, projection, depth sort, binning, tile sort, compositing
with the depth epilogue, backward compositing and backward projection,
driven by a fixed upstream gradient (N(0,1) on masked pixels).  Inputs are
resident in HBM before the timed region.

Also reported: per-stage times (HIP events on the launch stream, recorded
inside the timed steps), the roofline of the dominant kernel, the FP64
oracle timed on a bounded pixel sample on the host cores, and (unless
--no-batched) the batched-versus-per-region speedup on the 16-sub-region x
4-view workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3  # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
# the same without packed FP32 (this build disables packed FP32 code generation)
FP32_SINGLE_ISSUE_TFLOPS = 78.6

# Algorithmic FP32 operations per blended (pixel, Gaussian) pair, counted
# from the arithmetic of the method (see the kernel docs):
#  forward: alpha (14) + transmittance update and 7-channel blend (18)
#  backward: alpha (14) + transmittance recovery (4) + dL/dalpha and the
#            7-channel feature gradients and suffix sums (58) + conic, mean
#            and opacity gradients (22)
FLOPS_PER_BLEND_FWD = 32
FLOPS_PER_BLEND_BWD = 98


class HipEvents:
    """hipEvent_t handles created through the HIP runtime (timing only)."""

    def __init__(self, n):
        self.hip = C.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [C.c_void_p]
        self.hip.hipEventDestroy.argtypes = [C.c_void_p]
        self.ev = []
        for _ in range(n):
            e = C.c_void_p()
            rc = self.hip.hipEventCreate(C.byref(e))
            if rc != 0:
                raise RuntimeError(f"hipEventCreate failed ({rc})")
            self.ev.append(e.value)

    def elapsed_ms(self, a, b):
        self.hip.hipEventSynchronize(C.c_void_p(self.ev[b]))
        out = C.c_float()
        rc = self.hip.hipEventElapsedTime(C.byref(out), C.c_void_p(self.ev[a]), C.c_void_p(self.ev[b]))
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return out.value

    def close(self):
        for e in self.ev:
            self.hip.hipEventDestroy(C.c_void_p(e))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_batch(scene, cfg, torch, want_grads=True):
    from paper_2501_01677_amd.raster import Batch, gaussians_to_device
    sets = [gaussians_to_device(s) for s in scene.sets]
    renders = []
    for rd in scene.renders:
        m = None if rd.mask is None else torch.from_numpy(np.ascontiguousarray(rd.mask)).cuda()
        renders.append(dict(set=rd.set_index, camera=rd.camera, mask=m))
    return Batch(sets, renders, cfg, want_grads=want_grads)


def fill_gouts(batch, scene, seed, torch):
    import scenes
    for r, rd in enumerate(scene.renders):
        g = scenes.grad_outputs(seed + r, rd, scale={"depth": 0.05})
        for k, v in g.items():
            batch.gout[r][k].copy_(torch.from_numpy(v).reshape(batch.gout[r][k].shape))


def timed_steps(batch, steps, warmup, torch, events=True):
    """Runs warmup + timed forward/backward steps; returns wall ms/step and
    the mean per-stage times (ms) over the timed steps."""
    from paper_2501_01677_amd import _abi as A
    batch.forward()            # replans the pair capacity if needed
    batch.fit_capacity(1.1)
    for _ in range(warmup):
        batch.forward(check_overflow=False)
        batch.backward()
    torch.cuda.synchronize()
    ev = HipEvents(2 * A.NUM_STAGES * steps) if events else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        e = None if ev is None else ev.ev[2 * A.NUM_STAGES * k:2 * A.NUM_STAGES * (k + 1)]
        batch.forward(check_overflow=False, events=e)
        batch.backward(events=e)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    st = batch.status()
    if st.overflow:
        raise RuntimeError("pair capacity overflow inside the timed region")
    stage = {}
    if ev is not None:
        per_step = np.zeros((steps, A.NUM_STAGES))
        for s, name in enumerate(A.STAGES):
            for k in range(steps):
                base = 2 * A.NUM_STAGES * k
                per_step[k, s] = ev.elapsed_ms(base + 2 * s, base + 2 * s + 1)
            stage[name] = float(per_step[:, s].mean())
        ev.close()
        # forward = stages 0-5, backward = 6-7 (the order of pgsag_stage)
        fwd, bwd = per_step[:, :6].sum(1), per_step[:, 6:].sum(1)
        tot = fwd + bwd
        q = lambda x: {"p10": round(float(np.percentile(x, 10)), 4), "p50": round(float(np.median(x)), 4),
                       "p90": round(float(np.percentile(x, 90)), 4)}
        stage["_summary"] = {"forward_ms": q(fwd), "backward_ms": q(bwd), "step_kernels_ms": q(tot)}
    return wall, stage


def roofline(stage, batch, scene, torch, tile):
    """Roofline entry of the dominant stage."""
    dom = max(stage, key=stage.get)
    traffic = measured_traffic(dom, tile)
    t = stage[dom] * 1e-3
    blends = float(sum(int(o["n_contrib"].sum().item()) for o in batch.out))
    if dom in ("composite", "backward_composite"):
        per = FLOPS_PER_BLEND_FWD if dom == "composite" else FLOPS_PER_BLEND_BWD
        work = per * blends
        ach = work / t / 1e12
        return dom, dict(bound="alu", achieved=round(ach, 3), peak=FP32_VECTOR_PEAK_TFLOPS,
                         unit="TFLOP/s", frac=round(ach / FP32_VECTOR_PEAK_TFLOPS, 4), traffic=traffic,
                         kernel=dom, blends_per_launch=int(blends),
                         flops_per_blend=per, peak_single_issue=FP32_SINGLE_ISSUE_TFLOPS,
                         frac_single_issue=round(ach / FP32_SINGLE_ISSUE_TFLOPS, 4))
    nbytes = algorithmic_bytes(dom, batch, scene)
    ach = nbytes / t / 1e9
    return dom, dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                     frac=round(ach / HBM_PEAK_GBS, 4), traffic=traffic, kernel=dom)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hot_path_1080p_hbm_traffic.md")
KERNEL_SOURCES = {"backward_composite": ("paper_2501_01677_amd/csrc/composite.hip",
                                         "paper_2501_01677_amd/csrc/internal.h")}


def measured_traffic(kernel, tile):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    counter summary (copy-calibrated), or None when that summary does not
    cover this kernel source or launch shape."""
    import hashlib
    if kernel not in KERNEL_SOURCES or tile != 16 or not os.path.exists(TRAFFIC_PROFILE):
        return None
    sha = hashlib.sha256()
    for p in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, p), "rb") as f:
            sha.update(f.read())
    nbytes = src = None
    with open(TRAFFIC_PROFILE) as f:
        for ln in f:
            if "traffic_bytes_per_launch:" in ln:
                nbytes = int(ln.split("traffic_bytes_per_launch:")[1].split()[0])
            if ln.startswith("kernel_source_sha256:"):
                src = ln.split()[1]
    return nbytes if src == sha.hexdigest() else None


def algorithmic_bytes(stage, batch, scene):
    n = sum(s.n for s in scene.sets)
    P = sum(4 * (3 + 3 + 4 + 1 + 3 * (s.sh_degree + 1) ** 2) for s in scene.sets) / max(1, len(scene.sets))
    nrec = int(batch.info.n_records)
    if stage == "preprocess":
        return n * P + nrec * (52 + 12)
    if stage == "backward_preprocess":
        return n * P + nrec * 52 + n * P
    return float("nan")


def stage_bytes(batch, scene):
    """Algorithmic HBM bytes per launch of each HBM-bound stage: what the
    method itself must read and write (the sort at its floor of one read and
    one write per key), not what the kernels move."""
    st = batch.status()
    n = sum(s.n for s in scene.sets)
    nbytes_p = sum(s.n * 4 * (3 + 3 + 4 + 1 + 3 * (s.sh_degree + 1) ** 2) for s in scene.sets)
    nrec = int(batch.info.n_records)
    nvis = int(st.n_visible)
    K = int(st.pairs_needed)
    tiles = int(batch.info.n_tiles)
    px = int(batch.info.n_pixels)
    return {
        # mask read; per-tile counts and active-tile row prefixes written
        "tile_mask": px + 8 * tiles,
        # raw parameters read; 52-byte record and 12 bytes of binning info
        # (depth key, tile rect) written per (render, Gaussian)
        "preprocess": nbytes_p + nrec * (52 + 12),
        # counts and keys read; visible (key, record) pairs compacted, then
        # sorted (one read and one write of 8 bytes each)
        "depth_sort": nrec * 8 + nvis * (8 + 16),
        # counts scanned (read, offsets written), rect/count/offset read per
        # visible record; 8 bytes written per (tile, record) pair
        "emit": nvis * (4 + 4 + 16) + K * 8,
        # pairs sorted by tile (one read and one write of 8 bytes), ranges
        # (tile ids read, [start, end) written)
        "tile_sort": K * (16 + 4) + tiles * 8,
        # raw parameters read, 52-byte 2D-gradient slot read, gradients written
        "backward_preprocess": 2 * nbytes_p + nrec * 52,
    }


def hbm_kernels(stage, batch, scene):
    """Per HBM-bound stage: algorithmic bytes, achieved GB/s over its event
    time, fraction of the 8 TB/s peak."""
    out = {}
    for k, b in stage_bytes(batch, scene).items():
        if k not in stage or stage[k] <= 0:
            continue
        gbs = b / (stage[k] * 1e-3) / 1e9
        out[k] = {"bytes": int(b), "ms": round(stage[k], 4), "gb_s": round(gbs, 1),
                  "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def step_roofline(stage, batch, scene, step_ms):
    """Whole-step roofline fraction: sum over stages of max(bytes / HBM
    peak, FP32 operations / FP32 peak), divided by the measured step time.
    The compositing stages count the method's operations per blended pair;
    the HBM-bound stages their algorithmic bytes."""
    blends = float(sum(int(o["n_contrib"].sum().item()) for o in batch.out))
    bound = {k: b / (HBM_PEAK_GBS * 1e9) for k, b in stage_bytes(batch, scene).items()}
    flops = {"composite": FLOPS_PER_BLEND_FWD * blends, "backward_composite": FLOPS_PER_BLEND_BWD * blends}
    t_pub = sum(bound.values()) + sum(f / (FP32_VECTOR_PEAK_TFLOPS * 1e12) for f in flops.values())
    t_single = sum(bound.values()) + sum(f / (FP32_SINGLE_ISSUE_TFLOPS * 1e12) for f in flops.values())
    t = step_ms * 1e-3
    return {"frac": round(t_pub / t, 4), "frac_single_issue": round(t_single / t, 4),
            "floor_ms": round(t_pub * 1e3, 4), "floor_ms_single_issue": round(t_single * 1e3, 4),
            "hbm_floor_ms": round(sum(bound.values()) * 1e3, 4),
            "note": "sum over stages of max(algorithmic bytes / 8 TB/s, method FP32 operations / peak) "
                    "over the measured step; peaks 157.3 TFLOP/s published and 78.6 single-issue"}


def compositing_work(batch, torch, tile):
    """Evaluated list entries against blended pairs, from the per-(tile,
    wave) work counters the compositing kernels write: every entry a wave
    evaluates costs all 64 of its lanes, so E/C = 64 x entries / blended
    pairs is the lane-slots spent per blended (pixel, Gaussian) pair, the
    lever the per-block culling works on."""
    wpt = (tile // 8) ** 2
    n = int(batch.info.n_tiles)
    w = batch.view("work", torch.int32, n * wpt, 3).cpu().numpy().astype(np.int64)
    cnt = batch.view("tile_count", torch.int32, n).cpu().numpy()
    active = np.repeat(cnt > 0, wpt)
    blends = float(sum(int(o["n_contrib"].sum().item()) for o in batch.out))
    fwd, bwd, act = w[:, 0].sum(), w[:, 1].sum(), w[:, 2].sum()
    waves = int(active.sum())
    return {"waves": waves, "blended_pairs": int(blends),
            "fwd_entries": int(fwd), "fwd_E_per_lane": round(fwd / max(waves, 1), 1),
            "fwd_E_over_C": round(64 * fwd / max(blends, 1), 3),
            "bwd_entries": int(bwd), "bwd_E_per_lane": round(bwd / max(waves, 1), 1),
            "bwd_E_over_C": round(64 * bwd / max(blends, 1), 3),
            "bwd_entries_contributing": int(act), "bwd_contributing_share": round(act / max(bwd, 1), 4),
            "note": "E = list entries a wave evaluates (each for all 64 lanes) per wave of a tile holding masked "
                    "pixels; E/C = 64 E summed over waves / blended pairs"}


def tile_lists(batch, torch):
    """Per-tile list lengths over tiles holding masked pixels: the workload
    each compositing workgroup walks, whose spread is the thread-waiting
    cost the balance-load term targets."""
    n = int(batch.info.n_tiles)
    rg = batch.view("ranges", torch.int32, n, 2).cpu().numpy().astype(np.int64)
    cnt = batch.view("tile_count", torch.int32, n).cpu().numpy()
    ln = (rg[:, 1] - rg[:, 0])[cnt > 0]
    if ln.size == 0:
        return None
    return {"active_tiles": int(ln.size), "mean": round(float(ln.mean()), 1),
            "p50": int(np.median(ln)), "p99": int(np.percentile(ln, 99)), "max": int(ln.max()),
            "max_over_mean": round(float(ln.max() / max(ln.mean(), 1e-9)), 2)}


def cpu_baseline(scene, sample=4096, seed=7):
    """The FP64 oracle (as it is) on a fixed sample of masked pixels:
    forward at the sample plus the gradient of a loss on the sample."""
    import torch
    import scenes
    from oracle import OracleConfig
    from oracle import composite as oc
    torch.set_num_threads(os.cpu_count() or 1)
    cfg = OracleConfig()
    rd = scene.renders[0]
    gs = scene.sets[rd.set_index]
    pix = scenes.sample_pixels(seed, rd, sample)
    g = scenes.grad_outputs(seed + 1000, rd, scale={"depth": 0.05})
    sel = np.zeros((rd.camera.height, rd.camera.width), bool)
    sel[pix[:, 0], pix[:, 1]] = True
    g = {k: (v * sel).astype(np.float32) for k, v in g.items()}
    t0 = time.perf_counter()
    oc.render(gs, rd.camera, rd.mask, cfg, pixels=pix)
    oc.render_grad(gs, rd.camera, rd.mask, cfg, g, pixels=pix)
    dt = time.perf_counter() - t0
    return dict(value=round(len(pix) / dt / 1e6, 6), unit="Mpixels/s", cores=torch.get_num_threads(),
                kind="oracle",
                sample=f"{len(pix)} masked pixels (seed {seed}) of the same 1M-Gaussian 1080p workload, "
                       f"FP64 forward + gradient, full per-Gaussian preprocessing included; {dt:.1f} s")


def cpu_baseline_config1(seed=7, brute_sample=8192):
    """The FP64 oracle on config 1 (10k Gaussians, 256x256, full frame),
    forward plus gradient, in its two modes: culled (each pixel's Gaussians
    from the exact-support grid) over the whole frame, and brute force (every
    Gaussian at every pixel) on a fixed sample of pixels."""
    import torch
    import scenes
    from oracle import OracleConfig
    from oracle import composite as oc
    torch.set_num_threads(os.cpu_count() or 1)
    cfg = OracleConfig()
    sc = scenes.config1()
    rd = sc.renders[0]
    gs = sc.sets[rd.set_index]
    H, W = rd.camera.height, rd.camera.width
    g = scenes.grad_outputs(seed + 1000, rd, scale={"depth": 0.05})
    out = {}
    rng = np.random.default_rng(seed)
    for mode, npx in (("culled", H * W), ("brute", brute_sample)):
        idx = np.arange(H * W) if npx == H * W else np.sort(rng.choice(H * W, npx, replace=False))
        pix = np.stack([idx // W, idx % W], 1)
        sel = np.zeros((H, W), bool)
        sel[pix[:, 0], pix[:, 1]] = True
        gg = {k: (v * sel).astype(np.float32) for k, v in g.items()}
        t0 = time.perf_counter()
        oc.render(gs, rd.camera, rd.mask, cfg, pixels=pix, mode=mode)
        oc.render_grad(gs, rd.camera, rd.mask, cfg, gg, pixels=pix, mode=mode)
        dt = time.perf_counter() - t0
        out[mode] = dict(value=round(npx / dt / 1e6, 6), unit="Mpixels/s", pixels=int(npx), seconds=round(dt, 2))
    out.update(cores=torch.get_num_threads(), kind="oracle",
               workload="config 1: 10k Gaussians SH0, 256x256 full frame, FP64 forward + gradient; brute force on "
                        f"{brute_sample} sampled pixels (seed {seed})")
    return out


def _graph_time(bb, torch, steps):
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bb.forward(check_overflow=False)
            bb.backward()
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    if bb.status().overflow:
        raise RuntimeError("overflow in the batched graph")
    del g
    return dt


def _replay_time(fn, torch, steps):
    """Captures fn() once into a HIP graph and times `steps` replays (s)."""
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    del g
    return dt


def ground_truth(scene, torch, tile=16):
    """Training targets: renders of the generating scene (rgb planes)."""
    from paper_2501_01677_amd.raster import RenderConfig
    b = build_batch(scene, RenderConfig(tile=tile), torch, want_grads=False)
    b.forward()
    gt = [o["rgb"].clone() for o in b.out]
    del b.workspace
    del b
    torch.cuda.empty_cache()
    return gt


def with_loss_time(batch, gt, torch, steps):
    """Forward + loss (masked L1 + 0.01 boundary-aware normal L1) + backward
    of the 1080p workload, one captured graph; returns ms per step."""
    from paper_2501_01677_amd.raster import LossConfig
    out = torch.zeros((len(batch.renders), 4), dtype=torch.float32, device="cuda")
    lc = LossConfig()

    def step():
        batch.forward(check_overflow=False)
        batch.loss(gt, lc, out=out)
        batch.backward()

    return _replay_time(step, torch, steps) * 1e3, out


def train_step_bench(torch, steps):
    """The 10M-Gaussian, 2 x 5472x3648 training step (forward, loss with the
    balance-load term at lambda 0.41, backward, fused Adam), one captured
    graph, starting from the generating set plus noise."""
    import scenes
    from paper_2501_01677_amd.raster import LossConfig, RenderConfig, Trainer, gaussians_to_device
    sc = scenes.config5()
    gt = ground_truth(sc, torch)
    start = [gaussians_to_device(scenes.perturbed(55, s)) for s in sc.sets]
    renders = [dict(set=rd.set_index, camera=rd.camera, mask=torch.from_numpy(np.ascontiguousarray(rd.mask)).cuda())
               for rd in sc.renders]
    # launch configuration (plain or persistent, backward reduction) picked
    # by timing the captured fwd+bwd step on this batch shape
    from paper_2501_01677_amd.autotune import Autotuner
    tb = build_batch(sc, RenderConfig(tile=16), torch)
    fill_gouts(tb, sc, 5000, torch)
    gouts = [{k: v.clone() for k, v in g.items()} for g in tb.gout]
    cands = tuple(RenderConfig(tile=16, persistent=p, queue_chunk=8 if p else 1, workgroups_per_cu=8 if p else 4,
                               bwd_reduce=r) for p in (False, True) for r in (0, 1))
    tuner = Autotuner(candidates=cands, steps=2)
    cfg, times = tuner.best(tb.sets, tb.renders, gouts)
    del tb.workspace
    del tb, gouts
    torch.cuda.empty_cache()
    t = Trainer(start, renders, gt, cfg, LossConfig(lambda_load=0.41), lr=1e-3)
    del start
    t.fit(1.2)
    for _ in range(2):
        t.step()
    torch.cuda.synchronize()
    t.capture()
    t.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    if t.overflowed():
        raise RuntimeError("pair capacity overflow in the training step")
    masked = sum(int(rd.mask.sum()) for rd in sc.renders)
    loss = t.loss_out.cpu().numpy().tolist()
    res = dict(workload="10M Gaussians SH3, 2 views 5472x3648, box-silhouette masks; forward + loss "
                        "(masked L1 + 0.01 boundary-aware normal L1, 0.41 balance-load) + backward + Adam",
               ms_per_step=round(dt * 1e3, 3), masked_pixels=masked,
               config={"tile": cfg.tile, "persistent": cfg.persistent, "queue_chunk": cfg.queue_chunk,
                       "workgroups_per_cu": cfg.workgroups_per_cu, "bwd_reduce": cfg.bwd_reduce},
               autotune_ms={k: round(v * 1e3, 3) for k, v in times.items()},
               mpix_s=round(masked / dt / 1e6, 1), params=int(t.P.numel()),
               pairs=int(t.batch.status().pairs_needed), loss=[[round(x, 6) for x in r] for r in loss])
    del t
    torch.cuda.empty_cache()
    return res


def batched_speedup(torch, steps=5, scale=1.0):
    """Batched graph-captured step (autotuned launch configuration) vs the
    per-sub-region launch loop on 16 sub-regions x 4 views at 1600x1200 (one
    Batch per sub-region, 16x16 tiles and the tuned backward reduction,
    launched one after another, no graph)."""
    import scenes
    from paper_2501_01677_amd.raster import RenderConfig
    sc = scenes.config4(scale=scale)
    masked = sum(int(rd.mask.sum()) for rd in sc.renders)
    # one batch for all sub-regions and views; the launch configuration is
    # picked by the autotuner (captured fwd+bwd step timed per candidate)
    from paper_2501_01677_amd.autotune import Autotuner
    bb = build_batch(sc, RenderConfig(tile=16), torch)
    fill_gouts(bb, sc, 4000, torch)
    gouts = [{k: v.clone() for k, v in g.items()} for g in bb.gout]
    tuner = Autotuner(steps=steps)
    cfg, times = tuner.best(bb.sets, bb.renders, gouts)
    del bb.workspace
    del bb, gouts
    torch.cuda.empty_cache()
    # the loop: one Batch per sub-region with the same backward reduction
    loops = []
    for k, s in enumerate(sc.sets):
        sub = scenes.Scene([s], [scenes.Render(0, rd.camera, rd.mask) for rd in sc.renders
                                 if rd.set_index == k])
        b = build_batch(sub, RenderConfig(tile=16, bwd_reduce=cfg.bwd_reduce), torch)
        fill_gouts(b, sub, 4000 + k, torch)
        b.forward()
        b.fit_capacity(1.1)
        loops.append(b)
    for b in loops:
        b.forward(check_overflow=False)
        b.backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for b in loops:
            b.forward(check_overflow=False)
            b.backward()
    torch.cuda.synchronize()
    t_loop = (time.perf_counter() - t0) / steps

    # the same loop captured once into a graph: batching measured apart
    # from graph capture
    def loop_step():
        for b in loops:
            b.forward(check_overflow=False)
            b.backward()

    t_loop_graph = _replay_time(loop_step, torch, steps)
    if any(b.status().overflow for b in loops):
        raise RuntimeError("overflow in the captured loop")
    for b in loops:
        del b.workspace
    del loops
    torch.cuda.empty_cache()
    out = dict(workload="16 sub-regions x 4 views, 1600x1200, %d Gaussians" % sum(s.n for s in sc.sets),
               loop_ms=round(t_loop * 1e3, 3), loop_graph_ms=round(t_loop_graph * 1e3, 3))
    out["autotune_ms"] = {k: round(v * 1e3, 3) for k, v in times.items()}
    bb = build_batch(sc, cfg, torch)
    fill_gouts(bb, sc, 4000, torch)
    _, stage = timed_steps(bb, 2, 1, torch)
    stage.pop("_summary", None)
    best = _graph_time(bb, torch, steps)
    out["graph_ms"] = round(best * 1e3, 3)
    out["graph_config"] = {"tile": cfg.tile, "persistent": cfg.persistent, "queue_chunk": cfg.queue_chunk,
                           "workgroups_per_cu": cfg.workgroups_per_cu, "bwd_reduce": cfg.bwd_reduce}
    out["graph_stages_ms"] = {k: round(v, 3) for k, v in stage.items()}
    out["tile_lists"] = tile_lists(bb, torch)
    out["compositing_work"] = compositing_work(bb, torch, cfg.tile)
    out["hbm_kernels"] = hbm_kernels(stage, bb, sc)
    out["step_roofline"] = step_roofline(stage, bb, sc, best * 1e3)
    del bb.workspace
    del bb
    torch.cuda.empty_cache()
    out["speedup"] = round(t_loop / best, 3)
    out["speedup_vs_loop_graph"] = round(t_loop_graph / best, 3)
    out["batched_mpix_s"] = round(masked / best / 1e6, 1)
    return out


def _event_ms(fn, torch, reps=3):
    """Mean time (ms) of fn() on torch's current stream over reps runs after
    one warm-up run (HIP events around the calls)."""
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def survey_bench(torch):
    """The steps around the rasterizer on their full stand-in workloads: the
    voting filter (2M sparse points x 64 views at 5472x3648), DBSCAN over
    its reliable points and the views of every group, and the mean fusion
    and TSDF integration of an 8-view 1600x1200 depth stack (3 building
    groups and the background block per view) into a 0.5 m volume."""
    from scenes import survey as sv
    from paper_2501_01677_amd import survey as gs
    out = {}
    s = sv.vote_full()
    pts = torch.from_numpy(s.points).cuda()
    masks = [torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in s.masks]
    views = gs.pack_views(s.cameras, masks)
    M, V = pts.shape[1], len(masks)
    res = {}

    def vote():
        res["v"] = gs.vote(pts, s.cameras, masks, 3, views=views)

    t = _event_ms(vote, torch)
    votes, us, flags = res["v"]
    sightings = int(votes.to(torch.int64).sum() + us.to(torch.int64).sum())
    nbytes = 17 * M + sightings   # points read, votes/US/flags written, one mask byte per sighting
    out["vote"] = {"workload": f"{M} points x {V} views at {s.cameras[0].width}x{s.cameras[0].height}",
                   "ms": round(t, 4), "point_views_per_s": round(M * V / (t * 1e-3), 1),
                   "sightings": sightings, "bytes": nbytes,
                   "gb_s": round(nbytes / (t * 1e-3) / 1e9, 1),
                   "frac": round(nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "note": "bound by the mask gathers (a 64-byte line per sighting), not by the algorithmic bytes"}
    ws = {}

    def dbscan():
        ws["r"] = gs.dbscan(pts, 3.0, 10, flags=flags, workspace=ws.get("w"))
        ws["w"] = ws["r"]["workspace"]

    t = _event_ms(dbscan, torch)
    k = int(ws["r"]["n_clusters"][0])
    part = int(((flags & 2) != 0).sum())
    out["dbscan"] = {"workload": f"{part} reliable points of {M}, eps 3 m, min 10", "ms": round(t, 4),
                     "clusters": k, "points_per_s": round(part / (t * 1e-3), 1)}
    cl = ws["r"]["cluster"]
    t = _event_ms(lambda: gs.group_views(pts, cl, k, s.cameras, masks, 200, views=views), torch)
    out["group_views"] = {"workload": f"{k} groups x {V} views", "ms": round(t, 4)}
    del pts, masks, views, res, ws, cl, votes, us, flags
    torch.cuda.empty_cache()

    ds = sv.depth_full()
    maps = [[torch.from_numpy(np.ascontiguousarray(d)).cuda() for d in per] for per in ds.depths]
    fused = [torch.empty_like(m[0]) for m in maps]

    def fuse():
        for j, m in enumerate(maps):
            gs.fuse_depth(m, out=fused[j], count=False)

    t = _event_ms(fuse, torch)
    H, W = maps[0][0].shape
    K = len(maps[0])
    nbytes = len(maps) * H * W * (4 * K + 4)
    out["fuse"] = {"workload": f"{len(maps)} views x {K} maps at {W}x{H}", "ms": round(t, 4), "bytes": nbytes,
                   "gb_s": round(nbytes / (t * 1e-3) / 1e9, 1),
                   "frac": round(nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    vol = ds.volume
    tv = {}
    hv = gs.pack_depth_views(ds.cameras, fused)

    def tsdf():
        tv["r"] = gs.tsdf_integrate(vol, ds.cameras, fused, tsdf=tv.get("t"), weight=tv.get("w"), views=hv)
        tv["t"], tv["w"] = tv["r"]

    t = _event_ms(tsdf, torch)
    nvox = int(np.prod(vol["dims"]))
    out["tsdf"] = {"workload": f"{vol['dims'][0]}x{vol['dims'][1]}x{vol['dims'][2]} voxels x {len(fused)} views",
                   "ms": round(t, 4), "voxel_views_per_s": round(nvox * len(fused) / (t * 1e-3), 1),
                   "bytes": 8 * nvox, "gb_s": round(8 * nvox / (t * 1e-3) / 1e9, 1),
                   "note": "bound by the per-(voxel, view) projection with correctly rounded divisions"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-scale", type=float, default=1.0)
    ap.add_argument("--no-train", action="store_true", help="skip the 10M-Gaussian training step")
    ap.add_argument("--no-survey", action="store_true", help="skip the voting / grouping / fusion steps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    import torch
    import scenes
    from paper_2501_01677_amd.raster import RenderConfig
    torch.cuda.set_device(0)
    log("[bench] generating the 1M-Gaussian 1080p workload")
    sc = scenes.config2()
    gt = ground_truth(sc, torch, args.tile)
    cfg = RenderConfig(tile=args.tile)
    batch = build_batch(sc, cfg, torch)
    fill_gouts(batch, sc, 2 + 1000, torch)
    log("[bench] timing forward+backward")
    ms_eager, stage = timed_steps(batch, args.steps, args.warmup, torch)
    # the production path replays the captured step (one graph launch)
    ms_graph = _graph_time(batch, torch, args.steps) * 1e3
    ms_wall = min(ms_eager, ms_graph)
    masked = int(sc.renders[0].mask.sum())
    value = masked / (ms_wall * 1e-3) / 1e6
    summary = stage.pop("_summary", None)
    lists = tile_lists(batch, torch)
    work = compositing_work(batch, torch, args.tile)
    dom, roof = roofline(stage, batch, sc, torch, args.tile)
    hbm = hbm_kernels(stage, batch, sc)
    step_roof = step_roofline(stage, batch, sc, ms_wall)
    log("[bench] forward+loss+backward")
    ms_loss, _ = with_loss_time(batch, gt, torch, args.steps)
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    line = {
        "metric": "masked fwd+bwd Mpixels/s (1M Gaussians, 1080p); batched vs per-region speedup",
        "value": round(value, 2),
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_wall, 4),
        "ms_per_step_graph": round(ms_graph, 4),
        "ms_per_step_eager": round(ms_eager, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1M Gaussians SH3, 1920x1080, 40% rectangle-union building mask, "
                               "fwd+bwd with fixed dL/dout",
                   "masked_pixels": masked, "tile": args.tile, "pairs": int(batch.status().pairs_needed)},
        "stages_ms": {k: round(v, 4) for k, v in stage.items()},
        "step_event_ms": summary,
        "tile_lists": lists,
        "compositing_work": work,
        "device": {"name": torch.cuda.get_device_name(0), "hip": torch.version.hip, "torch": torch.__version__},
        "with_loss": {"ms_per_step": round(ms_loss, 4), "mpix_s": round(masked / (ms_loss * 1e-3) / 1e6, 2),
                      "note": "same step with the loss kernels in the graph (ground truth: the render of the "
                              "generating scene)"},
        "roofline": roof,
        "hbm_kernels": hbm,
        "step_roofline": step_roof,
    }
    del batch
    torch.cuda.empty_cache()
    if not args.no_batched:
        log("[bench] batched vs per-region loop")
        try:
            line["batched"] = batched_speedup(torch, steps=3, scale=args.batched_scale)
        except Exception as e:  # report, do not hide the headline
            line["batched"] = {"error": repr(e)}
    if not args.no_train:
        log("[bench] 10M-Gaussian training step")
        try:
            line["train_step"] = train_step_bench(torch, max(3, args.steps // 4))
        except Exception as e:  # report, do not hide the headline
            line["train_step"] = {"error": repr(e)}
    if not args.no_survey:
        log("[bench] voting filter, grouping, depth fusion and TSDF")
        try:
            line["survey"] = survey_bench(torch)
        except Exception as e:  # report, do not hide the headline
            line["survey"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(sc)
        log("[bench] CPU oracle on config 1 (culled and brute force)")
        line["cpu_baseline_config1"] = cpu_baseline_config1()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
