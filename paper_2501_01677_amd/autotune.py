"""Launch-configuration autotuner for batched renders.

The rendered values do not depend on the launch configuration (every pixel
blends the same records in the same order whatever the tile size, queue
chunk or workgroup count; the two backward reductions form the same sums in
a different order), only the speed does.  For a batch shape the tuner times
the captured forward + backward step of each candidate configuration -- tile
size T in {8, 16, 32}, plain or persistent launch, queue chunk, persistent
workgroups per CU and backward reduction -- and keeps the fastest.  Results are cached
per shape bucket: (number of renders, log2 of the masked pixels, log2 of the
Gaussians, SH degree), optionally persisted to a JSON file.
"""
import json
import math
import os
import time
from dataclasses import asdict

import torch

from .raster import Batch, RenderConfig

DEFAULT_CANDIDATES = tuple(
    RenderConfig(tile=t, persistent=p, queue_chunk=q, workgroups_per_cu=w, bwd_reduce=r)
    for (t, p, q, w) in ((16, False, 1, 4), (8, False, 1, 4), (32, False, 1, 4),
                         (16, True, 4, 8), (16, True, 8, 8), (16, True, 16, 8))
    for r in (0, 1))


def config_name(cfg):
    """Short label of a launch configuration, e.g. T16-p8x8-r1."""
    return (f"T{cfg.tile}" + (f"-p{cfg.queue_chunk}x{cfg.workgroups_per_cu}" if cfg.persistent else "")
            + f"-r{cfg.bwd_reduce}")


def shape_key(sets, renders):
    """Shape bucket of a batch (see the module docstring)."""
    masked = 0
    for rd in renders:
        m = rd.get("mask")
        cam = rd["camera"]
        masked += int(m.sum().item()) if m is not None else int(cam.width) * int(cam.height)
    n = sum(int(s["means"].shape[1]) for s in sets)
    deg = max(int(s["sh_degree"]) for s in sets)
    return f"r{len(renders)}-px{int(math.log2(max(masked, 1)))}-n{int(math.log2(max(n, 1)))}-sh{deg}"


def _step_time(batch, steps):
    """Seconds per captured forward + backward step (after a warm-up that
    sizes the pair capacity)."""
    batch.forward()
    batch.fit_capacity(1.1)
    batch.forward(check_overflow=False)
    batch.backward()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            batch.forward(check_overflow=False)
            batch.backward()
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    if batch.status().overflow:
        raise RuntimeError("pair capacity overflow while tuning")
    del g
    return dt


class Autotuner:
    def __init__(self, cache_path=None, candidates=DEFAULT_CANDIDATES, steps=3):
        self.cache_path = cache_path
        self.candidates = tuple(candidates)
        self.steps = steps
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def best(self, sets, renders, gouts=None):
        """Fastest configuration for this batch shape (tuned on first use)
        and the measured seconds per step of every candidate."""
        key = shape_key(sets, renders)
        if key in self.cache:
            e = self.cache[key]
            return RenderConfig(**{k: (tuple(v) if k == "bg" else v) for k, v in e["config"].items()}), e["times"]
        times = {}
        best_cfg, best_t = None, math.inf
        for cfg in self.candidates:
            b = Batch(sets, renders, cfg)
            if gouts is not None:
                for r, g in enumerate(gouts):
                    for k, v in g.items():
                        b.gout[r][k].copy_(v.reshape(b.gout[r][k].shape))
            t = _step_time(b, self.steps)
            times[config_name(cfg)] = t
            if t < best_t:
                best_cfg, best_t = cfg, t
            del b
            torch.cuda.empty_cache()
        self.cache[key] = {"config": asdict(best_cfg), "times": times}
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1)
        return best_cfg, times
