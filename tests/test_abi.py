"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, the ctypes mirror matches the C struct layouts, and the
host-only planning calls validate their arguments."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2501_01677_amd import _abi as A
from paper_2501_01677_amd.raster import RenderConfig, make_camera
import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pgsag.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(pgsag_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = A.lib()
    decl = declared_functions()
    assert len(decl) >= 12
    for name in decl:
        assert hasattr(L, name), name
    assert set(decl) == set(A.SYMBOLS)
    assert L.pgsag_version() == A.ABI_VERSION


STRUCTS = {
    "pgsag_camera": (A.Camera, ["width", "fx", "R", "t"]),
    "pgsag_gaussians": (A.Gaussians, ["n", "sh_degree", "means", "sh"]),
    "pgsag_grads": (A.Grads, ["means", "sh"]),
    "pgsag_outputs": (A.Outputs, ["rgb", "alpha", "n_contrib"]),
    "pgsag_grad_outputs": (A.GradOutputs, ["rgb", "alpha", "count"]),
    "pgsag_render": (A.Render, ["set", "cam", "mask", "out", "gout"]),
    "pgsag_config": (A.Config, ["tile", "alpha_min", "logit_min", "depth_guard", "bg", "bwd_reduce",
                                         "deterministic"]),
    "pgsag_adam_config": (A.AdamConfig, ["lr", "step_state", "m_offset", "v_offset", "write_grads"]),
    "pgsag_loss_config": (A.LossConfig, ["lambda_rgb", "lambda_load", "normal_norm", "normal_eps", "load_term",
                                         "reserved"]),
    "pgsag_plan_info": (A.PlanInfo, ["workspace_bytes", "pair_capacity", "tile_bits"]),
    "pgsag_layout": (A.Layout, ["status", "records", "grad2d", "work", "end"]),
    "pgsag_status": (A.Status, ["pairs_needed", "overflow", "n_visible", "error", "reserved"]),
    "pgsag_vote_view": (A.VoteView, ["cam", "mask"]),
    "pgsag_volume": (A.Volume, ["origin", "voxel", "nx", "nz", "trunc"]),
    "pgsag_depth_view": (A.DepthView, ["cam", "depth"]),
}


def test_ctypes_layouts_match_the_header():
    lines = ['#include "pgsag.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void) {"]
    for sname, (_, fields) in STRUCTS.items():
        lines.append(f'  printf("{sname} %zu\\n", sizeof({sname}));')
        for f in fields:
            lines.append(f'  printf("{sname}.{f} %zu\\n", offsetof({sname}, {f}));')
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(src, "w").write("\n".join(lines))
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), src, "-o", exe])
        out = subprocess.check_output([exe], text=True)
    got = dict(line.split() for line in out.strip().splitlines())
    for sname, (cls, fields) in STRUCTS.items():
        assert int(got[sname]) == C.sizeof(cls), sname
        for f in fields:
            assert int(got[f"{sname}.{f}"]) == getattr(cls, f).offset, (sname, f)


def _c_batch(n=100, W=70, H=50, tile=16, sets=1, renders=1):
    gs = (A.Gaussians * sets)()
    for i in range(sets):
        gs[i].n = n
        gs[i].sh_degree = 1
        for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
            setattr(gs[i], k, C.c_void_p(0x1000))
    rs = (A.Render * renders)()
    for i in range(renders):
        rs[i].set = i % sets
        rs[i].cam = make_camera(scenes.pinhole(W, H, 60.0, 60.0))
    cfg = RenderConfig(tile=tile).to_c()
    return cfg, gs, rs


def test_plan_sizes_and_validation():
    L = A.lib()
    cfg, gs, rs = _c_batch()
    info = A.PlanInfo()
    assert L.pgsag_plan(C.byref(cfg), gs, 1, rs, 1, 5000, C.byref(info)) == A.OK
    assert info.n_tiles == 5 * 4 and info.n_pixels == 70 * 50 and info.n_records == 100
    assert info.tile_bits == 5 and info.workspace_bytes > 100 * 64
    # invalid tile size
    cfg.tile = 12
    assert L.pgsag_plan(C.byref(cfg), gs, 1, rs, 1, 5000, C.byref(info)) == A.INVALID_ARGUMENT
    assert b"tile" in L.pgsag_last_error()
    cfg.tile = 16
    # unknown backward reduction
    cfg.bwd_reduce = 2
    assert L.pgsag_plan(C.byref(cfg), gs, 1, rs, 1, 5000, C.byref(info)) == A.INVALID_ARGUMENT
    assert b"bwd_reduce" in L.pgsag_last_error()
    cfg.bwd_reduce = 1
    assert L.pgsag_plan(C.byref(cfg), gs, 1, rs, 1, 5000, C.byref(info)) == A.OK
    cfg.bwd_reduce = 0
    # bad SH degree, bad set index, zero capacity, bad image
    gs[0].sh_degree = 4
    assert L.pgsag_plan(C.byref(cfg), gs, 1, rs, 1, 5000, C.byref(info)) == A.INVALID_ARGUMENT
    gs[0].sh_degree = 1
    rs[0].set = 3
    assert L.pgsag_plan(C.byref(cfg), gs, 1, rs, 1, 5000, C.byref(info)) == A.INVALID_ARGUMENT
    rs[0].set = 0
    assert L.pgsag_plan(C.byref(cfg), gs, 1, rs, 1, 0, C.byref(info)) == A.INVALID_ARGUMENT
    rs[0].cam.width = 0
    assert L.pgsag_plan(C.byref(cfg), gs, 1, rs, 1, 5000, C.byref(info)) == A.INVALID_ARGUMENT


def test_pack_and_layout_on_host():
    L = A.lib()
    cfg, gs, rs = _c_batch(n=1000, sets=2, renders=5)
    info = A.PlanInfo()
    assert L.pgsag_plan(C.byref(cfg), gs, 2, rs, 5, 1 << 20, C.byref(info)) == A.OK
    small = (C.c_uint8 * 16)()
    assert L.pgsag_pack(C.byref(cfg), gs, None, 2, rs, 5, 1 << 20, small, 16) == A.WORKSPACE_TOO_SMALL
    buf = (C.c_uint8 * info.desc_bytes)()
    assert L.pgsag_pack(C.byref(cfg), gs, None, 2, rs, 5, 1 << 20, buf, info.desc_bytes) == A.OK
    lay = A.Layout()
    assert L.pgsag_layout_of(buf, C.byref(lay)) == A.OK
    offs = [getattr(lay, f) for f, _ in A.Layout._fields_]
    assert all(o % 256 == 0 for o in offs)
    assert lay.end == info.workspace_bytes
    assert lay.records < lay.grad2d < lay.end
    # a depth gradient without the normal/dist outputs is rejected
    rs[0].gout.depth = C.c_void_p(0x2000)
    assert L.pgsag_pack(C.byref(cfg), gs, None, 2, rs, 5, 1 << 20, buf, info.desc_bytes) == A.INVALID_ARGUMENT
    # garbage descriptors are rejected before any device work
    junk = (C.c_uint8 * 4096)()
    assert L.pgsag_layout_of(junk, C.byref(lay)) == A.INVALID_ARGUMENT
    assert L.pgsag_forward(junk, None, None, 0, None, None) == A.INVALID_ARGUMENT


def test_adam_rejects_bad_arguments_without_touching_memory():
    L = A.lib()
    assert L.pgsag_adam_step(None, None, None, None, -1, 1e-3, 0.9, 0.999, 1e-8, 1, None) == A.INVALID_ARGUMENT
    assert L.pgsag_adam_step(None, None, None, None, 10, 1e-3, 0.9, 0.999, 1e-8, 1, None) == A.INVALID_ARGUMENT
    p = C.c_void_p(0x1000)
    assert L.pgsag_adam_step(p, p, p, p, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == A.INVALID_ARGUMENT


def test_vote_validates_on_the_host_without_touching_memory():
    L = A.lib()
    views = (A.VoteView * 2)()
    for j in range(2):
        views[j].cam = make_camera(scenes.pinhole(64, 48, 50.0, 50.0))
    p = C.c_void_p(0x1000)
    ok_args = (views, p, 2, p, 10, 0.2, 2, p, p, p, None)
    bad = [
        (None, p, 2, p, 10, 0.2, 2, p, p, p, None),        # no host views
        (views, p, 0, p, 10, 0.2, 2, p, p, p, None),       # no view
        (views, p, 2, p, -1, 0.2, 2, p, p, p, None),       # n < 0
        (views, p, 2, None, 10, 0.2, 2, p, p, p, None),    # no points
        (views, p, 2, p, 10, 0.2, 2, p, p, None, None),    # no flags
        (views, p, 2, p, 10, 0.0, 2, p, p, p, None),       # z_near <= 0
        (views, p, 2, p, 10, 0.2, -1, p, p, p, None),      # tau < 0
    ]
    for args in bad:
        assert L.pgsag_vote(*args) == A.INVALID_ARGUMENT, args
    views[1].cam.width = 0
    assert L.pgsag_vote(*ok_args) == A.INVALID_ARGUMENT
    assert b"view 1" in L.pgsag_last_error()
    # nothing to do: returns before any launch
    views[1].cam.width = 64
    assert L.pgsag_vote(views, p, 2, None, 0, 0.2, 2, None, None, None, None) == A.OK


def test_static_scratch_dbscan_validates_on_the_host_before_any_device_call():
    """pgsag_dbscan_static rejects sizes beyond its scratch (and bad
    arguments) before it looks up the scratch or launches anything."""
    L = A.lib()
    p = C.c_void_p(0x1000)
    mx = 1 << 19
    hdr = open(HEADER).read()
    assert re.search(r"#define PGSAG_DBSCAN_STATIC_MAX_POINTS \(1 << 19\)", hdr)
    bad = [
        (p, mx + 1, None, 2, 3.0, 10, p, p, p, p, None),   # beyond the scratch
        (p, -1, None, 2, 3.0, 10, p, p, p, p, None),       # n < 0
        (p, 10, None, 2, 0.0, 10, p, p, p, p, None),       # eps <= 0
        (p, 10, None, 2, 3.0, 0, p, p, p, p, None),        # min_pts < 1
        (p, 10, None, 2, 3.0, 10, p, None, p, None, None),  # no n_clusters
        (None, 10, None, 2, 3.0, 10, p, p, p, p, None),    # no points
        (p, 10, None, 2, 3.0, 10, p, None, p, p, None),    # no labels
    ]
    for args in bad:
        assert L.pgsag_dbscan_static(*args) == A.INVALID_ARGUMENT, args
    L.pgsag_dbscan_static(p, mx + 1, None, 2, 3.0, 10, p, p, p, p, None)
    assert b"0..524288" in L.pgsag_last_error()


def test_autotune_shape_key_buckets():
    import torch
    from paper_2501_01677_amd.autotune import shape_key
    cam = type("Cam", (), dict(width=64, height=32))()
    sets = [dict(means=torch.zeros(3, 1000), sh_degree=2), dict(means=torch.zeros(3, 3000), sh_degree=1)]
    mask = torch.zeros(32, 64, dtype=torch.uint8)
    mask[:, :16] = 1
    renders = [dict(set=0, camera=cam, mask=mask), dict(set=1, camera=cam, mask=None)]
    # 512 + 2048 masked pixels, 4000 Gaussians, max SH degree 2
    assert shape_key(sets, renders) == "r2-px11-n11-sh2"


def test_default_loss_weights_are_the_papers():
    """The default boundary weight (Sec. 4.2, after Eq. 8) and normal-loss
    weight lambda_4 (Sec. 4.3, Eq. 10) of the C library, the binding and the
    oracle equal the constants the paper prints (tests/golden).  The
    balance-load weight lambda (Eq. 11) is off by default; training passes it."""
    import json
    from oracle import losses as ol
    from paper_2501_01677_amd.raster import LossConfig
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")
    k = json.load(open(path))
    lc = A.LossConfig()
    A.lib().pgsag_default_loss_config(C.byref(lc))
    for cfg in (lc, LossConfig(), ol.LossConfig()):
        assert np.float32(cfg.boundary_weight) == np.float32(k["boundary_weight"]["value"])
        assert np.float32(cfg.lambda_normal) == np.float32(k["lambda4"]["value"])
        assert cfg.lambda_load == 0.0
