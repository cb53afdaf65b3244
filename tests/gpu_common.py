"""Helpers shared by the GPU parity tests: run scenes through the HIP
library and compare with the FP64 oracle under the tolerance protocol.

Tolerances (per output channel, at every masked pixel):
  rgb, normal, alpha   |gpu - ref| <= 1e-4 + allowance
  dist                 |gpu - ref| <= 1e-4 * max(1, |ref|) + allowance
  depth                relative 1e-4 where |N . r| >= 0.1 alpha, else 1e-3;
                       pixels whose depth decision is near its guard or that
                       carry any normal/distance allowance are excluded
  n_contrib            exact unless the pixel carries an allowance
  unmasked pixels      exactly 0 on every output
The allowance is the oracle's bound on what an FP32 decision taken the
other way (alpha cut-off, transmittance stop, normal flip) can change.
"""
import numpy as np
import torch

import scenes
from oracle import OracleConfig
from oracle import composite as oc
from paper_2501_01677_amd.raster import Batch, RenderConfig, gaussians_to_device

CFG = OracleConfig()


def cuda_available():
    return torch.cuda.is_available()


def device_scene(scene, cfg=None, want_grads=True, pair_capacity=None, **kw):
    sets = [gaussians_to_device(s) for s in scene.sets]
    renders = []
    for rd in scene.renders:
        m = None if rd.mask is None else torch.from_numpy(np.ascontiguousarray(rd.mask)).cuda()
        renders.append(dict(set=rd.set_index, camera=rd.camera, mask=m))
    return Batch(sets, renders, cfg or RenderConfig(), pair_capacity=pair_capacity,
                 want_grads=want_grads, **kw)


def outputs_numpy(batch, r):
    return {k: v.detach().cpu().numpy() for k, v in batch.out[r].items()}


def compare_images(gpu, ref, render, report=None):
    """Checks GPU output planes against an oracle ``render`` result at its
    pixels (the masked pixels or a sample) and zeros elsewhere."""
    pix = ref["pix"]
    v, u = pix[:, 0], pix[:, 1]
    allow = ref["allow"]
    bad = {}
    used = np.zeros(len(pix), bool)  # pixels whose error exceeds the tolerance without the allowance

    def chk(name, got, want, tol, base=None):
        err = np.abs(got - want)
        fail = err > tol
        if base is not None:
            used[(err > base).reshape(len(pix), -1).any(1)] = True
        if np.any(fail):
            i = np.flatnonzero(fail.reshape(len(pix), -1).any(1))[:5]
            bad[name] = (int(fail.sum()), float(err.max()), [tuple(pix[j]) for j in i])

    chk("rgb", gpu["rgb"][:, v, u].T, ref["rgb"], 1e-4 + allow[:, 0:3], 1e-4)
    chk("normal", gpu["normal"][:, v, u].T, ref["normal"], 1e-4 + allow[:, 3:6], 1e-4)
    dbase = 1e-4 * np.maximum(1, np.abs(ref["dist"]))
    chk("dist", gpu["dist"][v, u], ref["dist"], dbase + allow[:, 6], dbase)
    chk("alpha", gpu["alpha"][v, u], ref["alpha"], 1e-4 + allow[:, 7], 1e-4)
    ok = ~ref["depth_unreliable"]
    rel = np.where(np.abs(ref["den"]) >= 0.1 * ref["alpha"], 1e-4, 1e-3)
    dtol = rel * np.maximum(1.0, np.abs(ref["depth"]))
    chk("depth", gpu["depth"][v, u][ok], ref["depth"][ok], dtol[ok])
    exact = allow.sum(1) == 0
    nc_bad = gpu["n_contrib"][v, u][exact] != ref["n_contrib"][exact]
    if np.any(nc_bad):
        bad["n_contrib"] = int(nc_bad.sum())
    if report is not None:
        report["allow_pixels"] = int((allow.sum(1) > 0).sum())
        report["pixels"] = len(pix)
        report["depth_excluded"] = int((~ok).sum())
        report["used_allowance"] = int(used.sum())
    return bad


def check_unmasked_zero(gpu, mask):
    if mask is None:
        return True
    off = mask == 0
    for k, a in gpu.items():
        plane = a if a.ndim == 2 else a.reshape(-1, *a.shape[-2:])
        if a.ndim == 2:
            if np.any(plane[off] != 0):
                return False
        else:
            if np.any(plane[:, off] != 0):
                return False
    return True


def grad_tolerance_check(got, ref, exclude=None):
    """|g - g_ref| <= 1e-3 |g_ref| + 1e-4 max|g_ref| elementwise; returns
    (ok, worst ratio, relative L2 error)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    if exclude is not None:
        got = got[..., ~exclude]
        ref = ref[..., ~exclude]
    scale = np.abs(ref).max() if ref.size else 0.0
    tol = 1e-3 * np.abs(ref) + 1e-4 * scale + 1e-12
    err = np.abs(got - ref)
    ratio = float((err / tol).max()) if err.size else 0.0
    rel = float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30))
    return ratio <= 1.0, ratio, rel
