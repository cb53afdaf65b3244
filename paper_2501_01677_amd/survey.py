"""Python boundary of the survey-side steps around the rasterizer: the
multi-view building-point voting filter (Sec. 4.1, Eq. 6-7) and the
building grouping (Sec. 4.1: DBSCAN and the views of each group), and the
depth fusion and TSDF integration ahead of meshing (Sec. 4.4).

Argument marshalling only: the views are packed into the C structs of
include/pgsag.h, uploaded into a caller-owned device tensor, and every step
runs in the library's HIP kernels.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi as A
from .raster import _p, _stream, make_camera


def pack_views(cameras, masks):
    """Host array of pgsag_vote_view and its device copy (uint8 tensor).
    masks: device uint8 [H][W] tensors (or None = every pixel); they must
    outlive every call that uses the returned views."""
    n = len(cameras)
    if len(masks) != n:
        raise ValueError("one mask (or None) per camera")
    host = (A.VoteView * n)()
    for j, (cam, m) in enumerate(zip(cameras, masks)):
        host[j].cam = make_camera(cam)
        if m is not None:
            if m.dtype != torch.uint8 or not m.is_cuda or not m.is_contiguous():
                raise ValueError("masks must be contiguous uint8 device tensors")
            if tuple(m.shape) != (cam.height, cam.width):
                raise ValueError(f"mask {j} has shape {tuple(m.shape)}, camera is {cam.height}x{cam.width}")
        host[j].mask = None if m is None else m.data_ptr()
    raw = np.frombuffer(bytes(host), dtype=np.uint8)
    dev = torch.from_numpy(raw.copy()).cuda()
    return host, dev


def vote(points, cameras, masks, tau, z_near=0.2, views=None, out=None, stream=None):
    """Eq. 6-7 for every point of points (device float32 [3][M]) over the
    views: returns (votes uint16 [M], us uint16 [M], flags uint8 [M]);
    flags bit 0 = potential building point, bit 1 = reliable.
    `views` may pass a (host, device) pair from pack_views to skip packing."""
    if points.dtype != torch.float32 or not points.is_cuda or points.dim() != 2 or points.shape[0] != 3:
        raise ValueError("points must be a float32 device tensor [3][M]")
    points = points.contiguous()
    m = points.shape[1]
    host, dev = views if views is not None else pack_views(cameras, masks)
    if out is None:
        out = (torch.empty(m, dtype=torch.uint16, device=points.device),
               torch.empty(m, dtype=torch.uint16, device=points.device),
               torch.empty(m, dtype=torch.uint8, device=points.device))
    votes, us, flags = out
    A.check(A.lib().pgsag_vote(host, _p(dev), len(host), _p(points), m, float(z_near), int(tau),
                               _p(votes), _p(us), _p(flags), _stream(stream)), "pgsag_vote")
    return votes, us, flags


def dbscan(points, eps, min_pts, flags=None, flag_mask=2, workspace=None, stream=None):
    """DBSCAN over the (x, y) of points (device float32 [3][M]) that take part
    (flags & flag_mask, or all).  Returns dict(count, label, cluster int32
    [M], n_clusters uint32 [1] device tensors)."""
    if points.dtype != torch.float32 or not points.is_cuda or points.dim() != 2 or points.shape[0] != 3:
        raise ValueError("points must be a float32 device tensor [3][M]")
    points = points.contiguous()
    m = points.shape[1]
    L = A.lib()
    need = C.c_uint64()
    A.check(L.pgsag_dbscan_workspace(m, C.byref(need)), "pgsag_dbscan_workspace")
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(max(1, need.value), dtype=torch.uint8, device=points.device)
    if flags is not None and (flags.dtype != torch.uint8 or flags.numel() != m or not flags.is_cuda):
        raise ValueError("flags must be a uint8 device tensor [M]")
    dev = points.device
    out = dict(count=torch.empty(m, dtype=torch.int32, device=dev), label=torch.empty(m, dtype=torch.int32, device=dev),
               cluster=torch.empty(m, dtype=torch.int32, device=dev),
               n_clusters=torch.empty(1, dtype=torch.int32, device=dev))
    A.check(L.pgsag_dbscan(_p(points), m, _p(flags), int(flag_mask), float(eps), int(min_pts), _p(out["count"]),
                           _p(out["label"]), _p(out["cluster"]), _p(out["n_clusters"]), _p(workspace),
                           workspace.numel(), _stream(stream)), "pgsag_dbscan")
    out["workspace"] = workspace
    return out


DBSCAN_STATIC_MAX_POINTS = 1 << 19


def dbscan_static(points, eps, min_pts, flags=None, flag_mask=2, out=None, stream=None):
    """dbscan() on the library's static scratch (pgsag_dbscan_static): no
    workspace, and with ``out`` (a dict as dbscan returns) nothing allocated.
    At most DBSCAN_STATIC_MAX_POINTS points; calls overlapping on one GPU
    race."""
    if points.dtype != torch.float32 or not points.is_cuda or points.dim() != 2 or points.shape[0] != 3:
        raise ValueError("points must be a float32 device tensor [3][M]")
    if not points.is_contiguous():
        raise ValueError("points must be contiguous")
    m = points.shape[1]
    if flags is not None and (flags.dtype != torch.uint8 or flags.numel() != m or not flags.is_cuda):
        raise ValueError("flags must be a uint8 device tensor [M]")
    if out is None:
        dev = points.device
        out = dict(count=torch.empty(m, dtype=torch.int32, device=dev),
                   label=torch.empty(m, dtype=torch.int32, device=dev),
                   cluster=torch.empty(m, dtype=torch.int32, device=dev),
                   n_clusters=torch.empty(1, dtype=torch.int32, device=dev))
    A.check(A.lib().pgsag_dbscan_static(_p(points), m, _p(flags), int(flag_mask), float(eps), int(min_pts),
                                        _p(out["count"]), _p(out["label"]), _p(out["cluster"]),
                                        _p(out["n_clusters"]), _stream(stream)), "pgsag_dbscan_static")
    return out


def group_views(points, cluster, max_clusters, cameras, masks, min_hits, z_near=0.2, views=None, stream=None):
    """hits [max_clusters][V] uint32 (as int32 storage) and assigned uint8."""
    points = points.contiguous()
    m = points.shape[1]
    host, dev = views if views is not None else pack_views(cameras, masks)
    nv = len(host)
    hits = torch.empty((max(1, max_clusters), nv), dtype=torch.int32, device=points.device)
    assigned = torch.empty((max(1, max_clusters), nv), dtype=torch.uint8, device=points.device)
    A.check(A.lib().pgsag_group_views(host, _p(dev), nv, _p(points), m, _p(cluster), int(max_clusters),
                                      float(z_near), int(min_hits), _p(hits), _p(assigned), _stream(stream)),
            "pgsag_group_views")
    return hits[:max_clusters], assigned[:max_clusters]


def fuse_depth(maps, out=None, count=True, stream=None):
    """Mean fusion (Sec. 4.4) of device float32 [H][W] depth maps of one view:
    returns (fused float32 [H][W], count uint8 [H][W] or None)."""
    if not maps:
        raise ValueError("need at least one depth map")
    H, W = maps[0].shape
    for m in maps:
        if m.dtype != torch.float32 or not m.is_cuda or not m.is_contiguous() or tuple(m.shape) != (H, W):
            raise ValueError("depth maps must be contiguous float32 device tensors of one size")
    fused = out if out is not None else torch.empty((H, W), dtype=torch.float32, device=maps[0].device)
    cnt = torch.empty((H, W), dtype=torch.uint8, device=maps[0].device) if count else None
    ptrs = (C.c_void_p * len(maps))(*[m.data_ptr() for m in maps])
    A.check(A.lib().pgsag_fuse_depth(ptrs, len(maps), W, H, _p(fused), _p(cnt), _stream(stream)),
            "pgsag_fuse_depth")
    return fused, cnt


def make_volume(origin, voxel, dims, trunc) -> A.Volume:
    v = A.Volume()
    v.origin = (C.c_float * 3)(*[float(x) for x in np.asarray(origin, np.float32)])
    v.voxel = float(voxel)
    v.nx, v.ny, v.nz = (int(d) for d in dims)
    v.trunc = float(trunc)
    return v


def pack_depth_views(cameras, depths):
    n = len(cameras)
    host = (A.DepthView * n)()
    for j, (cam, d) in enumerate(zip(cameras, depths)):
        if d.dtype != torch.float32 or not d.is_cuda or not d.is_contiguous():
            raise ValueError("depth maps must be contiguous float32 device tensors")
        if tuple(d.shape) != (cam.height, cam.width):
            raise ValueError(f"depth map {j} has shape {tuple(d.shape)}, camera is {cam.height}x{cam.width}")
        host[j].cam = make_camera(cam)
        host[j].depth = d.data_ptr()
    raw = np.frombuffer(bytes(host), dtype=np.uint8) if n else np.zeros(1, np.uint8)
    return host, torch.from_numpy(raw.copy()).cuda()


def tsdf_integrate(volume, cameras, depths, z_near=0.2, tsdf=None, weight=None, accumulate=False, views=None,
                   stream=None):
    """Projective TSDF (Sec. 4.4) of the depth maps (device float32 [H][W],
    one per camera) into the volume dict(origin, voxel, dims, trunc).
    Returns (tsdf, weight), device float32 [nz][ny][nx]."""
    nx, ny, nz = volume["dims"]
    vol = make_volume(volume["origin"], volume["voxel"], volume["dims"], volume["trunc"])
    dev = torch.device("cuda")
    if tsdf is None:
        tsdf = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
    if weight is None:
        weight = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
    host, dv = views if views is not None else pack_depth_views(cameras, depths)
    A.check(A.lib().pgsag_tsdf_integrate(C.byref(vol), host, _p(dv), len(host), float(z_near), _p(tsdf),
                                         _p(weight), int(bool(accumulate)), _stream(stream)),
            "pgsag_tsdf_integrate")
    return tsdf, weight
