"""GPU parity of the multi-view building-point voting filter (Sec. 4.1,
Eq. 6-7) against the oracle: bit-exact votes, unreliability scores and
flags, on the small survey, on edge cases (exact image borders, the near
plane, points behind the camera, views without a mask, more views than one
LDS chunk, empty input) and on the full 2M-point, 64-view 5472x3648
workload."""
import numpy as np
import pytest
import torch

import scenes
from oracle import grouping as og
from oracle import voting as ov
from paper_2501_01677_amd import survey as gs
from scenes import survey as sv

pytestmark = pytest.mark.gpu


def _run_vote(s, tau, masks=None, z_near=0.2):
    masks = s.masks if masks is None else masks
    pts = torch.from_numpy(s.points).cuda()
    dm = [None if m is None else torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in masks]
    votes, us, flags = gs.vote(pts, s.cameras, dm, tau, z_near)
    torch.cuda.synchronize()
    return (votes.cpu().numpy().astype(np.int64), us.cpu().numpy().astype(np.int64), flags.cpu().numpy())


def _check(s, tau, masks=None, z_near=0.2):
    masks = s.masks if masks is None else masks
    ref = ov.vote(s.points, s.cameras, masks, tau, z_near)
    votes, us, flags = _run_vote(s, tau, masks, z_near)
    assert np.array_equal(votes, ref["votes"]), int((votes != ref["votes"]).sum())
    assert np.array_equal(us, ref["us"]), int((us != ref["us"]).sum())
    assert np.array_equal(flags, ref["flags"])
    return ref


@pytest.mark.parametrize("seed,tau", [(61, 2), (62, 0), (63, 5)])
def test_vote_small_bit_exact(seed, tau):
    print(f"[case] vote small seed={seed} tau={tau}", flush=True)
    s = sv.vote_small(seed=seed)
    ref = _check(s, tau)
    assert ref["votes"].sum() > 0 and ref["us"].sum() > 0


def test_vote_views_without_masks_and_many_views():
    """70 views (more than one 64-view LDS chunk), every third without a mask."""
    print("[case] vote 70 views, some without masks", flush=True)
    s = sv.vote_small(seed=64, n_points=5000, n_views=70, width=320, height=214)
    masks = [None if j % 3 == 0 else m for j, m in enumerate(s.masks)]
    _check(s, 3, masks)


def test_vote_exact_borders_near_plane_and_behind():
    """Projections exactly on u = 0, just below W, exactly on W (outside),
    on v = H; depths exactly at, just above and below the near plane, and
    behind the camera."""
    print("[case] vote borders", flush=True)
    W, H = 8, 6
    cam = scenes.pinhole(W, H, 1.0, 1.0, 0.0, 0.0)
    lt = float(np.nextafter(np.float32(W), np.float32(0)))
    xs = [0.0, lt, float(W), 3.5, 3.5, 0.1, 0.1, -0.0, 2.0, 2.0]
    ys = [1.0, 1.0, 1.0, 0.0, float(H), 0.5, 0.5, 0.0, 2.0, 2.0]
    zs = [1.0, 1.0, 1.0, 1.0, 1.0, 0.2, float(np.nextafter(np.float32(0.2), np.float32(1))), 1.0, -1.0, 0.0]
    pts = np.array([xs, ys, zs], np.float32)
    mask = np.zeros((H, W), np.uint8)
    mask[1, 0] = 1
    mask[1, W - 1] = 1
    mask[0, 3] = 1
    s = sv.Survey(pts, np.zeros(pts.shape[1], np.int8), [cam], [mask], np.zeros((0, 5)))
    ref = _check(s, 1)
    # u = 0 and u just below W land on masked pixels; u = W and v = H are
    # outside; depth exactly 0.2 is culled, just above is not
    assert ref["votes"].tolist()[:5] == [1, 1, 0, 1, 0]
    assert ref["us"].tolist()[5:7] == [0, 1]
    assert ref["votes"][8] == 0 and ref["us"][8] == 0 and ref["us"][9] == 0


def test_vote_empty_and_tiny_inputs():
    print("[case] vote empty / single point", flush=True)
    s = sv.vote_small(seed=65, n_points=1, n_views=3)
    _check(s, 1)
    cam = s.cameras[0]
    dm = [torch.from_numpy(s.masks[0]).cuda()]
    pts = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    votes, us, flags = gs.vote(pts, [cam], dm, 1)
    torch.cuda.synchronize()
    assert votes.numel() == 0 and flags.numel() == 0


@pytest.mark.timeout(900)
def test_vote_full_size_bit_exact():
    """The benchmarked workload: 2M points, 64 views at 5472x3648."""
    print("[case] vote full 2M points x 64 views", flush=True)
    s = sv.vote_full()
    ref = _check(s, 3)
    rel = (ref["flags"] & 2) != 0
    print(f"[info] full vote: {int(rel.sum())} reliable of {s.points.shape[1]} points, "
          f"{int((ref['votes'] + ref['us']).sum())} sightings", flush=True)


# ------------------------------------------------------------ grouping

def _dbscan_gpu(points, eps, min_pts, flags=None):
    r = gs.dbscan(torch.from_numpy(np.ascontiguousarray(points)).cuda(), eps, min_pts,
                  flags=None if flags is None else torch.from_numpy(flags).cuda())
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if k != "workspace" else v) for k, v in r.items()}


def _check_dbscan(points, eps, min_pts, flags=None):
    part = None if flags is None else (flags & 2) != 0
    ref = og.dbscan_points(points, eps, min_pts, part)
    got = _dbscan_gpu(points, eps, min_pts, flags)
    assert np.array_equal(got["count"], ref["count"]), int((got["count"] != ref["count"]).sum())
    assert np.array_equal(got["label"], ref["label"]), int((got["label"] != ref["label"]).sum())
    assert np.array_equal(got["cluster"], ref["cluster"])
    assert int(got["n_clusters"][0]) == ref["n_clusters"]
    return ref, got


@pytest.mark.parametrize("seed,eps,min_pts", [(61, 5.0, 20), (62, 3.0, 10), (63, 8.0, 40)])
def test_dbscan_reliable_points_bit_exact(seed, eps, min_pts):
    print(f"[case] dbscan small seed={seed} eps={eps} min_pts={min_pts}", flush=True)
    s = sv.vote_small(seed=seed)
    v = ov.vote(s.points, s.cameras, s.masks, tau=2)
    ref, _ = _check_dbscan(s.points, eps, min_pts, v["flags"])
    assert ref["n_clusters"] > 3


def test_dbscan_lattice_ties_hand_cases_and_degenerate_inputs():
    print("[case] dbscan lattice / hand cases / degenerate", flush=True)
    rng = np.random.default_rng(5)
    g = np.stack(np.meshgrid(np.arange(0, 40, 0.5), np.arange(0, 30, 0.5)), 0).reshape(2, -1)
    g = g[:, rng.uniform(size=g.shape[1]) < 0.5]
    pts = np.vstack([g, np.zeros((1, g.shape[1]))]).astype(np.float32)
    _check_dbscan(pts, 1.0, 4)
    x = np.array([0, 1, 2, 3, 4.5, 6, 7, 8, 20], np.float32)
    _check_dbscan(np.stack([x, np.zeros_like(x), np.zeros_like(x)]), 1.5, 3)
    a = np.array([[4, 4, 4, 5, 0, 0, 0, -1, 2], [-1, 0, 1, 0, -1, 0, 1, 0, 0], [0] * 9], np.float32)
    _check_dbscan(a, 2.0, 4)
    # everything noise; everything one cluster; a single point; no point taking part
    pts = sv.vote_small(seed=66, n_points=3000).points
    ref, _ = _check_dbscan(pts, 0.5, 1000)
    assert ref["n_clusters"] == 0
    ref, _ = _check_dbscan(pts, 5000.0, 1)
    assert ref["n_clusters"] == 1
    _check_dbscan(pts[:, :1].copy(), 1.0, 1)
    _check_dbscan(pts, 3.0, 5, np.zeros(pts.shape[1], np.uint8))


def test_group_views_bit_exact():
    print("[case] group views small", flush=True)
    s = sv.vote_small(seed=61)
    v = ov.vote(s.points, s.cameras, s.masks, tau=2)
    ref = og.dbscan_points(s.points, 5.0, 20, (v["flags"] & 2) != 0)
    hits_ref, asg_ref = og.assign_views(s.points, ref["cluster"], ref["n_clusters"], s.cameras, s.masks, 30)
    pts = torch.from_numpy(s.points).cuda()
    dm = [torch.from_numpy(m).cuda() for m in s.masks]
    cl = torch.from_numpy(ref["cluster"].astype(np.int32)).cuda()
    hits, asg = gs.group_views(pts, cl, ref["n_clusters"], s.cameras, dm, 30)
    torch.cuda.synchronize()
    assert np.array_equal(hits.cpu().numpy().astype(np.int64), hits_ref)
    assert np.array_equal(asg.cpu().numpy().astype(bool), asg_ref)
    # ids beyond max_clusters are ignored
    hits2, _ = gs.group_views(pts, cl, 3, s.cameras, dm, 30)
    torch.cuda.synchronize()
    assert np.array_equal(hits2.cpu().numpy().astype(np.int64), hits_ref[:3])


@pytest.mark.timeout(900)
def test_grouping_full_size_bit_exact():
    """The benchmarked grouping: the reliable points of the 2M-point,
    64-view survey (about 1.36M points), eps 3 m, 10 points; then the views
    of every group."""
    print("[case] grouping full size", flush=True)
    s = sv.vote_full()
    v = ov.vote(s.points, s.cameras, s.masks, tau=3)
    ref, got = _check_dbscan(s.points, 3.0, 10, v["flags"])
    print(f"[info] full grouping: {ref['n_clusters']} groups over {int((ref['label'] >= 0).sum())} points",
          flush=True)
    hits_ref, asg_ref = og.assign_views(s.points, ref["cluster"], ref["n_clusters"], s.cameras, s.masks, 200)
    pts = torch.from_numpy(s.points).cuda()
    dm = [torch.from_numpy(m).cuda() for m in s.masks]
    hits, asg = gs.group_views(pts, torch.from_numpy(got["cluster"]).cuda(), ref["n_clusters"], s.cameras, dm, 200)
    torch.cuda.synchronize()
    assert np.array_equal(hits.cpu().numpy().astype(np.int64), hits_ref)
    assert np.array_equal(asg.cpu().numpy().astype(bool), asg_ref)
