"""pgsag_dbscan_static (DBSCAN on the library's static device scratch, for
callers that cannot allocate) against pgsag_dbscan (the same kernels on a
caller workspace): bit-exact counts, labels, cluster ids and cluster count,
through the C ABI, on two calls in a row -- the second on a smaller input,
so it runs on the scratch the first call left behind -- and once more at the
scratch's maximum size."""
import numpy as np
import pytest
import torch

from oracle import voting as ov
from paper_2501_01677_amd import survey as gs
from scenes import survey as sv

pytestmark = pytest.mark.gpu


def _run_both(points, eps, min_pts, flags=None):
    pts = torch.from_numpy(np.ascontiguousarray(points)).cuda()
    fl = None if flags is None else torch.from_numpy(flags).cuda()
    m = pts.shape[1]
    # outputs filled with garbage first: every element must be written
    out = {k: torch.full((m,), -7, dtype=torch.int32, device="cuda") for k in ("count", "label", "cluster")}
    out["n_clusters"] = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    got = gs.dbscan_static(pts, eps, min_pts, flags=fl, out=out)
    want = gs.dbscan(pts, eps, min_pts, flags=fl)
    torch.cuda.synchronize()
    for k in ("count", "label", "cluster", "n_clusters"):
        a, b = got[k].cpu().numpy(), want[k].cpu().numpy()
        assert np.array_equal(a, b), (k, int((a != b).sum()))
    return int(want["n_clusters"][0])


def test_static_scratch_dbscan_matches_workspace_dbscan_twice():
    print("[case] dbscan static scratch: 30000 points, then 3000", flush=True)
    s = sv.vote_small(seed=61)
    v = ov.vote(s.points, s.cameras, s.masks, tau=2)
    k1 = _run_both(s.points, 5.0, 20, v["flags"])
    assert k1 > 3
    # smaller input, other parameters, every point taking part
    sub = np.ascontiguousarray(s.points[:, ::10][:, :3000])
    k2 = _run_both(sub, 8.0, 4)
    assert k2 >= 1
    print(f"[info] {k1} then {k2} clusters", flush=True)


def test_static_scratch_dbscan_at_its_maximum_size_and_beyond():
    n = gs.DBSCAN_STATIC_MAX_POINTS
    print(f"[case] dbscan static scratch at {n} points", flush=True)
    s = sv.survey(67, n, 4, width=1600, height=1200, f=1400.0, n_boxes=40, half_extent=300.0)
    assert s.points.shape[1] == n
    k = _run_both(s.points, 1.5, 12)
    assert k > 100
    pts = torch.zeros((3, n + 1), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError, match="n_points must be in"):
        gs.dbscan_static(pts, 3.0, 10)
