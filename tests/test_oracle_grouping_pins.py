"""Pins of the building-grouping oracle (Sec. 4.1, DBSCAN and the views of
each group) against what fixes it from outside: scikit-learn's DBSCAN (a
library routine) on inputs without distance near-ties, a plain sequential
DBSCAN written here (seed expansion in index order, the textbook form),
hand-worked cases (a neighbour exactly at eps, a border point between two
clusters, noise) and the vote counts of the voting oracle."""
import numpy as np
import pytest
from sklearn.cluster import DBSCAN

from oracle import grouping as og
from oracle import voting as ov
from scenes import survey as sv


def _tie_free_points(seed, n, eps, blobs=6):
    """Blobs plus uniform clutter, with the points of every pair whose
    distance is within 1e-4 relative of eps removed (no near-ties, so FP32
    and FP64 decisions agree)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, 60, (blobs, 2))
    p = c[rng.integers(0, blobs, n)] + rng.normal(0, 2.0, (n, 2))
    p = np.vstack([p, rng.uniform(-10, 70, (n // 10, 2))]).astype(np.float32)
    d = np.sqrt(((p[:, None, :].astype(np.float64) - p[None, :, :]) ** 2).sum(-1))
    near = np.abs(d - eps) <= 1e-4 * eps
    drop = np.zeros(len(p), bool)
    for i, j in zip(*np.nonzero(np.triu(near, 1))):
        if not drop[i] and not drop[j]:
            drop[j] = True
    return p[~drop].T.copy()


def _partition(labels):
    """Canonical partition: each label replaced by the smallest index holding it."""
    out = np.full(len(labels), -1, np.int64)
    for lab in np.unique(labels[labels >= 0]):
        idx = np.flatnonzero(labels == lab)
        out[idx] = idx.min()
    return out


@pytest.mark.parametrize("seed,eps,min_pts", [(0, 1.5, 5), (1, 2.5, 10), (2, 1.0, 3)])
def test_matches_sklearn_on_tie_free_points(seed, eps, min_pts):
    xy = _tie_free_points(seed, 900, eps)
    r = og.dbscan(xy, eps, min_pts)
    sk = DBSCAN(eps=eps, min_samples=min_pts).fit(xy.T.astype(np.float64))
    core_sk = np.zeros(xy.shape[1], bool)
    core_sk[sk.core_sample_indices_] = True
    assert np.array_equal(r["core"], core_sk)
    # the same clusters over the core points
    assert np.array_equal(_partition(np.where(core_sk, r["label"], -1)),
                          _partition(np.where(core_sk, sk.labels_, -1)))
    # the same noise
    assert np.array_equal(r["label"] < 0, sk.labels_ < 0)
    # border points: both join a cluster of one of their core neighbours;
    # the oracle takes the one with the smallest name
    d2 = ((xy[:, :, None] - xy[:, None, :]) ** 2).sum(0)
    border = (~r["core"]) & (r["label"] >= 0)
    assert border.sum() > 0
    for p in np.flatnonzero(border):
        nb = np.flatnonzero((d2[p] <= eps * eps) & r["core"])
        names = set(r["label"][nb].tolist())
        assert r["label"][p] == min(names)
        sk_names = set(sk.labels_[nb].tolist())
        assert sk.labels_[p] in sk_names
    assert r["n_clusters"] == len(set(sk.labels_.tolist()) - {-1})


def _sequential_dbscan(xy, eps, min_pts):
    """Textbook DBSCAN: visit points in index order, grow a cluster from each
    unvisited core point by expanding its core neighbours; border points get
    the first cluster that reaches them (kept here only for core points)."""
    x, y = xy[0].astype(np.float32), xy[1].astype(np.float32)
    n = len(x)
    e2 = np.float32(eps) * np.float32(eps)
    nbrs = []
    for p in range(n):
        dx = x[p] - x
        dy = y[p] - y
        nbrs.append(np.flatnonzero(dx * dx + dy * dy <= e2))
    core = np.array([len(nb) >= min_pts for nb in nbrs])
    lab = np.full(n, -1)
    for p in range(n):
        if not core[p] or lab[p] >= 0:
            continue
        lab[p] = p
        stack = [p]
        while stack:
            q = stack.pop()
            for r in nbrs[q]:
                if lab[r] < 0:
                    lab[r] = p
                    if core[r]:
                        stack.append(r)
    return core, lab, nbrs


@pytest.mark.parametrize("seed", [3, 4])
def test_matches_sequential_dbscan_on_grid_points_with_exact_ties(seed):
    """Points on a 0.5 m lattice (many distances exactly eps) with a few
    removed: the FP32 rule includes neighbours at exactly eps."""
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(np.arange(0, 12, 0.5), np.arange(0, 8, 0.5)), 0).reshape(2, -1)
    keep = rng.uniform(size=g.shape[1]) < 0.55
    xy = g[:, keep].astype(np.float32)
    eps, min_pts = 1.0, 4
    r = og.dbscan(xy, eps, min_pts)
    core, lab, nbrs = _sequential_dbscan(xy, eps, min_pts)
    assert np.array_equal(r["core"], core)
    assert np.array_equal(r["count"], np.array([len(nb) for nb in nbrs]))
    # clusters named by their first core point, as the sequential visit names them
    assert np.array_equal(np.where(core, r["label"], -1), np.where(core, lab, -1))
    assert np.array_equal(r["label"] < 0, lab < 0)


def test_hand_worked_line():
    # x = 0, 1, 2, 3 | 4.5 | 6, 7, 8 | 20 on y = 0, eps = 1.5, min_pts = 3:
    #   N(0) = {0,1}        border (1 is core)      -> cluster of 1 (name 1)
    #   N(1) = {0,1,2}      core;  N(2) = {1,2,3} core
    #   N(3) = {2,3,4}      core (3 to 4.5 is exactly 1.5: included)
    #   N(4) = {3,4,5}      core (4.5 to 6 is exactly 1.5) -> joins 1..7
    #   N(5) = {4,5,6}, N(6) = {5,6,7} core; N(7) = {6,7} border
    #   N(8) = {8}          noise
    x = np.array([0, 1, 2, 3, 4.5, 6, 7, 8, 20], np.float32)
    xy = np.stack([x, np.zeros_like(x)])
    r = og.dbscan(xy, 1.5, 3)
    assert r["count"].tolist() == [2, 3, 3, 3, 3, 3, 3, 2, 1]
    assert r["core"].tolist() == [False, True, True, True, True, True, True, False, False]
    assert r["label"].tolist() == [1, 1, 1, 1, 1, 1, 1, 1, -1]
    # moving 4.5 to 4.6 breaks the chain: 3 and 5 lose a neighbour
    x2 = x.copy()
    x2[4] = 4.6
    r2 = og.dbscan(np.stack([x2, np.zeros_like(x2)]), 1.5, 3)
    #   N(3) = {2,3} border of 1; N(4) = {4,5} border of 5; N(5) = {4,5,6} core
    assert r2["core"].tolist() == [False, True, True, False, False, True, True, False, False]
    assert r2["label"].tolist() == [1, 1, 1, 1, 5, 5, 5, 5, -1]
    assert r2["cluster"].tolist() == [0, 0, 0, 0, 1, 1, 1, 1, -1]
    assert r2["n_clusters"] == 2


def test_border_point_between_two_clusters_joins_the_smaller_name():
    # cluster A: (4,-1), (4,0), (4,1), (5,0); cluster B mirrored at x <= 0;
    # P = (2, 0) is exactly eps = 2 from (4,0) and (0,0) and sqrt(5) from
    # the others: |N(P)| = 3 < 4, a border point of both clusters
    a = [[4, 4, 4, 5], [-1, 0, 1, 0]]
    b = [[0, 0, 0, -1], [-1, 0, 1, 0]]
    xy = np.array([a[0] + b[0] + [2], a[1] + b[1] + [0]], np.float32)
    r = og.dbscan(xy, 2.0, 4)
    assert r["count"].tolist() == [4, 5, 4, 4, 4, 5, 4, 4, 3]
    assert r["core"].tolist() == [True] * 8 + [False]
    assert r["label"].tolist() == [0, 0, 0, 0, 4, 4, 4, 4, 0]
    # with B listed first, B holds the smaller name and P joins B
    xy2 = xy[:, [4, 5, 6, 7, 0, 1, 2, 3, 8]]
    r2 = og.dbscan(xy2, 2.0, 4)
    assert r2["label"].tolist() == [0, 0, 0, 0, 4, 4, 4, 4, 0]
    assert r2["cluster"].tolist() == [0, 0, 0, 0, 1, 1, 1, 1, 0]


def test_subset_labels_and_view_hits_on_the_survey():
    s = sv.vote_small(seed=61)
    v = ov.vote(s.points, s.cameras, s.masks, tau=2)
    rel = (v["flags"] & 2) != 0
    g = og.dbscan_points(s.points, 5.0, 20, rel)
    assert g["n_clusters"] > 10
    # points that take no part are never labelled; names are indices of
    # core points of their own cluster
    assert np.all(g["label"][~rel] == -1)
    lab = g["label"]
    named = lab >= 0
    assert np.all(g["core"][lab[named]]) and np.all(lab[lab[named]] == lab[named])
    # the same clustering run directly on the selected points
    sub = og.dbscan(s.points[:2, rel], 5.0, 20)
    assert np.array_equal(g["core"][rel], sub["core"])
    assert np.array_equal(g["cluster"][rel], sub["cluster"])
    # per cluster, the hits summed over views equal the votes of its points
    hits, assigned = og.assign_views(s.points, g["cluster"], g["n_clusters"], s.cameras, s.masks, 30)
    per = np.bincount(g["cluster"][named], weights=v["votes"][named], minlength=g["n_clusters"])
    assert np.array_equal(hits.sum(1), per.astype(np.int64))
    assert np.array_equal(assigned, hits >= 30)
    assert assigned.any() and not assigned.all()
