"""Building grouping (Sec. 4.1, "Building Grouping"): DBSCAN over the
reliable building points by geographic proximity, and the views each group
keeps.  TEST INFRASTRUCTURE ONLY.

DBSCAN (the clustering the paper names), written as its definition:

  N(p)      = { q : |p - q| <= eps }   (p itself included), on the ground
              plane coordinates (x, y) -- "geographic proximity"
  core(p)   = |N(p)| >= min_pts
  clusters  = connected components of the graph whose vertices are the core
              points and whose edges join core points within eps
  border p  = non-core point with a core point in N(p): it joins a cluster
              of one of those core points
  noise     = every other point (label -1)

Readings (where DBSCAN leaves a choice or the paper is silent):
  - Distances are decided in FP32 with one operation order on both sides:
    dx = px - qx, dy = py - qy, d2 = dx*dx + dy*dy, each operation rounded
    on its own, compared with e2 = eps*eps rounded to FP32: q in N(p) iff
    d2 <= e2.  The relation is symmetric (the squares of dx and -dx agree).
  - A cluster is named by the smallest point index among its core points.
  - A border point reachable from several clusters joins the one with the
    smallest name (DBSCAN itself leaves this to the visiting order).  With
    these two rules the labelling is unique.
  - Compact cluster ids 0..k-1 number the clusters in ascending order of
    their names.

View assignment ("subgroups that each contain the ... original images"):
view j belongs to group c when at least `min_hits` points of c land inside
the view's building mask, with the FP32 projection of the voting filter
(``oracle.voting.project``).
"""
import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

from . import voting as ov

F32 = np.float32


def neighbour_pairs(xy, eps):
    """The neighbour relation, in the order of a uniform grid of cell side
    1.001 eps (every neighbour of a point lies in the 3x3 cells around it,
    so the grid only picks the candidates; the decision is the FP32 rule of
    the module docstring).  Returns (order, rows, cols): order = the point
    of each grid position; rows, cols = int32 grid positions of every
    ordered pair within eps (self pairs included), rows nondecreasing."""
    x = np.asarray(xy[0], F32)
    y = np.asarray(xy[1], F32)
    n = len(x)
    e2 = F32(eps) * F32(eps)
    if n == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32)
    side = 1.001 * float(eps)
    cx = np.floor((x.astype(np.float64) - x.min()) / side).astype(np.int64)
    cy = np.floor((y.astype(np.float64) - y.min()) / side).astype(np.int64)
    gx = int(cx.max()) + 1
    cell = cy * gx + cx
    order = np.argsort(cell, kind="stable")
    xs, ys = x[order], y[order]
    uniq, start, count = np.unique(cell[order], return_index=True, return_counts=True)
    where = {int(c): (int(s), int(k)) for c, s, k in zip(uniq, start, count)}
    rows, cols = [], []
    for c, (s0, k) in where.items():
        ccx, ccy = c % gx, c // gx
        cand = []
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                key = (ccy + dy) * gx + ccx + dx
                if 0 <= ccx + dx < gx and key in where:
                    s2, k2 = where[key]
                    cand.append(np.arange(s2, s2 + k2))
        b = np.concatenate(cand)
        ddx = xs[s0:s0 + k, None] - xs[b][None, :]
        ddy = ys[s0:s0 + k, None] - ys[b][None, :]
        d2 = ddx * ddx + ddy * ddy
        assert d2.dtype == F32
        ii, jj = np.nonzero(d2 <= e2)
        rows.append((ii + s0).astype(np.int32))
        cols.append(b[jj].astype(np.int32))
    return order, np.concatenate(rows), np.concatenate(cols)


def dbscan(xy, eps, min_pts):
    """Returns dict(count = |N(p)| int64, core bool, label int64 (cluster
    name or -1), cluster int64 (compact id or -1), n_clusters)."""
    n = np.asarray(xy).shape[1]
    out = dict(count=np.zeros(n, np.int64), core=np.zeros(n, bool), label=np.full(n, -1, np.int64),
               cluster=np.full(n, -1, np.int64), n_clusters=0)
    if n == 0:
        return out
    order, R, Cc = neighbour_pairs(xy, eps)
    # everything below is in grid positions; `order` maps back to points
    cnt = np.bincount(R, minlength=n)
    core = cnt >= min_pts
    # clusters: connected components over core-core pairs (each pair once)
    keep = core[R] & core[Cc] & (R < Cc)
    R2, C2 = R[keep], Cc[keep]
    indptr = np.zeros(n + 1, np.int64)
    indptr[1:] = np.cumsum(np.bincount(R2, minlength=n))
    g = csr_matrix((np.ones(len(R2), np.int8), C2, indptr), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    # a cluster's name: the smallest point index among its core points
    big = np.iinfo(np.int64).max
    name = np.full(comp.max() + 1, big, np.int64)
    cpos = np.flatnonzero(core)
    np.minimum.at(name, comp[cpos], order[cpos])
    label = np.full(n, -1, np.int64)
    label[cpos] = name[comp[cpos]]
    # border points: the smallest name among their core neighbours
    b = ~core[R] & core[Cc]
    best = np.full(n, big, np.int64)
    np.minimum.at(best, R[b], label[Cc[b]])
    border = ~core & (best != big)
    label[border] = best[border]
    # back to point order
    out["count"][order] = cnt
    out["core"][order] = core
    out["label"][order] = label
    names = np.unique(label[label >= 0])
    lab = out["label"]
    out["cluster"][lab >= 0] = np.searchsorted(names, lab[lab >= 0])
    out["n_clusters"] = len(names)
    return out


def dbscan_points(points, eps, min_pts, part=None):
    """DBSCAN over the points [2 or 3][M] (x, y used) that take part
    (part: bool [M] or None = all).  Labels are returned for all M points:
    cluster names are original point indices, -1 for noise and for points
    that take no part."""
    pts = np.asarray(points)
    m = pts.shape[1]
    sel = np.arange(m) if part is None else np.flatnonzero(part)
    r = dbscan(pts[:2, sel], eps, min_pts)
    out = dict(count=np.zeros(m, np.int64), core=np.zeros(m, bool), label=np.full(m, -1, np.int64),
               cluster=np.full(m, -1, np.int64), n_clusters=r["n_clusters"])
    out["count"][sel] = r["count"]
    out["core"][sel] = r["core"]
    lab = r["label"]
    out["label"][sel] = np.where(lab >= 0, sel[np.maximum(lab, 0)], -1)
    out["cluster"][sel] = r["cluster"]
    return out


def assign_views(points, cluster, n_clusters, cams, masks, min_hits, z_near=0.2):
    """hits[c][j] = points of cluster c inside view j's mask; assigned =
    hits >= min_hits.  points float32 [3][M] (world), cluster int [M]."""
    hits = np.zeros((n_clusters, len(cams)), np.int64)
    lab = np.asarray(cluster)
    for j, (cam, mask) in enumerate(zip(cams, masks)):
        inside, iu, iv = ov.project(points, cam, z_near)
        hit = np.ones(len(iu), bool) if mask is None else np.asarray(mask)[iv, iu] != 0
        sel = np.flatnonzero(inside)[hit]
        sel = sel[lab[sel] >= 0]
        hits[:, j] = np.bincount(lab[sel], minlength=n_clusters)
    return hits, hits >= min_hits
