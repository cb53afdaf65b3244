"""Pins of the voting-filter oracle (Sec. 4.1, Eq. 6-7) against what the
definition and geometry fix, independently of the oracle's own code:
a hand-worked two-view example, an FP64 3x4 projection-matrix route to the
pixel of every point, and the invariants of the counts (full, empty and
complemented masks, view order)."""
import numpy as np
import pytest

import scenes
from oracle import voting as ov
from scenes import survey as sv


def _cam(W, H, f, cx, cy, R=None, t=None):
    return scenes.pinhole(W, H, f, f, cx, cy, R, t)


def test_hand_worked_two_view_example():
    # View 0: R = I, t = 0, f = 2, principal point (2, 2), 4 x 3 pixels.
    #   p0 (0, 0, 1)      -> (2, 2): pixel (2, 2)
    #   p1 (-1, -1, 1)    -> (0, 0): pixel (0, 0)
    #   p2 (1, 0, 1)      -> (4, 2): x = W, outside
    #   p3 (0, 0.45, 1)   -> (2, 2.9): pixel (2, 2)
    #   p4 (0, 0, 0.1)    -> depth 0.1 <= 0.2: not in the image
    #   p5 (-0.5, 0.2, 2) -> (1.5, 2.2): pixel (1, 2)
    # View 1: the camera moved 1 along +x (t = (-1, 0, 0)):
    #   p0 -> (0, 2): pixel (0, 2);  p1 -> (-2, 0): outside;
    #   p2 -> (2, 2): pixel (2, 2);  p3 -> (0, 2.9): pixel (0, 2);
    #   p4 -> not in the image;      p5 -> (0.5, 2.2): pixel (0, 2)
    # Masks (row v, column u): view 0 marks (2, 2) and (0, 0);
    # view 1 marks only (2, 2).
    pts = np.array([[0, -1, 1, 0, 0, -0.5],
                    [0, -1, 0, 0.45, 0, 0.2],
                    [1, 1, 1, 1, 0.1, 2]], np.float32)
    c0 = _cam(4, 3, 2.0, 2.0, 2.0)
    c1 = _cam(4, 3, 2.0, 2.0, 2.0, t=np.array([-1.0, 0, 0]))
    m0 = np.zeros((3, 4), np.uint8)
    m0[2, 2] = 1
    m0[0, 0] = 1
    m1 = np.zeros((3, 4), np.uint8)
    m1[2, 2] = 1
    r = ov.vote(pts, [c0, c1], [m0, m1], tau=1)
    # p0: in M_0, outside M_1 (pixel (0,2) unmasked)  -> votes 1, US 1
    # p1: in M_0, outside image 1                     -> votes 1, US 0
    # p2: outside image 0, in M_1                     -> votes 1, US 0
    # p3: in M_0, outside M_1                         -> votes 1, US 1
    # p4: in neither image                            -> votes 0, US 0
    # p5: pixel (1,2) unmasked in view 0, (0,2) in 1  -> votes 0, US 2
    assert r["votes"].tolist() == [1, 1, 1, 1, 0, 0]
    assert r["us"].tolist() == [1, 0, 0, 1, 0, 2]
    # potential iff votes > 0; reliable iff also US < tau = 1
    assert r["flags"].tolist() == [1, 3, 3, 1, 0, 0]
    r2 = ov.vote(pts, [c0, c1], [m0, m1], tau=2)
    assert r2["flags"].tolist() == [3, 3, 3, 3, 0, 0]


def _pixels_by_projection_matrix(points, cam, z_near):
    """FP64 route: P = K [R | t], h = P X~; pixel = floor(h0 / h2), floor(h1 / h2)."""
    K = np.array([[cam.fx, 0, cam.cx], [0, cam.fy, cam.cy], [0, 0, 1]], np.float64)
    P = K @ np.hstack([cam.R.astype(np.float64), cam.t.astype(np.float64)[:, None]])
    X = np.vstack([points.astype(np.float64), np.ones((1, points.shape[1]))])
    h = P @ X
    with np.errstate(divide="ignore", invalid="ignore"):
        x, y = h[0] / h[2], h[1] / h[2]
    inside = (h[2] > z_near) & (x >= 0) & (x < cam.width) & (y >= 0) & (y < cam.height)
    # distance of each projection to the nearest pixel or image edge, to keep
    # only points whose FP32 and FP64 decisions cannot differ
    margin = np.minimum(np.abs(x - np.round(x)), np.abs(y - np.round(y)))
    margin = np.where(np.abs(h[2] - z_near) < 1e-3, 0, margin)
    return inside, np.floor(x), np.floor(y), margin


@pytest.mark.parametrize("seed", [0, 1])
def test_pixels_match_an_fp64_projection_matrix(seed):
    s = sv.vote_small(seed=70 + seed, n_points=20000, n_views=6)
    for cam in s.cameras:
        inside64, x64, y64, margin = _pixels_by_projection_matrix(s.points, cam, 0.2)
        safe = margin > 1e-3
        inside, iu, iv = ov.project(s.points, cam)
        assert np.array_equal(inside[safe], inside64[safe])
        got_u = np.full(s.points.shape[1], -1)
        got_v = np.full(s.points.shape[1], -1)
        got_u[inside] = iu
        got_v[inside] = iv
        sel = safe & inside64
        assert sel.sum() > 1000
        assert np.array_equal(got_u[sel], x64[sel].astype(int))
        assert np.array_equal(got_v[sel], y64[sel].astype(int))


def test_count_invariants():
    s = sv.vote_small(seed=75, n_points=20000, n_views=6)
    pts, cams, masks = s.points, s.cameras, s.masks
    seen = np.zeros(pts.shape[1], np.int64)
    for cam in cams:
        seen += ov.project(pts, cam)[0]
    r = ov.vote(pts, cams, masks, tau=2)
    # every in-image sighting is either a vote or an unreliability count
    assert np.array_equal(r["votes"] + r["us"], seen)
    # full masks: no unreliability; every seen point is a potential point
    full = ov.vote(pts, cams, [None] * len(cams), tau=1)
    assert np.array_equal(full["votes"], seen) and not full["us"].any()
    assert np.array_equal(full["flags"] != 0, seen > 0)
    # empty masks: no votes, so no potential or reliable point
    empty = ov.vote(pts, cams, [np.zeros_like(m) for m in masks], tau=100)
    assert not empty["votes"].any() and not empty["flags"].any()
    assert np.array_equal(empty["us"], seen)
    # complemented masks swap the two counts
    comp = ov.vote(pts, cams, [1 - m for m in masks], tau=2)
    assert np.array_equal(comp["votes"], r["us"]) and np.array_equal(comp["us"], r["votes"])
    # the order of the views does not matter
    perm = [3, 0, 5, 1, 4, 2]
    rp = ov.vote(pts, [cams[i] for i in perm], [masks[i] for i in perm], tau=2)
    for k in ("votes", "us", "flags"):
        assert np.array_equal(rp[k], r[k])
    # flags follow Eq. 6 and the tolerance
    assert np.array_equal(r["flags"] & 1, (r["votes"] > 0).astype(np.uint8))
    assert np.array_equal(r["flags"] >> 1, ((r["votes"] > 0) & (r["us"] < 2)).astype(np.uint8))


def test_filter_separates_building_points_on_the_survey_stand_in():
    """On the synthetic survey the building points keep consistent votes
    across views and the ground and clutter points mostly do not (those
    that stay reliable sit where buildings hide them, inside silhouettes,
    from every view but one): almost every building point that some view
    sees is reliable, and at most about a third of the others are."""
    s = sv.vote_small(seed=61)
    r = ov.vote(s.points, s.cameras, s.masks, tau=2)
    rel = (r["flags"] & 2) != 0
    seen = (r["votes"] + r["us"]) > 0
    building = (s.kind == 0) & seen
    other = (s.kind != 0) & seen
    assert building.sum() > 10000 and other.sum() > 5000
    assert rel[building].mean() > 0.99
    assert rel[other].mean() < 0.4
