"""Pin the oracle to textbook geometry that does not come from the PSDF
pipeline: with eta -> inf, eps = 0 and eps_sat = 0 the PSDF of one convex
obstacle equals sd = dist - pen of Sec. III-B, computed here through the
Minkowski difference (oracle/textbook.py), dense boundary sampling and the
support-function penetration depth."""
import math

import numpy as np
import pytest

import oracle
from oracle import textbook
from paper_2607_04310_amd import inputs

HARD = dict(eps=0.0, eps_sat=0.0, eta=math.inf)


def _random_case(rng, kind):
    m = int(rng.integers(3, 9))
    fp = inputs.random_convex_footprint(rng, m)
    if rng.random() < 0.3:
        fp = fp[::-1].copy()                      # CW footprints are accepted too
    if kind == "rect":
        edges = inputs.random_rects(rng, 1, 0.1, 1.2, -0.8, 0.8)
    elif kind == "segment":
        edges = inputs.segment_edges(rng.uniform(-0.8, 0.8, (1, 2)), rng.uniform(0.1, 2.0, 1),
                                     rng.uniform(-np.pi, np.pi, 1))
    else:                                         # general convex polygon, either orientation
        poly = inputs._hull_ccw(rng.uniform(-0.7, 0.7, (int(rng.integers(3, 12)), 2)))
        poly = poly.astype(np.float32)
        if rng.random() < 0.5:
            poly = poly[::-1]
        edges = np.concatenate([poly, np.roll(poly, -1, axis=0)], axis=1)
    pose = inputs.uniform_poses(rng, 1, -1.2, 1.2)
    return fp, pose, edges.astype(np.float32)


def _textbook(fp, pose, edges):
    world = textbook.place(fp.astype(np.float64), pose[0].astype(np.float64))
    pts = np.concatenate([edges[:, :2], edges[:, 2:]], 0).astype(np.float64)
    return world, pts


@pytest.mark.parametrize("kind", ["rect", "segment", "poly"])
def test_minkowski_sd(kind):
    rng = np.random.default_rng(101 + ["rect", "segment", "poly"].index(kind))
    n_sep = n_pen = 0
    for _ in range(300):
        fp, pose, edges = _random_case(rng, kind)
        off = np.array([0, len(edges)], np.int32)
        r = oracle.psdf(fp, pose, edges, off, **HARD)
        world, pts = _textbook(fp, pose, edges)
        ref = textbook.minkowski_sd(world, pts)
        assert abs(r["phi"][0] - ref) <= 1e-9, (kind, r["phi"][0], ref)
        n_sep += ref > 0
        n_pen += ref < 0
    assert n_sep > 30 and n_pen > 30   # both branches exercised


def test_dense_sampling_distance():
    rng = np.random.default_rng(7)
    h = 2e-3
    checked = 0
    while checked < 25:
        kind = ["rect", "segment", "poly"][checked % 3]
        fp, pose, edges = _random_case(rng, kind)
        off = np.array([0, len(edges)], np.int32)
        r = oracle.psdf(fp, pose, edges, off, **HARD)
        if r["phi"][0] <= 0:
            continue
        world, _ = _textbook(fp, pose, edges)
        if kind == "segment":
            obst, closed = edges[0].reshape(2, 2).astype(np.float64), False
        else:
            obst, closed = edges[:, :2].astype(np.float64), True
        brute = textbook.sampled_dist(world, obst, closed, h)
        assert r["phi"][0] <= brute + 1e-12 and brute - r["phi"][0] <= h
        checked += 1


def test_support_function_penetration():
    rng = np.random.default_rng(8)
    checked = 0
    while checked < 40:
        fp, pose, edges = _random_case(rng, ["rect", "poly"][checked % 2])
        off = np.array([0, len(edges)], np.int32)
        r = oracle.psdf(fp, pose, edges, off, **HARD)
        if r["phi"][0] >= -1e-3:
            continue
        world, pts = _textbook(fp, pose, edges)
        pen = textbook.support_pen(world, pts)
        assert -r["phi"][0] <= pen + 1e-9 and pen - (-r["phi"][0]) <= 1e-6
        checked += 1


def test_gradient_matches_textbook_fd():
    """d/d(x, y, theta) of the oracle (hard-min) against central differences of
    the Minkowski-difference sd, away from feature switches."""
    rng = np.random.default_rng(9)
    h = 1e-6
    checked = 0
    while checked < 60:
        fp, pose, edges = _random_case(rng, ["rect", "segment", "poly"][checked % 3])
        pose = pose.astype(np.float64)
        off = np.array([0, len(edges)], np.int32)
        r = oracle.psdf(fp, pose, edges, off, **HARD)
        fd = np.zeros(3)
        smooth = True
        pts = np.concatenate([edges[:, :2], edges[:, 2:]], 0).astype(np.float64)
        f0 = textbook.minkowski_sd(textbook.place(fp, pose[0]), pts)
        for k in range(3):
            dp = np.zeros(3)
            dp[k] = h
            fp_ = textbook.minkowski_sd(textbook.place(fp, pose[0] + dp), pts)
            fm_ = textbook.minkowski_sd(textbook.place(fp, pose[0] - dp), pts)
            fd[k] = (fp_ - fm_) / (2 * h)
            # one-sided slopes disagree at a kink: skip such samples
            smooth &= abs((fp_ - f0) / h - (f0 - fm_) / h) < 1e-4
        if not smooth:
            continue
        np.testing.assert_allclose(r["grad"][0], fd, atol=2e-5)
        checked += 1


def test_reported_edge_is_nearest_segment():
    """For a separated winner, the reported edge is the obstacle edge nearest
    to the placed footprint (textbook distance of the footprint to each edge
    as a one-segment set), lowest index on ties."""
    checked = 0
    for seed in range(6):
        inst = inputs.c1(seed)
        r = oracle.psdf(inst.footprint, inst.poses, inst.edges, inst.obst_off, **HARD)
        for s in range(inst.N):
            if r["pen"][s]:
                continue
            i = r["obst"][s]
            e0, e1 = inst.obst_off[i], inst.obst_off[i + 1]
            world = textbook.place(inst.footprint, inst.poses[s])
            d = np.array([textbook.minkowski_sd(world, inst.edges[j].reshape(2, 2).astype(np.float64))
                          for j in range(e0, e1)])
            best = np.flatnonzero(d <= d.min() + 1e-12)
            assert r["edge"][s] == e0 + best[0]
            checked += 1
    assert checked > 10
