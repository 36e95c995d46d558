"""Textbook signed distance between convex polygons (test infrastructure only).

These routines pin the oracle to geometry that does not come from the PSDF
pipeline:

* ``minkowski_sd`` - sd = dist - pen of Sec. III-B computed through the
  Minkowski difference D = P - P0 = {q - r}: the sets intersect iff the origin
  lies in D; dist(P0, P) is the distance from the origin to D, and pen(P0, P)
  is the distance from the origin to the boundary of D when it lies inside.
  The convex hull comes from scipy (Qhull), not from any code of the oracle.
* ``sampled_dist`` - brute force minimum distance between densely sampled
  polygon boundaries (an upper bound within the sampling spacing).
* ``support_pen`` - penetration depth as min over dense unit directions u of
  h_P(u) + h_P0(-u) (support functions), i.e. the smallest translation that
  separates two overlapping convex sets.

All arithmetic is float64 numpy.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import ConvexHull


def place(footprint, pose):
    """World coordinates of the footprint vertices at pose (x, y, theta)."""
    fp = np.asarray(footprint, dtype=np.float64)
    x, y, th = (float(v) for v in pose)
    c, s = np.cos(th), np.sin(th)
    rot = np.array([[c, -s], [s, c]])
    return fp @ rot.T + np.array([x, y])


def hull_ccw(points):
    """Vertices of the convex hull of ``points`` in counter-clockwise order."""
    pts = np.asarray(points, dtype=np.float64)
    h = ConvexHull(pts)
    return pts[h.vertices]  # Qhull returns 2-D hull vertices counter-clockwise


def _point_segment_distance(o, a, b):
    ab = b - a
    t = np.clip(np.dot(o - a, ab) / np.dot(ab, ab), 0.0, 1.0)
    return float(np.linalg.norm(o - (a + t * ab)))


def minkowski_sd(robot_world, obstacle_pts):
    """Signed distance sd = dist - pen between conv(robot) and conv(obstacle)."""
    r = np.asarray(robot_world, dtype=np.float64)
    q = np.asarray(obstacle_pts, dtype=np.float64)
    diff = (q[:, None, :] - r[None, :, :]).reshape(-1, 2)
    D = hull_ccw(diff)
    n = len(D)
    o = np.zeros(2)
    boundary = min(_point_segment_distance(o, D[k], D[(k + 1) % n]) for k in range(n))
    # The origin is inside the CCW polygon D iff it is left of (or on) every edge.
    inside = all((D[(k + 1) % n][0] - D[k][0]) * (o[1] - D[k][1])
                 - (D[(k + 1) % n][1] - D[k][1]) * (o[0] - D[k][0]) >= 0 for k in range(n))
    return -boundary if inside else boundary


def _sample_boundary(poly, closed, h):
    poly = np.asarray(poly, dtype=np.float64)
    n = len(poly)
    segs = [(poly[k], poly[(k + 1) % n]) for k in range(n if closed else n - 1)]
    out = []
    for a, b in segs:
        k = max(2, int(np.ceil(np.linalg.norm(b - a) / h)) + 1)
        t = np.linspace(0.0, 1.0, k)[:, None]
        out.append(a + t * (b - a))
    return np.concatenate(out)


def sampled_dist(robot_world, obstacle_pts, obstacle_closed=True, h=1e-3):
    """Min distance between boundaries sampled at spacing <= h (brute force)."""
    a = _sample_boundary(robot_world, True, h)
    b = _sample_boundary(obstacle_pts, obstacle_closed, h)
    best = np.inf
    for k in range(0, len(a), 2048):
        d2 = ((a[k:k + 2048, None, :] - b[None, :, :]) ** 2).sum(-1)
        best = min(best, float(d2.min()))
    return float(np.sqrt(best))


def support_pen(robot_world, obstacle_pts, n_dirs=20000, refine=4):
    """min over unit u of h_P(u) + h_P0(-u): the penetration depth of two
    overlapping convex sets (negative when they are disjoint).  A coarse grid
    of directions is refined ``refine`` times around its minimiser; each
    level shrinks the angular step (and the error, which is of order
    |D| * step) by a factor n_dirs / 4."""
    r = np.asarray(robot_world, dtype=np.float64)
    q = np.asarray(obstacle_pts, dtype=np.float64)

    def h(ang):
        u = np.stack([np.cos(ang), np.sin(ang)], axis=1)
        return (q @ u.T).max(axis=0) + (-(r @ u.T)).max(axis=0)

    ang = np.linspace(0.0, 2.0 * np.pi, n_dirs, endpoint=False)
    step = 2.0 * np.pi / n_dirs
    vals = h(ang)
    best = float(vals.min())
    centre = ang[int(vals.argmin())]
    for _ in range(refine):
        ang = centre + np.linspace(-2.0 * step, 2.0 * step, n_dirs)
        vals = h(ang)
        k = int(vals.argmin())
        best = min(best, float(vals[k]))
        centre, step = ang[k], 4.0 * step / n_dirs
    return best
