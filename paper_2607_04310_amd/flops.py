"""Algorithmic work model of the PSDF pipeline, used for roofline figures.

Counts the floating-point operations the method needs per (stage, obstacle)
in the separated branch of the paper's pipeline (Sec. IV-A..IV-D), an FMA
counting as 2 FLOP and min / max / clamp / compare / select as 0; square roots
and reciprocals are counted apart as transcendental ops.  The soft-min
(only reached by non-separated pairs) is not counted, so the figure is a
lower bound of the work per pair.

For a footprint of m vertices and an obstacle of mi edges and ni vertices in
V_obs (ni = mi for a closed polygon, 2 * mi for open chains, 2 for a free
segment):
    transform of ni vertices                  8 ni
    edge vectors and |v|^2 + eps              6 mi
    point-segment pairs, 13 FLOP each         13 (m mi + ni m)
    obstacle axes n' = rot90(v)/(|v| + eps)   3 mi
    projections, 3 FLOP each                  3 (m mi + ni m + ni mi)
    overlaps (two differences per axis)       2 (m + mi)
Rectangle (mi = ni = 4): m = 4 -> 644 FLOP (161 per edge); m = 6 -> 904 (226).

Memory: the edges are read once per work-group as 16 B per edge (ax, ay, bx,
by float32) plus 4 B per obstacle offset; poses 12 B per stage; outputs and
keys 32 B per stage.
"""
from __future__ import annotations

import numpy as np


def flops_pair(m: int, mi: int, ni: int) -> int:
    return (8 * ni + 6 * mi + 13 * (m * mi + ni * m) + 3 * mi
            + 3 * (m * mi + ni * m + ni * mi) + 2 * (m + mi))


def obstacle_shapes(edges, obst_off):
    """(mi, ni) for every obstacle of a CSR edge set."""
    e = np.asarray(edges, dtype=np.float32).reshape(-1, 4)
    off = np.asarray(obst_off)
    out = []
    for i in range(len(off) - 1):
        a, b = int(off[i]), int(off[i + 1])
        mi = b - a
        if mi == 0:
            continue
        nxt = np.roll(e[a:b, :2], -1, axis=0)
        closed = mi >= 3 and np.array_equal(e[a:b, 2:].view(np.uint32), nxt.view(np.uint32))
        out.append((mi, mi if closed else 2 * mi))
    return out


def flops_instance(m: int, N: int, edges, obst_off) -> float:
    """Algorithmic FLOP of one evaluation of N stages against an edge set."""
    shapes = obstacle_shapes(edges, obst_off)
    per_stage = sum(flops_pair(m, mi, ni) for mi, ni in shapes)
    return float(N) * float(per_stage)


def bytes_instance(N: int, E: int, M: int, work_groups_per_obstacle: int = 1) -> float:
    """Algorithmic HBM bytes of one evaluation: every edge and offset read
    once (per stage block), poses read, per-stage outputs written."""
    return float(work_groups_per_obstacle * (16 * E + 4 * (M + 1)) + 12 * N + 32 * N)
