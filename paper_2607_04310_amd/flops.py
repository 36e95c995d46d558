"""Algorithmic work model of the PSDF pipeline, used for roofline figures.

Counts the floating-point operations of the paper's pipeline (Sec. IV-A..IV-D)
per (stage, obstacle), an FMA counting as 2 FLOP and min / max / clamp /
compare / select as 0; square roots, reciprocals, exponentials and the
logarithm are counted apart as transcendental ops.  For a footprint of m
vertices and an obstacle of mi edges and ni points in V_obs (ni = mi for a
closed polygon, 2 mi for an open chain, 2 for a free segment):
    transform of the ni obstacle points                         8 ni
    edge vectors and |v|^2 + eps                                6 mi
    point-segment pairs, 13 FLOP each                           13 (m mi + m ni)
    projections of the obstacle points on the robot axes        3 m ni
    robot-side constants                                        2 m
    obstacle axes and the projections on them                   mi (5 + 3 m + 3 ni)
    overlaps and the separated test                             3 (m + mi)
    the final selection                                         1
A closed polygon gives 32 m mi + 3 mi^2 + 22 mi + 5 m + 1 (a rectangle:
935 FLOP at m = 6, 669 at m = 4), a free segment 37 + 53 m.

Memory: the edges are read once per work-group as 16 B per edge (ax, ay, bx,
by float32) plus 4 B per obstacle offset; poses 12 B per stage; outputs and
keys 32 B per stage.
"""
from __future__ import annotations

import numpy as np


def flops_pair(m: int, mi: int, ni: int) -> int:
    return (8 * ni + 6 * mi + 13 * (m * mi + m * ni) + 3 * m * ni + 2 * m
            + mi * (5 + 3 * m + 3 * ni) + 3 * (m + mi) + 1)


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
