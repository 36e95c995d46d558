"""Tie-aware comparison of the HIP path against the FP64 oracle.

Bars (the stated tolerance of the FP32 path): |d - phi| <= 1e-5 m; gradient
||dg||_inf <= 1e-4 * max(1, ||g_ref||_inf); winning obstacle and edge
bit-exact when the oracle's minimum is unique within TAU, otherwise inside
the oracle's tie set (every candidate within TAU of the minimum).  Where the
GPU picked a different member of a tie set, the gradient is compared with the
oracle's gradient for the GPU's choice (any active branch is a valid
subgradient, Sec. IV-D).
"""
import numpy as np

import oracle

D_TOL = 1e-5
G_RTOL = 1e-4
TAU = 2e-5


def check_stages(footprint, poses, edges, obst_off, eta, d, edge, obst, grad=None, stages=None,
                 eps=1e-12, eps_sat=1e-6, gscale=None):
    """Compare per-stage GPU outputs (numpy) with the oracle; returns counters."""
    poses = np.asarray(poses)
    N = poses.shape[0]
    stages = np.arange(N) if stages is None else np.asarray(stages)
    sub = poses[stages]
    ref = oracle.psdf(footprint, sub, edges, obst_off, eps=eps, eps_sat=eps_sat, eta=eta)
    sdm = oracle.sd_matrix(footprint, sub, edges, obst_off, eps=eps, eps_sat=eps_sat, eta=eta)
    stats = dict(stages=0, obst_ties=0, edge_ties=0, pen=int(ref["pen"].sum()))
    for r, s in enumerate(stages):
        phi = ref["phi"][r]
        ctx = f"stage {s}: gpu d={d[s]!r} obst={obst[s]} edge={edge[s]}; oracle phi={phi!r} obst={ref['obst'][r]} edge={ref['edge'][r]}"
        if np.isnan(phi):
            assert np.isnan(d[s]) and obst[s] == -1 and edge[s] == -1, ctx
            continue
        if np.isinf(phi):
            assert np.isinf(d[s]) and d[s] > 0 and obst[s] == -1 and edge[s] == -1, ctx
            if grad is not None:
                assert np.all(grad[s] == 0), ctx
            continue
        assert abs(float(d[s]) - phi) <= D_TOL, ctx
        ties = np.flatnonzero(sdm[r] <= phi + TAU)
        assert obst[s] in ties, ctx
        if len(ties) == 1:
            assert obst[s] == ref["obst"][r], ctx
        else:
            stats["obst_ties"] += 1
        i = int(obst[s])
        e0, e1 = int(obst_off[i]), int(obst_off[i + 1])
        det = oracle.obstacle(footprint, poses[s], edges[e0:e1], eps=eps, eps_sat=eps_sat, eta=eta)
        pool = det["edge_pool"]
        eties = e0 + np.flatnonzero(pool <= pool.min() + TAU)
        assert edge[s] in eties, ctx + f" edge ties {eties}"
        if len(eties) > 1:
            stats["edge_ties"] += 1
        elif i == ref["obst"][r]:
            assert edge[s] == ref["edge"][r], ctx
        if grad is not None:
            gref = det["grad"] * (1.0 if gscale is None else gscale[s])
            tol = G_RTOL * max(1.0, float(np.abs(gref).max()))
            assert np.abs(grad[s] - gref).max() <= tol, ctx + f" grad {grad[s]} vs {gref}"
        stats["stages"] += 1
    return stats
