"""Tie-aware comparison of the HIP path against the FP64 oracle.

Bars (the stated tolerance of the FP32 path): |d - phi| <= 1e-5 m; gradient
||dg||_inf <= 1e-4 * max(1, ||g_ref||_inf); winning obstacle and edge
bit-exact when the oracle's minimum is unique within TAU, otherwise inside
the oracle's tie set (every candidate within TAU of the minimum).  Where the
GPU picked a different member of a tie set, the gradient is compared with the
oracle's gradient for the GPU's choice.  At a kink of that obstacle's
pipeline (a min / max with several active entries, a ReLU at zero) the GPU
takes one active branch where the oracle splits evenly; the gradient then
has to be one of the oracle's active-branch gradients (or in their convex
hull): any active branch is a valid subgradient (Sec. IV-D).
"""
import numpy as np

import oracle

D_TOL = 1e-5
G_RTOL = 1e-4
TAU = 2e-5
# kinks whose branches lie within this distance of each other count as ties
# when the oracle lists the active-branch gradients (FP32 rounding can move
# the GPU to any of them)
KINK_TOL = 1e-5


def in_hull(g, pts, tol):
    """True if g lies within tol (max norm) of the convex hull of pts (k, 3)."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    if len(pts) == 0:
        return False
    return in_branch_hull(g, dict(mode="union", terms=[(1.0, pts)]), tol)


def in_branch_hull(g, bs, tol):
    """True if g lies within tol (max norm) of the convex hull of the
    active-branch gradients described by oracle.branch_sets: mode "sum" is
    sum_t c_t conv(S_t) (one member per term), mode "union" conv(U_t c_t S_t)."""
    g = np.asarray(g, dtype=np.float64)
    terms = [(float(c), np.asarray(S, np.float64).reshape(-1, 3)) for c, S in bs["terms"]]
    if any(len(S) == 0 for _, S in terms):
        return False
    if bs["mode"] == "union":
        cols = np.concatenate([c * S for c, S in terms])
        groups = [np.arange(len(cols))]
    else:
        cols = np.concatenate([c * S for c, S in terms])
        sizes = [len(S) for _, S in terms]
        starts = np.concatenate([[0], np.cumsum(sizes)])
        groups = [np.arange(starts[t], starts[t + 1]) for t in range(len(terms))]
        if all(sz == 1 for sz in sizes):
            return bool(np.abs(cols.sum(axis=0) - g).max() <= tol)
    if len(groups) == 1 and np.abs(cols - g).max(axis=1).min() <= tol:
        return True
    from scipy.optimize import linprog
    n = len(cols)
    A_eq = np.zeros((len(groups), n))
    for t, idx in enumerate(groups):
        A_eq[t, idx] = 1.0
    A_ub = np.concatenate([cols.T, -cols.T])
    b_ub = np.concatenate([g + tol, -(g - tol)])
    res = linprog(np.zeros(n), A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=np.ones(len(groups)),
                  bounds=[(0, None)] * n, method="highs")
    return bool(res.status == 0)


def branch_directional_values(bs, d):
    """Every value <g, d> that one choice of active branches gives (sum
    mode: one member per term; union mode: any member of any term)."""
    d = np.asarray(d, dtype=np.float64)
    if bs["mode"] == "union":
        return np.unique(np.concatenate([c * (np.asarray(S).reshape(-1, 3) @ d)
                                         for c, S in bs["terms"]]))
    vals = np.zeros(1)
    for c, S in bs["terms"]:
        v = c * (np.asarray(S).reshape(-1, 3) @ d)
        vals = np.unique(np.round((vals[:, None] + v[None, :]).ravel(), 13))
    return vals


def grad_ok(g, footprint, pose, obst_edges, gref, tol, eps=1e-12, eps_sat=1e-6, eta=1000.0,
            scale=1.0):
    """The GPU gradient g of one stage against the oracle: equal to the
    oracle's gradient gref (even split at ties) within tol, or else within
    tol of the convex hull of the active-branch gradients at the stage's
    kinks (any active branch is a valid subgradient, Sec. IV-D)."""
    if np.abs(g - gref).max() <= tol:
        return True
    bs = oracle.branch_sets(footprint, pose, obst_edges, eps=eps, eps_sat=eps_sat, eta=eta,
                            tol=KINK_TOL)
    bs = dict(bs, terms=[(c * scale, S) for c, S in bs["terms"]])
    return in_branch_hull(np.asarray(g, np.float64), bs, tol)


def oracle_reference(footprint, poses, edges, obst_off, eta, stages=None, eps=1e-12, eps_sat=1e-6):
    """The oracle's per-stage results and sd matrix for the given stages
    (reusable by several check_stages calls on the same inputs)."""
    poses = np.asarray(poses)
    stages = np.arange(poses.shape[0]) if stages is None else np.asarray(stages)
    sub = poses[stages]
    return (oracle.psdf(footprint, sub, edges, obst_off, eps=eps, eps_sat=eps_sat, eta=eta),
            oracle.sd_matrix(footprint, sub, edges, obst_off, eps=eps, eps_sat=eps_sat, eta=eta))


def check_stages(footprint, poses, edges, obst_off, eta, d, edge, obst, grad=None, stages=None,
                 eps=1e-12, eps_sat=1e-6, gscale=None, reference=None):
    """Compare per-stage GPU outputs (numpy) with the oracle; returns counters.
    reference: oracle_reference(...) of the same stages, to reuse."""
    poses = np.asarray(poses)
    N = poses.shape[0]
    stages = np.arange(N) if stages is None else np.asarray(stages)
    if reference is None:
        reference = oracle_reference(footprint, poses, edges, obst_off, eta, stages, eps, eps_sat)
    ref, sdm = reference
    stats = dict(stages=0, obst_ties=0, edge_ties=0, kink_grads=0, pen=int(ref["pen"].sum()))
    for r, s in enumerate(stages):
        phi = ref["phi"][r]
        ev = -1 if edge is None else edge[s]
        ctx = f"stage {s}: gpu d={d[s]!r} obst={obst[s]} edge={ev}; oracle phi={phi!r} obst={ref['obst'][r]} edge={ref['edge'][r]}"
        if np.isnan(phi):
            assert np.isnan(d[s]) and obst[s] == -1 and ev == -1, ctx
            continue
        if np.isinf(phi):
            assert np.isinf(d[s]) and d[s] > 0 and obst[s] == -1 and ev == -1, ctx
            if grad is not None:
                assert np.all(grad[s] == 0), ctx
            continue
        assert abs(float(d[s]) - phi) <= D_TOL, ctx
        ties = np.flatnonzero(sdm[r] <= phi + TAU)
        assert obst[s] in ties, ctx
        if edge is None:   # the caller has no edge output (constraint rows)
            i = int(obst[s])
            e0, e1 = int(obst_off[i]), int(obst_off[i + 1])
            if grad is not None:
                det = oracle.obstacle(footprint, poses[s], edges[e0:e1], eps=eps, eps_sat=eps_sat,
                                      eta=eta)
                sc = 1.0 if gscale is None else float(gscale[s])
                gref = det["grad"] * sc
                tol = G_RTOL * max(1.0, float(np.abs(gref).max()))
                assert grad_ok(grad[s], footprint, poses[s], edges[e0:e1], gref, tol, eps=eps,
                               eps_sat=eps_sat, eta=eta, scale=sc), ctx + f" grad {grad[s]} vs {gref}"
            stats["stages"] += 1
            continue
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
            sc = 1.0 if gscale is None else float(gscale[s])
            gref = det["grad"] * sc
            tol = G_RTOL * max(1.0, float(np.abs(gref).max()))
            if np.abs(grad[s] - gref).max() > tol:
                assert grad_ok(grad[s], footprint, poses[s], edges[e0:e1], gref, tol, eps=eps,
                               eps_sat=eps_sat, eta=eta, scale=sc), \
                    ctx + f" grad {grad[s]} vs {gref}, not an active-branch gradient either"
                stats["kink_grads"] += 1
        stats["stages"] += 1
    return stats
