"""Pins of the oracle's geometry gradient (d phi / d edge endpoints and
d phi / d footprint vertices), independent of the code that computes it:
central finite differences of the oracle's value, and the identities that
rigid motions impose (Sec. IV-A: phi depends on the pose and the geometry
only through R^T (A - p) and the footprint in its own frame)."""
import numpy as np
import pytest

import oracle
from paper_2607_04310_amd import inputs


def _convex(rng, k, r, c):
    ang = np.sort(rng.uniform(0, 2 * np.pi, k))
    pts = c + r * np.stack([np.cos(ang), 0.8 * np.sin(ang)], 1)
    return inputs._hull_ccw(pts.astype(np.float32)).astype(np.float64)


def _polygon_edges(pts):
    return np.concatenate([pts, np.roll(pts, -1, 0)], 1)


def _points(E, closed):
    """Unique points of an obstacle and, per point, the (edge, column) copies."""
    if closed:
        mi = E.shape[0]
        return [E[k, :2] for k in range(mi)], [[(k, 0), ((k - 1) % mi, 2)] for k in range(mi)]
    pts, copies = [], []
    for j in range(E.shape[0]):
        pts += [E[j, :2], E[j, 2:]]
        copies += [[(j, 0)], [(j, 2)]]
    return pts, copies


def _cases(seed):
    rng = np.random.default_rng(seed)
    fp = _convex(rng, int(rng.integers(3, 9)), 0.35, np.array([0.02, -0.01]))
    if seed % 2:
        fp = fp[::-1].copy()          # clockwise input
    out = []
    for closed in (True, False):
        if closed:
            E = _polygon_edges(_convex(rng, int(rng.integers(3, 9)), rng.uniform(0.2, 0.6),
                                       rng.uniform(-0.5, 0.5, 2)))
        else:
            a = rng.uniform(-0.6, 0.6, 2)
            E = np.concatenate([a, a + rng.uniform(-1, 1, 2)])[None, :]
        for _ in range(4):
            pose = np.array([*rng.uniform(-0.8, 0.8, 2), rng.uniform(-np.pi, np.pi)])
            out.append((fp, pose, E, closed))
    return out


def _sd(fp, pose, E, eta):
    return oracle.obstacle(fp, pose, E, eta=eta)["sd"]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("eta", [1000.0, np.inf])
def test_geom_grad_matches_finite_differences(seed, eta):
    h = 1e-6
    seen = set()
    for fp, pose, E, closed in _cases(seed):
        det = oracle.obstacle(fp, pose, E, eta=eta)
        seen.add(det["separated"])
        ge, gf = oracle.geom_grad(fp, pose, E, eta=eta)
        scale = max(1.0, np.abs(ge).max(), np.abs(gf).max())
        pts, copies = _points(E, closed)
        for p, cp in zip(pts, copies):
            g = sum(ge[j, c:c + 2] for j, c in cp)
            for r in range(2):
                Ep, Em = E.copy(), E.copy()
                for j, c in cp:
                    Ep[j, c + r] += h
                    Em[j, c + r] -= h
                fd = (_sd(fp, pose, Ep, eta) - _sd(fp, pose, Em, eta)) / (2 * h)
                assert abs(fd - g[r]) <= 2e-5 * scale, (closed, p, r, fd, g[r])
        for k in range(fp.shape[0]):
            for r in range(2):
                fpp, fpm = fp.copy(), fp.copy()
                fpp[k, r] += h
                fpm[k, r] -= h
                fd = (_sd(fpp, pose, E, eta) - _sd(fpm, pose, E, eta)) / (2 * h)
                assert abs(fd - gf[k, r]) <= 2e-5 * scale, (k, r, fd, gf[k, r])
    assert seen == {True, False}


def _rigid_identities(fp, pose, E, eta):
    """Residuals of the four identities (should all vanish):
    world translation  sum_points g + grad_p = 0,
    world rotation     sum_points rot90(P) . g + rot90(p) . grad_p + d_theta = 0,
    footprint shift    sum_k g_k - R^T grad_p = 0,
    footprint turn     sum_k rot90(v_k) . g_k - d_theta = 0."""
    det = oracle.obstacle(fp, pose, E, eta=eta)
    gp = det["grad"]
    ge, gf = oracle.geom_grad(fp, pose, E, eta=eta)
    rot = lambda v: np.array([-v[1], v[0]])
    c, s = np.cos(pose[2]), np.sin(pose[2])
    R = np.array([[c, -s], [s, c]])
    t1 = ge[:, 0:2].sum(0) + ge[:, 2:4].sum(0) + gp[:2]
    t2 = (sum(rot(E[j, 0:2]) @ ge[j, 0:2] + rot(E[j, 2:4]) @ ge[j, 2:4] for j in range(len(E)))
          + rot(pose[:2]) @ gp[:2] + gp[2])
    t3 = gf.sum(0) - R.T @ gp[:2]
    t4 = sum(rot(fp[k]) @ gf[k] for k in range(len(fp))) - gp[2]
    return np.concatenate([t1, [t2], t3, [t4]])


@pytest.mark.parametrize("eta", [1000.0, np.inf])
def test_geom_grad_rigid_motion_identities(eta):
    cases = []
    for seed in range(4):
        cases += _cases(100 + seed)
    inst = inputs.c1(0)           # rectangles: parallel-edge ties included
    ref = oracle.psdf(inst.footprint, inst.poses, inst.edges, inst.obst_off)
    for s in range(inst.N):
        i = int(ref["obst"][s])
        a, b = int(inst.obst_off[i]), int(inst.obst_off[i + 1])
        cases.append((inst.footprint.astype(np.float64), inst.poses[s].astype(np.float64),
                      inst.edges[a:b].astype(np.float64), True))
    for fp, pose, E, _ in cases:
        res = _rigid_identities(fp, pose, E, eta)
        assert np.abs(res).max() <= 1e-9, res


def test_geom_grad_accumulates_over_stages():
    inst = inputs.c1(1)
    gout = np.random.default_rng(3).normal(size=inst.N)
    gE, gF = oracle.psdf_geom(inst.footprint, inst.poses, inst.edges, inst.obst_off, gout)
    ref = oracle.psdf(inst.footprint, inst.poses, inst.edges, inst.obst_off)
    # translation identity summed over stages
    assert np.allclose(gE[:, :2].sum(0) + gE[:, 2:].sum(0), -(gout[:, None] * ref["grad"][:, :2]).sum(0),
                       atol=1e-9)
    # edges of obstacles that never win get nothing
    winners = set(ref["obst"].tolist())
    for i in range(inst.M):
        if i not in winners:
            assert not gE[inst.obst_off[i]:inst.obst_off[i + 1]].any()
