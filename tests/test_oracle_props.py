"""Properties the paper and the mathematics fix for the oracle: rigid-motion
invariance (Sec. IV-A: p cancels in every distance and overlap), invariance
to vertex order, obstacle order, padding (Sec. IV-A, S = 0 entries are
ignored), lowest-index tie rule (Sec. IV-D), the soft-min bracket
0 <= delta_hard - delta_soft <= ln|N^i| / eta (Sec. IV-C), unit translational
gradient when separated, and central finite differences of the value
(h = 1e-6) for the pose gradient, including penetrating stages."""
import math

import numpy as np

import oracle
from paper_2607_04310_amd import inputs


def _mixed(seed, n_obst=10, n_poses=24, segments=3):
    return inputs.random_small(np.random.default_rng(seed), n_obst=n_obst, n_poses=n_poses,
                               segments=segments, lo=-1.5, hi=1.5)


def _run(inst, **kw):
    return oracle.psdf(inst.footprint, inst.poses, inst.edges, inst.obst_off, **kw)


def test_rigid_motion_invariance():
    inst = _mixed(1)
    r0 = _run(inst)
    ang, t = 0.7, np.array([3.0, -2.0])
    c, s = math.cos(ang), math.sin(ang)
    Rg = np.array([[c, -s], [s, c]])
    e = inst.edges.astype(np.float64)
    e2 = np.concatenate([e[:, :2] @ Rg.T + t, e[:, 2:] @ Rg.T + t], 1)
    p = inst.poses.astype(np.float64)
    p2 = np.concatenate([p[:, :2] @ Rg.T + t, p[:, 2:] + ang], 1)
    r1 = oracle.psdf(inst.footprint, p2, e2, inst.obst_off)
    np.testing.assert_allclose(r1["phi"], r0["phi"], atol=1e-9)
    assert np.array_equal(r1["obst"], r0["obst"])
    np.testing.assert_allclose(r1["grad"][:, :2], r0["grad"][:, :2] @ Rg.T, atol=1e-6)
    np.testing.assert_allclose(r1["grad"][:, 2], r0["grad"][:, 2], atol=1e-6)


def test_footprint_and_obstacle_orientation():
    inst = _mixed(2, segments=0)
    r0 = _run(inst)
    r1 = oracle.psdf(inst.footprint[::-1].copy(), inst.poses, inst.edges, inst.obst_off)
    np.testing.assert_allclose(r1["phi"], r0["phi"], atol=1e-12)
    # reverse every rectangle: edges (B, A) in reverse order
    e = inst.edges.reshape(-1, 4, 4)[:, ::-1][:, :, [2, 3, 0, 1]].reshape(-1, 4)
    r2 = oracle.psdf(inst.footprint, inst.poses, e, inst.obst_off)
    np.testing.assert_allclose(r2["phi"], r0["phi"], atol=1e-12)
    np.testing.assert_allclose(r2["grad"], r0["grad"], atol=1e-9)


def test_obstacle_permutation_and_cyclic_edges():
    inst = _mixed(3, segments=0)
    r0 = _run(inst)
    M = inst.M
    perm = np.random.default_rng(0).permutation(M)
    e = inst.edges.reshape(M, 4, 4)[perm]
    e = np.roll(e, 1, axis=1).reshape(-1, 4)      # also rotate each rectangle's edge list
    r1 = oracle.psdf(inst.footprint, inst.poses, e, inst.obst_off)
    np.testing.assert_allclose(r1["phi"], r0["phi"], atol=1e-12)
    assert np.array_equal(perm[r1["obst"]], r0["obst"])


def test_padding_and_duplicates():
    inst = _mixed(4, segments=2)
    r0 = _run(inst)
    sizes = np.diff(inst.obst_off)
    # insert an empty obstacle (all-padding row) in front of every obstacle
    padded = np.concatenate([[0], np.cumsum(np.ravel(np.stack([np.zeros_like(sizes), sizes], 1)))])
    r1 = oracle.psdf(inst.footprint, inst.poses, inst.edges, padded.astype(np.int32))
    np.testing.assert_allclose(r1["phi"], r0["phi"], atol=0)
    assert np.array_equal(r1["obst"], 2 * r0["obst"] + 1)
    # duplicate the whole edge set: the lowest index wins every tie
    e2 = np.concatenate([inst.edges, inst.edges], 0)
    off2 = np.concatenate([inst.obst_off, inst.obst_off[1:] + inst.E]).astype(np.int32)
    r2 = oracle.psdf(inst.footprint, inst.poses, e2, off2)
    np.testing.assert_allclose(r2["phi"], r0["phi"], atol=0)
    assert np.array_equal(r2["obst"], r0["obst"]) and np.array_equal(r2["edge"], r0["edge"])


def test_soft_min_bracket():
    inst = _mixed(5, n_obst=16, n_poses=40)
    eta = 1000.0
    soft = oracle.sd_matrix(inst.footprint, inst.poses, inst.edges, inst.obst_off, eta=eta)
    hard = oracle.sd_matrix(inst.footprint, inst.poses, inst.edges, inst.obst_off, eta=math.inf)
    m = inst.footprint.shape[0]
    K = m + np.diff(inst.obst_off)[None, :]        # |N^i| = m robot axes + m_i obstacle axes
    diff = soft - hard
    pen = hard <= 0
    assert pen.sum() > 20
    assert np.all(diff[pen] >= -1e-12) and np.all(diff[pen] <= np.log(K + 0 * diff)[pen] / eta + 1e-12)
    np.testing.assert_array_equal(diff[~pen & (soft > 1e-2)], 0)


def test_unit_gradient_when_separated():
    n_sep = 0
    for seed in range(6):
        r = _run(inputs.c1(seed), eta=math.inf)
        sep = r["pen"] == 0
        n_sep += sep.sum()
        np.testing.assert_allclose(np.linalg.norm(r["grad"][sep, :2], axis=1), 1.0, atol=1e-9)
    assert n_sep > 10


def _fd_check(inst, eta, h=1e-6, tol=1e-5):
    r = _run(inst, eta=eta)
    poses = inst.poses.astype(np.float64)
    ok = 0
    for s in range(inst.N):
        fd = np.zeros(3)
        smooth = True
        f0 = r["phi"][s]
        for k in range(3):
            dp = np.zeros(3)
            dp[k] = h
            fp_ = oracle.psdf(inst.footprint, (poses[s] + dp)[None], inst.edges, inst.obst_off, eta=eta)["phi"][0]
            fm_ = oracle.psdf(inst.footprint, (poses[s] - dp)[None], inst.edges, inst.obst_off, eta=eta)["phi"][0]
            fd[k] = (fp_ - fm_) / (2 * h)
            smooth &= abs((fp_ - f0) / h - (f0 - fm_) / h) < 1e-4
        if smooth:
            np.testing.assert_allclose(r["grad"][s], fd, atol=tol, err_msg=f"stage {s}")
            ok += 1
    return ok, int(r["pen"].sum())


def test_finite_differences_c3_shapes():
    """Config 3 shapes: rectangle footprint, 64 rectangles, N = 20, with
    penetrating stages included."""
    for seed in range(3):
        ok, pen = _fd_check(inputs.c3(seed), 1000.0)
        assert ok >= 15


def test_finite_differences_penetration():
    inst = _mixed(11, n_obst=12, n_poses=40)
    ok, pen = _fd_check(inst, 1000.0)
    assert ok >= 30 and pen >= 10
    ok, pen = _fd_check(inst, 50.0)
    assert ok >= 30
