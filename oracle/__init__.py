"""FP64 CPU oracle of the PSDF (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it and shares no code with it.

``psdf_oracle.cpp`` holds the arithmetic (the paper's four-stage pipeline,
Sec. IV); this module only compiles it with g++ and marshals numpy arrays.
``textbook.py`` holds independent checks of that arithmetic (Minkowski
difference signed distance, dense boundary sampling) used to pin the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psdf_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

DEFAULT_EPS = 1e-12
DEFAULT_EPS_SAT = 1e-6
DEFAULT_ETA = 1000.0


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O3, OpenMP) into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["g++", "-O3", "-ffp-contract=off", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
               _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def use_native_build(directory=None) -> str:
    """Compile the oracle for the host it runs on (g++ -O3 -march=native,
    OpenMP, no contraction of multiplies and adds) into ``directory`` (a
    temporary directory by default) and load that build in place of
    ``liboracle.so`` for the rest of the process: the CPU-baseline timing
    uses it.  Same source, same arithmetic."""
    global _lib, _LIB_PATH
    import tempfile
    directory = directory or tempfile.mkdtemp(prefix="psdf_oracle_")
    path = os.path.join(directory, "liboracle_native.so")
    cmd = ["g++", "-O3", "-march=native", "-ffp-contract=off", "-std=c++17", "-fopenmp",
           "-shared", "-fPIC", _SRC, "-o", path]
    subprocess.run(cmd, check=True)
    _lib = None
    _LIB_PATH = path
    return path


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            if os.path.dirname(_LIB_PATH) != _HERE:
                raise RuntimeError(f"{_LIB_PATH} is missing or older than {_SRC}")
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_psdf.restype = ctypes.c_int
        lib.oracle_psdf.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int, dp, dp, dp, dp, ip,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, dp, ip, ip, dp, ip, ctypes.c_int]
        lib.oracle_obstacle.restype = None
        lib.oracle_obstacle.argtypes = [dp, ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        dp, ip, dp, dp, dp]
        lib.oracle_obstacle_selections.restype = ctypes.c_int
        lib.oracle_obstacle_selections.argtypes = [dp, ctypes.c_int, dp, dp, dp, dp, dp,
                                                   ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                   ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                   ctypes.c_int, ctypes.c_int, dp, dp, dp,
                                                   ctypes.POINTER(ctypes.c_int64), ip]
        lib.oracle_obstacle_axes.restype = ctypes.c_int
        lib.oracle_obstacle_axes.argtypes = [dp, ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             dp, ip]
        lib.oracle_obstacle_geom_grad.restype = None
        lib.oracle_obstacle_geom_grad.argtypes = [dp, ctypes.c_int, dp, dp, dp, dp, dp,
                                                  ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                  ctypes.c_double, dp, dp]
        lib.oracle_sd_matrix.restype = None
        lib.oracle_sd_matrix.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int, dp, dp, dp, dp, ip,
                                         ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, dp, ctypes.c_int]
        _lib = lib
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def psdf(footprint, poses, edges, obst_off, eps=DEFAULT_EPS, eps_sat=DEFAULT_EPS_SAT,
         eta=DEFAULT_ETA, nthreads=0):
    """PSDF value, winning obstacle/edge, gradient and branch flag per stage.

    footprint: (m, 2); poses: (N, 3); edges: (E, 4) rows (ax, ay, bx, by);
    obst_off: (M + 1,) CSR offsets.  Inputs are promoted to float64.
    Returns dict(phi, obst, edge, grad, pen, threads).
    """
    lib = _load()
    fp, fpp = _d(footprint)
    ps, psp = _d(poses)
    ed = np.ascontiguousarray(edges, dtype=np.float64).reshape(-1, 4)
    cols = [_d(ed[:, k]) for k in range(4)]
    off, offp = _i(obst_off)
    N = ps.shape[0]
    M = off.shape[0] - 1
    phi, phip = _d(np.zeros(N))
    grad, gradp = _d(np.zeros((N, 3)))
    obst, obstp = _i(np.zeros(N))
    edge, edgep = _i(np.zeros(N))
    pen, penp = _i(np.zeros(N))
    used = lib.oracle_psdf(fpp, fp.shape[0], psp, N, cols[0][1], cols[1][1], cols[2][1],
                           cols[3][1], offp, M, eps, eps_sat, eta, phip, obstp, edgep, gradp,
                           penp, int(nthreads))
    return dict(phi=phi, obst=obst, edge=edge, grad=grad, pen=pen, threads=used)


def obstacle(footprint, pose, edges, eps=DEFAULT_EPS, eps_sat=DEFAULT_EPS_SAT, eta=DEFAULT_ETA):
    """sd, separated flag, d_sep, per-edge pool distance and gradient for one
    (pose, obstacle); ``edges`` are the obstacle's (mi, 4) edges."""
    lib = _load()
    fp, fpp = _d(footprint)
    ps, psp = _d(pose)
    ed = np.ascontiguousarray(edges, dtype=np.float64).reshape(-1, 4)
    mi = ed.shape[0]
    cols = [_d(ed[:, k]) for k in range(4)]
    sd, sdp = _d(np.zeros(1))
    sep, sepp = _i(np.zeros(1))
    dsep, dsepp = _d(np.zeros(1))
    pool, poolp = _d(np.zeros(max(mi, 1)))
    grad, gradp = _d(np.zeros(3))
    lib.oracle_obstacle(fpp, fp.shape[0], psp, cols[0][1], cols[1][1], cols[2][1], cols[3][1],
                        mi, eps, eps_sat, eta, sdp, sepp, dsepp, poolp, gradp)
    return dict(sd=float(sd[0]), separated=bool(sep[0]), d_sep=float(dsep[0]),
                edge_pool=pool[:mi].copy(), grad=grad.copy())


def selection_grads(footprint, pose, edges, eps=DEFAULT_EPS, eps_sat=DEFAULT_EPS_SAT,
                    eta=DEFAULT_ETA, tol=0.0, probe=-1, max_out=4096, samples=20000):
    """Active-branch pose gradients of sd for one (pose, obstacle) (Sec. IV-D):
    each min / max attained by several entries within ``tol`` and each ReLU
    within ``tol`` of its kink takes one active branch; every combination of
    the kinks that matter is visited up to 65536 of them, else ``samples``
    random ones.  With probe = q >= 0 the quantity is axis q's term
    max(delta(n_q), 0) instead of sd.  Returns dict(grads (k, 3) distinct
    gradients, first (3,) the gradient with the first active entry at every
    kink, mean (3,) the default-convention average (NaN when sampled),
    combos, sampled)."""
    lib = _load()
    fp, fpp = _d(footprint)
    ps, psp = _d(pose)
    ed = np.ascontiguousarray(edges, dtype=np.float64).reshape(-1, 4)
    mi = ed.shape[0]
    cols = [_d(ed[:, k]) for k in range(4)]
    out, outp = _d(np.zeros((max_out, 3)))
    first, firstp = _d(np.zeros(3))
    mean, meanp = _d(np.zeros(3))
    combos = ctypes.c_int64(0)
    sampled = ctypes.c_int32(0)
    n = lib.oracle_obstacle_selections(fpp, fp.shape[0], psp, cols[0][1], cols[1][1], cols[2][1],
                                       cols[3][1], mi, eps, eps_sat, eta, float(tol), int(probe),
                                       max_out, int(samples), outp, firstp, meanp,
                                       ctypes.byref(combos), ctypes.byref(sampled))
    return dict(grads=out[:n].copy(), first=first.copy(), mean=mean.copy(),
                combos=int(combos.value), sampled=bool(sampled.value))


def branch_sets(footprint, pose, edges, eps=DEFAULT_EPS, eps_sat=DEFAULT_EPS_SAT, eta=DEFAULT_ETA,
                tol=0.0):
    """The structure of sd's active-branch gradients for one (pose,
    obstacle), for the subgradient check of Sec. IV-D.

    Separated (Sec. IV-C test): sd = d_sep and the gradients are
    selection_grads of sd itself: terms = [(1.0, S)], mode "sum".
    Penetration: sd = -depth.  With the soft-min, grad sd = -sum_q w_q
    grad max(delta_q, 0), w = softmax(-eta max(delta, 0)), each axis's term
    having its own active-branch set S_q: terms = [(-w_q, S_q)], mode "sum"
    (every choice of one member per term).  With the hard minimum, grad sd
    = -grad of one axis term attaining the minimum (within tol): terms =
    [(-1, S_q)] over those axes, mode "union".  Axes with weight below 1e-16
    are dropped."""
    lib = _load()
    fp, fpp = _d(footprint)
    ps, psp = _d(pose)
    ed = np.ascontiguousarray(edges, dtype=np.float64).reshape(-1, 4)
    mi = ed.shape[0]
    cols = [_d(ed[:, k]) for k in range(4)]
    m = fp.shape[0]
    dp_, dpp = _d(np.zeros(m + mi))
    sep = ctypes.c_int32(0)
    K = lib.oracle_obstacle_axes(fpp, m, psp, cols[0][1], cols[1][1], cols[2][1], cols[3][1], mi,
                                 eps, eps_sat, eta, dpp, ctypes.byref(sep))
    if sep.value:
        return dict(separated=True, mode="sum",
                    terms=[(1.0, selection_grads(footprint, pose, edges, eps, eps_sat, eta,
                                                 tol=tol)["grads"])])
    dplus = dp_[:K].copy()
    hard = not (eta > 0) or np.isinf(eta)
    mu = dplus.min()
    if hard:
        axes = np.flatnonzero(dplus <= mu + tol)
        wts = {int(q): -1.0 for q in axes}
    else:
        e = np.exp(-eta * (dplus - mu))
        w = e / e.sum()
        wts = {int(q): -float(w[q]) for q in range(K) if w[q] > 1e-16}
    terms = [(wq, selection_grads(footprint, pose, edges, eps, eps_sat, eta, tol=tol,
                                  probe=q)["grads"]) for q, wq in wts.items()]
    return dict(separated=False, mode="union" if hard else "sum", terms=terms, dplus=dplus)


def geom_grad(footprint, pose, edges, eps=DEFAULT_EPS, eps_sat=DEFAULT_EPS_SAT, eta=DEFAULT_ETA):
    """d sd / d(geometry) for one (pose, obstacle): ``edges`` (mi, 4) of
    (A_x, A_y, B_x, B_y) -> (g_edges (mi, 4), g_fp (m, 2) in the caller's
    vertex order)."""
    lib = _load()
    fp, fpp = _d(footprint)
    ps, psp = _d(pose)
    ed = np.ascontiguousarray(edges, dtype=np.float64).reshape(-1, 4)
    mi = ed.shape[0]
    cols = [_d(ed[:, k]) for k in range(4)]
    ge, gep = _d(np.zeros((mi, 4)))
    gf, gfp = _d(np.zeros((fp.shape[0], 2)))
    lib.oracle_obstacle_geom_grad(fpp, fp.shape[0], psp, cols[0][1], cols[1][1], cols[2][1],
                                  cols[3][1], mi, eps, eps_sat, eta, gep, gfp)
    return ge.copy(), gf.copy()


def psdf_geom(footprint, poses, edges, obst_off, gout, eps=DEFAULT_EPS, eps_sat=DEFAULT_EPS_SAT,
              eta=DEFAULT_ETA):
    """Vector-Jacobian product of phi with respect to the geometry:
    sum over stages of gout[s] * d phi_s / d(edges) -> (E, 4), and
    / d(footprint vertices) -> (m, 2), through each stage's winning obstacle
    (lowest index on ties).  Stages with no obstacle contribute nothing."""
    ed = np.asarray(edges, dtype=np.float64).reshape(-1, 4)
    off = np.asarray(obst_off)
    ref = psdf(footprint, poses, edges, obst_off, eps=eps, eps_sat=eps_sat, eta=eta)
    gE = np.zeros_like(ed)
    gF = np.zeros((np.asarray(footprint).reshape(-1, 2).shape[0], 2))
    for s in range(len(poses)):
        i = int(ref["obst"][s])
        if i < 0:
            continue
        a, b = int(off[i]), int(off[i + 1])
        ge, gf = geom_grad(footprint, poses[s], ed[a:b], eps=eps, eps_sat=eps_sat, eta=eta)
        gE[a:b] += gout[s] * ge
        gF += gout[s] * gf
    return gE, gF


def sd_matrix(footprint, poses, edges, obst_off, eps=DEFAULT_EPS, eps_sat=DEFAULT_EPS_SAT,
              eta=DEFAULT_ETA, nthreads=0):
    """sd^i for every (stage, obstacle), shape (N, M)."""
    lib = _load()
    fp, fpp = _d(footprint)
    ps, psp = _d(poses)
    ed = np.ascontiguousarray(edges, dtype=np.float64).reshape(-1, 4)
    cols = [_d(ed[:, k]) for k in range(4)]
    off, offp = _i(obst_off)
    N, M = ps.shape[0], off.shape[0] - 1
    out, outp = _d(np.zeros((N, M)))
    lib.oracle_sd_matrix(fpp, fp.shape[0], psp, N, cols[0][1], cols[1][1], cols[2][1],
                         cols[3][1], offp, M, eps, eps_sat, eta, outp, int(nthreads))
    return out
