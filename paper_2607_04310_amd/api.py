"""Python API over the C ABI: device-resident edge sets and the PSDF calls.

Every function here allocates its output tensors with torch on the poses'
device and calls the library on torch's current stream; the arithmetic is
all in the HIP kernels.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from types import SimpleNamespace

import numpy as np
import torch

from . import _lib

DEFAULT_EPS = 1e-12
DEFAULT_EPS_SAT = 1e-6
DEFAULT_ETA = 1000.0


@dataclass
class Params:
    """Method constants (Sec. IV-B eps, Sec. IV-C eps_sat and eta; eta <= 0 or
    inf selects the hard minimum)."""
    eps: float = DEFAULT_EPS
    eps_sat: float = DEFAULT_EPS_SAT
    eta: float = DEFAULT_ETA

    def c(self):
        return _lib.PsdfParams(self.eps, self.eps_sat, self.eta)


class EdgeSet:
    """Obstacle boundary edges on the device: SoA float32 columns and int32 CSR
    offsets (obstacle i owns edges [obst_off[i], obst_off[i+1]))."""

    def __init__(self, edges, obst_off, mbar=None, device="cuda"):
        e = torch.as_tensor(np.asarray(edges, dtype=np.float32).reshape(-1, 4))
        off = torch.as_tensor(np.asarray(obst_off, dtype=np.int32))
        self.E = int(e.shape[0])
        self.M = int(off.shape[0] - 1)
        if mbar is None:
            sizes = np.diff(np.asarray(obst_off))
            mbar = int(max(1, sizes.max() if len(sizes) else 1))
        self.mbar = int(mbar)
        cols = e.t().contiguous().to(device)
        self.ax, self.ay, self.bx, self.by = (cols[k].contiguous() for k in range(4))
        self.obst_off = off.to(device).contiguous()

    @classmethod
    def from_device(cls, ax, ay, bx, by, obst_off, mbar):
        self = cls.__new__(cls)
        self.ax, self.ay, self.bx, self.by = ax, ay, bx, by
        self.obst_off = obst_off
        self.E = int(ax.numel())
        self.M = int(obst_off.numel() - 1)
        self.mbar = int(mbar)
        return self

    _staged = None   # ctypes PsdfStaged, while staged
    _table = None    # its device table

    def stage(self, params: Params | None = None):
        """Take the edge set's pose-independent constants once
        (psdf_stage_edges, Alg. 1 EncodeEdges): later calls with this EdgeSet
        read them from a device table.  Stage again after changing the edge
        tensors in place (the table is rewritten in place)."""
        params = params or Params()
        nbytes = int(_lib.lib().psdf_staged_bytes(self.M, self.mbar))
        # staging again rewrites the same table, so that graphs captured on
        # this edge set keep reading it
        table = self._table
        if table is None or table.numel() < max(nbytes, 16):
            table = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=self.ax.device)
        st = _lib.PsdfStaged()
        ec, pc = self._plain(), params.c()
        _lib.check(_lib.lib().psdf_stage_edges(ctypes.byref(ec), ctypes.byref(pc),
                                               table.data_ptr(), table.numel(),
                                               ctypes.byref(st), _lib.stream_handle()))
        self._table, self._staged = table, st
        return self

    def unstage(self):
        self._table = self._staged = None
        return self

    @property
    def staged(self):
        return self._staged is not None

    def _plain(self):
        return _lib.PsdfEdges(self.ax.data_ptr(), self.ay.data_ptr(), self.bx.data_ptr(),
                              self.by.data_ptr(), self.obst_off.data_ptr(), self.E, self.M,
                              self.mbar)

    def c(self):
        ec = self._plain()
        if self._staged is not None:
            ec.staged = ctypes.pointer(self._staged)
        return ec


def _fp(footprint):
    fp = np.ascontiguousarray(np.asarray(footprint, dtype=np.float32).reshape(-1, 2))
    return fp, fp.ctypes.data_as(ctypes.c_void_p), int(fp.shape[0])


def _poses(poses):
    assert poses.dtype == torch.float32 and poses.is_cuda and poses.dim() == 2 and poses.shape[1] == 3
    return poses.contiguous()


def workspace(N, M, device):
    """Scratch tensor for psdf_eval / psdf_grad of N stages and M obstacles."""
    nbytes = int(_lib.lib().psdf_workspace_bytes(int(N), int(M)))
    return torch.empty(max(nbytes, 8), dtype=torch.uint8, device=device)


def psdf_eval(footprint, poses, edges: EdgeSet, params: Params | None = None, ws=None):
    """phi, edge, obstacle and winner keys per stage (psdf_eval of the C ABI)."""
    params = params or Params()
    poses = _poses(poses)
    N = poses.shape[0]
    dev = poses.device
    d = torch.empty(N, dtype=torch.float32, device=dev)
    edge = torch.empty(N, dtype=torch.int32, device=dev)
    obst = torch.empty(N, dtype=torch.int32, device=dev)
    keys = torch.empty(N, dtype=torch.int64, device=dev)
    ws = workspace(N, edges.M, dev) if ws is None else ws
    fp, fpp, m = _fp(footprint)
    ec, pc = edges.c(), params.c()
    _lib.check(_lib.lib().psdf_eval(fpp, m, poses.data_ptr(), N, ctypes.byref(ec),
                                    ctypes.byref(pc), d.data_ptr(), edge.data_ptr(),
                                    obst.data_ptr(), keys.data_ptr(), ws.data_ptr(),
                                    ws.numel(), _lib.stream_handle()))
    return d, edge, obst, keys


def psdf_grad(footprint, poses, edges: EdgeSet, params: Params | None = None, out=None,
              ws=None):
    """phi, edge, obstacle, dphi/d(x, y, theta) and winner keys per stage."""
    params = params or Params()
    poses = _poses(poses)
    N = poses.shape[0]
    dev = poses.device
    if out is None:
        out = (torch.empty(N, dtype=torch.float32, device=dev),
               torch.empty(N, dtype=torch.int32, device=dev),
               torch.empty(N, dtype=torch.int32, device=dev),
               torch.empty((N, 3), dtype=torch.float32, device=dev),
               torch.empty(N, dtype=torch.int64, device=dev))
    d, edge, obst, grad, keys = out
    ws = workspace(N, edges.M, dev) if ws is None else ws
    fp, fpp, m = _fp(footprint)
    ec, pc = edges.c(), params.c()
    _lib.check(_lib.lib().psdf_grad(fpp, m, poses.data_ptr(), N, ctypes.byref(ec),
                                    ctypes.byref(pc), d.data_ptr(), edge.data_ptr(),
                                    obst.data_ptr(), grad.data_ptr(), keys.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _lib.stream_handle()))
    return d, edge, obst, grad, keys


def psdf_bwd(footprint, poses, edges: EdgeSet, keys, gout, params: Params | None = None):
    """gpose[s] = gout[s] * dphi_s/d(x, y, theta), from the keys of a psdf_eval."""
    params = params or Params()
    poses = _poses(poses)
    N = poses.shape[0]
    gout = gout.contiguous().to(torch.float32)
    gpose = torch.empty((N, 3), dtype=torch.float32, device=poses.device)
    fp, fpp, m = _fp(footprint)
    ec, pc = edges.c(), params.c()
    _lib.check(_lib.lib().psdf_bwd(fpp, m, poses.data_ptr(), N, ctypes.byref(ec),
                                   ctypes.byref(pc), keys.data_ptr(), gout.data_ptr(),
                                   gpose.data_ptr(), _lib.stream_handle()))
    return gpose


def psdf_constraints(footprint, poses, edges: EdgeSet, d_min, params: Params | None = None,
                     host=None, ws=None):
    """Linearised safety-constraint parameters per stage: (N, 4) rows
    (phi - d_min, -dphi/dx, -dphi/dy, -dphi/dtheta) on the device, plus the
    winner keys; with ``host`` (a pinned CPU float32 (N, 4) tensor) the rows
    are also copied there on the stream."""
    params = params or Params()
    poses = _poses(poses)
    N = poses.shape[0]
    dev = poses.device
    hj = torch.empty((N, 4), dtype=torch.float32, device=dev)
    keys = torch.empty(N, dtype=torch.int64, device=dev)
    ws = workspace(N, edges.M, dev) if ws is None else ws
    if host is not None and (host.dtype != torch.float32 or tuple(host.shape) != (N, 4)
                             or not host.is_contiguous() or host.is_cuda):
        raise ValueError("host must be a contiguous CPU float32 tensor of shape (N, 4)")
    fp, fpp, m = _fp(footprint)
    ec, pc = edges.c(), params.c()
    _lib.check(_lib.lib().psdf_constraints(fpp, m, poses.data_ptr(), N, ctypes.byref(ec),
                                           ctypes.byref(pc), float(d_min), hj.data_ptr(),
                                           None if host is None else host.data_ptr(),
                                           keys.data_ptr(), ws.data_ptr(), ws.numel(),
                                           _lib.stream_handle()))
    return hj, keys


def psdf_bwd_geometry(footprint, poses, edges: EdgeSet, keys, gout, params: Params | None = None):
    """(gedges (E, 4), gfp (m, 2)): sum over stages of gout[s] times the
    gradient of phi_s with respect to the edge endpoints (A_x, A_y, B_x, B_y)
    and the footprint vertices (caller's order), from the keys of a
    psdf_eval / psdf_grad on the same inputs."""
    params = params or Params()
    poses = _poses(poses)
    N = poses.shape[0]
    dev = poses.device
    gout = gout.contiguous().to(torch.float32)
    fp, fpp, m = _fp(footprint)
    gedges = torch.empty((edges.E, 4), dtype=torch.float32, device=dev)
    gfp = torch.empty((m, 2), dtype=torch.float32, device=dev)
    ec, pc = edges.c(), params.c()
    _lib.check(_lib.lib().psdf_bwd_geometry(fpp, m, poses.data_ptr(), N, ctypes.byref(ec),
                                            ctypes.byref(pc), keys.data_ptr(), gout.data_ptr(),
                                            gedges.data_ptr(), gfp.data_ptr(),
                                            _lib.stream_handle()))
    return gedges, gfp


def time_stage_min(footprint, poses, edges: EdgeSet, reps, params: Params | None = None,
                   ws=None):
    """Mean duration in ms of `reps` back-to-back launches of the
    per-stage-minimum kernel (measurement aid; synchronises the stream)."""
    params = params or Params()
    poses = _poses(poses)
    N = poses.shape[0]
    ws = workspace(N, edges.M, poses.device) if ws is None else ws
    fp, fpp, m = _fp(footprint)
    ec, pc = edges.c(), params.c()
    ms = ctypes.c_float(0.0)
    _lib.check(_lib.lib().psdf_time_stage_min(fpp, m, poses.data_ptr(), N, ctypes.byref(ec),
                                              ctypes.byref(pc), ws.data_ptr(), ws.numel(),
                                              int(reps), _lib.stream_handle(), ctypes.byref(ms)))
    return float(ms.value)


def psdf_sd_matrix(footprint, poses, edges: EdgeSet, params: Params | None = None, out=None):
    """sd[s, i] of every obstacle i at every stage s, before the minimum."""
    params = params or Params()
    poses = _poses(poses)
    N = poses.shape[0]
    sd = torch.empty((N, edges.M), dtype=torch.float32, device=poses.device) if out is None else out
    fp, fpp, m = _fp(footprint)
    ec, pc = edges.c(), params.c()
    _lib.check(_lib.lib().psdf_sd_matrix(fpp, m, poses.data_ptr(), N, ctypes.byref(ec),
                                         ctypes.byref(pc), sd.data_ptr(), _lib.stream_handle()))
    return sd


def validate_edges(edges: EdgeSet):
    """(count, lowest index) of the obstacles outside the edge-set contract:
    edge count negative or above mbar, range outside [0, E], or a non-finite
    coordinate (psdf_validate_edges).  The index is M when all are valid."""
    out = torch.empty(2, dtype=torch.int32, device=edges.obst_off.device)
    ec = edges.c()
    _lib.check(_lib.lib().psdf_validate_edges(ctypes.byref(ec), out.data_ptr(),
                                              _lib.stream_handle()))
    count, first = out.tolist()
    return count, first


def psdf_encode_padded(A, B, S):
    """EncodeEdges (Alg. 1): padded (A, B, S) device tensors -> device EdgeSet."""
    Mbar, mbar = int(S.shape[0]), int(S.shape[1])
    dev = S.device
    A = A.contiguous().to(torch.float32)
    B = B.contiguous().to(torch.float32)
    S8 = S.contiguous().to(torch.uint8)
    cap = max(1, Mbar * mbar)
    ax, ay, bx, by = (torch.empty(cap, dtype=torch.float32, device=dev) for _ in range(4))
    off = torch.empty(Mbar + 1, dtype=torch.int32, device=dev)
    wsb = int(_lib.lib().psdf_encode_ws_bytes(Mbar))
    ws = torch.empty(max(1, wsb), dtype=torch.uint8, device=dev)
    _lib.check(_lib.lib().psdf_encode_padded(A.data_ptr(), B.data_ptr(), S8.data_ptr(), Mbar, mbar,
                                             ax.data_ptr(), ay.data_ptr(), bx.data_ptr(),
                                             by.data_ptr(), off.data_ptr(), ws.data_ptr(),
                                             wsb, _lib.stream_handle()))
    E = int(off[-1].item()) if Mbar > 0 else 0
    return EdgeSet.from_device(ax[:E], ay[:E], bx[:E], by[:E], off, max(1, min(mbar, 16)))


class PsdfFunction(torch.autograd.Function):
    """phi = PsdfFunction.apply(poses, footprint, edges, params); backward runs
    the psdf_bwd adjoint kernel on the winners saved by the forward call.
    Gradients flow to the poses only."""

    @staticmethod
    def forward(ctx, poses, footprint, edges, params=None):
        d, edge, obst, keys = psdf_eval(footprint, poses.detach(), edges, params)
        ctx.save_for_backward(poses.detach(), keys)
        ctx.footprint, ctx.edges, ctx.params = footprint, edges, params
        return d

    @staticmethod
    def backward(ctx, gd):
        poses, keys = ctx.saved_tensors
        gpose = psdf_bwd(ctx.footprint, poses, ctx.edges, keys, gd, ctx.params)
        return gpose, None, None, None


class Batch:
    """Uneven batch of independent instances evaluated by one persistent
    launch (psdf_batch).  ``instances`` is a sequence of objects with
    ``footprint`` (m, 2), ``poses`` (N, 3), ``edges`` (E, 4) and ``obst_off``
    (M + 1,); they are packed host-side once and uploaded."""

    def __init__(self, instances, mbar=None, params: Params | None = None, graph=True,
                 autotune=False, device="cuda"):
        self.params = params or Params()
        fps, poses, edges, offs, desc = [], [], [], [], []
        nfp = npose = nedge = noff = 0
        for inst in instances:
            fp = np.asarray(inst.footprint, dtype=np.float32).reshape(-1, 2)
            ps = np.asarray(inst.poses, dtype=np.float32).reshape(-1, 3)
            ed = np.asarray(inst.edges, dtype=np.float32).reshape(-1, 4)
            of = np.asarray(inst.obst_off, dtype=np.int32)
            desc.append((nfp, len(fp), npose, len(ps), nedge, len(ed), noff, len(of) - 1))
            fps.append(fp); poses.append(ps); edges.append(ed); offs.append(of)
            nfp += len(fp); npose += len(ps); nedge += len(ed); noff += len(of)
        if mbar is None:
            sizes = np.concatenate([np.diff(o) for o in offs]) if offs else np.ones(1)
            mbar = int(max(1, sizes.max() if len(sizes) else 1))
        self.mbar = int(mbar)
        self.desc = desc
        self.n_inst = len(desc)
        self.footprints = np.ascontiguousarray(np.concatenate(fps) if fps else np.zeros((1, 2), np.float32))
        dev = torch.device(device)
        self.poses = torch.tensor(np.concatenate(poses) if poses else np.zeros((0, 3), np.float32), device=dev)
        ed = np.concatenate(edges) if edges else np.zeros((0, 4), np.float32)
        cols = torch.tensor(ed, device=dev).t().contiguous()
        self.ax, self.ay, self.bx, self.by = (cols[k].contiguous() for k in range(4))
        self.obst_off = torch.tensor(np.concatenate(offs) if offs else np.zeros(1, np.int32), device=dev)
        S = int(self.poses.shape[0])
        self.d = torch.empty(S, dtype=torch.float32, device=dev)
        self.edge = torch.empty(S, dtype=torch.int32, device=dev)
        self.obst = torch.empty(S, dtype=torch.int32, device=dev)
        self.grad = torch.empty((S, 3), dtype=torch.float32, device=dev)
        self.keys = torch.empty(S, dtype=torch.int64, device=dev)
        arr = (_lib.PsdfBatchDesc * max(1, self.n_inst))(*[_lib.PsdfBatchDesc(*d) for d in desc])
        flags = (_lib.PSDF_BATCH_GRAPH if graph else 0) | (_lib.PSDF_BATCH_AUTOTUNE if autotune else 0)
        plan = ctypes.c_void_p(0)
        pc = self.params.c()
        _lib.check(_lib.lib().psdf_batch_plan_create(
            ctypes.byref(plan), arr, self.n_inst, self.footprints.ctypes.data_as(ctypes.c_void_p),
            self.mbar, ctypes.byref(pc), flags))
        self.plan = plan

    def _args(self):
        return [self.poses.data_ptr(), self.ax.data_ptr(), self.ay.data_ptr(), self.bx.data_ptr(),
                self.by.data_ptr(), self.obst_off.data_ptr(), self.d.data_ptr(),
                self.edge.data_ptr(), self.obst.data_ptr(), self.grad.data_ptr(),
                self.keys.data_ptr()]

    def run(self):
        _lib.check(_lib.lib().psdf_batch(self.plan, *self._args(), _lib.stream_handle()))
        return self.d, self.edge, self.obst, self.grad, self.keys

    def autotune(self):
        best = ctypes.c_float(0.0)
        _lib.check(_lib.lib().psdf_batch_autotune(self.plan, *self._args(), _lib.stream_handle(),
                                                  ctypes.byref(best)))
        return best.value

    def set_shape(self, stages_per_item, obstacles_per_tile, direct=0):
        """Set the launch shape explicitly (psdf_batch_set_shape)."""
        _lib.check(_lib.lib().psdf_batch_set_shape(self.plan, int(stages_per_item),
                                                   int(obstacles_per_tile), int(direct)))

    def info(self):
        vals = [ctypes.c_int32(0) for _ in range(5)]
        _lib.check(_lib.lib().psdf_batch_plan_info(self.plan, *[ctypes.byref(v) for v in vals]))
        return dict(stages_per_item=vals[0].value, obstacles_per_tile=vals[1].value,
                    n_items=vals[2].value, grid=vals[3].value, direct=vals[4].value)

    def stage(self):
        """Take the obstacles' bounding circles once for the screened forms
        (psdf_batch_stage); stage again after changing the edge tensors in
        place."""
        _lib.check(_lib.lib().psdf_batch_stage(
            self.plan, self.ax.data_ptr(), self.ay.data_ptr(), self.bx.data_ptr(),
            self.by.data_ptr(), self.obst_off.data_ptr(), _lib.stream_handle()))
        return self

    def unstage(self):
        _lib.check(_lib.lib().psdf_batch_unstage(self.plan))
        return self

    def screened(self, theta=None, pool=256, topk=256, stats=False):
        """Certified screened evaluation (psdf_batch_screened); theta None
        ranks the pool's edges by distance instead of the MLP.  With
        stats=True also returns (stage_cand, stage_cert, cand_keys)."""
        S = int(self.poses.shape[0])
        dev = self.poses.device
        cand = torch.empty(S, dtype=torch.int32, device=dev) if stats else None
        cert = torch.empty(S, dtype=torch.int32, device=dev) if stats else None
        ck = torch.empty(S, dtype=torch.int64, device=dev) if stats else None
        tptr = theta.data_ptr() if theta is not None else None
        _lib.check(_lib.lib().psdf_batch_screened(
            self.plan, tptr, int(pool), int(topk), *self._args(),
            cand.data_ptr() if stats else None, cert.data_ptr() if stats else None,
            ck.data_ptr() if stats else None, _lib.stream_handle()))
        out = (self.d, self.edge, self.obst, self.grad, self.keys)
        return (out, (cand, cert, ck)) if stats else out

    def screened_bound(self, stats=False):
        """Certified screened evaluation without a ranking
        (psdf_batch_screened_bound): the lowest-bound obstacle's exact sd sets
        the bar; with stats=True also returns (stage_cand, stage_cert,
        cand_keys)."""
        S = int(self.poses.shape[0])
        dev = self.poses.device
        cand = torch.empty(S, dtype=torch.int32, device=dev) if stats else None
        cert = torch.empty(S, dtype=torch.int32, device=dev) if stats else None
        ck = torch.empty(S, dtype=torch.int64, device=dev) if stats else None
        _lib.check(_lib.lib().psdf_batch_screened_bound(
            self.plan, *self._args(), cand.data_ptr() if stats else None,
            cert.data_ptr() if stats else None, ck.data_ptr() if stats else None,
            _lib.stream_handle()))
        out = (self.d, self.edge, self.obst, self.grad, self.keys)
        return (out, (cand, cert, ck)) if stats else out

    def labels(self, stage, edge):
        """Features (n, 4) and exact pool-distance labels (n,) of (stage row,
        local edge) pairs (psdf_screen_labels)."""
        dev = self.poses.device
        st = torch.as_tensor(np.asarray(stage, dtype=np.int32), device=dev)
        ed = torch.as_tensor(np.asarray(edge, dtype=np.int32), device=dev)
        n = int(st.numel())
        X = torch.empty((n, 4), dtype=torch.float32, device=dev)
        T = torch.empty(n, dtype=torch.float32, device=dev)
        _lib.check(_lib.lib().psdf_screen_labels(
            self.plan, self.poses.data_ptr(), self.ax.data_ptr(), self.ay.data_ptr(),
            self.bx.data_ptr(), self.by.data_ptr(), st.data_ptr(), ed.data_ptr(), n,
            X.data_ptr(), T.data_ptr(), _lib.stream_handle()))
        return X, T

    def instance_views(self, k):
        """(footprint, poses, EdgeSet) views of instance k in the packed arrays."""
        fo, m, po, N, eo, E, oo, M = self.desc[k]
        es = EdgeSet.from_device(self.ax[eo:eo + E], self.ay[eo:eo + E], self.bx[eo:eo + E],
                                 self.by[eo:eo + E], self.obst_off[oo:oo + M + 1], self.mbar)
        return self.footprints[fo:fo + m], self.poses[po:po + N], es

    def close(self):
        if self.plan:
            _lib.lib().psdf_batch_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def horizon_batch(footprint, poses, stage_edges, stage_offsets, **kw):
    """Per-stage (time-varying) edge sets: stage s of a horizon is evaluated
    against its own edge set (stage_edges[s] (E_s, 4), stage_offsets[s]
    (M_s + 1,)).  Each stage is a one-stage instance of one batch, so the
    whole horizon is still one persistent launch; outputs are in stage order
    and edge / obstacle indices are local to the stage's set."""
    poses = np.asarray(poses, dtype=np.float32).reshape(-1, 3)
    if not (len(poses) == len(stage_edges) == len(stage_offsets)):
        raise ValueError("one edge set and one offset array per stage")
    insts = [SimpleNamespace(footprint=footprint, poses=poses[s:s + 1], edges=stage_edges[s],
                             obst_off=stage_offsets[s]) for s in range(len(poses))]
    return Batch(insts, **kw)


def set_launch_shape(blk=0, sb=0):
    """Override the per-stage minimum kernel's launch shape (blk 0 = automatic)."""
    _lib.check(_lib.lib().psdf_set_launch_shape(int(blk), int(sb)))


def hard_min():
    return Params(eta=math.inf)


# ------------------------------------------------------------------ screener MLP

def mlp_forward(theta, X):
    """MLP outputs for feature rows X (device (B, 4) float32)."""
    X = X.contiguous()
    B = int(X.shape[0])
    y = torch.empty(B, dtype=torch.float32, device=X.device)
    _lib.check(_lib.lib().psdf_mlp_forward(theta.data_ptr(), X.data_ptr(), B, y.data_ptr(),
                                           _lib.stream_handle()))
    return y


def _mlp_ws(B, device):
    nbytes = int(_lib.lib().psdf_mlp_ws_bytes(int(B)))
    return torch.empty(max(nbytes, 4), dtype=torch.uint8, device=device)


def mlp_grad(theta, X, T, ws=None):
    """(gradient of the mean squared error, loss) on the device."""
    X, T = X.contiguous(), T.contiguous()
    B = int(X.shape[0])
    ws = _mlp_ws(B, X.device) if ws is None else ws
    g = torch.empty(_lib.MLP_PARAMS + 1, dtype=torch.float32, device=X.device)
    _lib.check(_lib.lib().psdf_mlp_grad(theta.data_ptr(), X.data_ptr(), T.data_ptr(), B,
                                        g.data_ptr(), ws.data_ptr(), ws.numel(),
                                        _lib.stream_handle()))
    return g[:-1], g[-1]


def mlp_train_step(theta, m, v, step, lr, X, T, loss=None, ws=None):
    """One forward/backward/Adam step on the device (psdf_mlp_train_step)."""
    B = int(X.shape[0])
    ws = _mlp_ws(B, X.device) if ws is None else ws
    _lib.check(_lib.lib().psdf_mlp_train_step(
        theta.data_ptr(), m.data_ptr(), v.data_ptr(), int(step), float(lr), X.data_ptr(),
        T.data_ptr(), B, loss.data_ptr() if loss is not None else None, ws.data_ptr(),
        ws.numel(), _lib.stream_handle()))
