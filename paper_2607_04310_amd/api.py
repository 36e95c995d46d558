"""Python API over the C ABI: device-resident edge sets and the PSDF calls.

Every function here allocates its output tensors with torch on the poses'
device and calls the library on torch's current stream; the arithmetic is
all in the HIP kernels.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

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

    def c(self):
        return _lib.PsdfEdges(self.ax.data_ptr(), self.ay.data_ptr(), self.bx.data_ptr(),
                              self.by.data_ptr(), self.obst_off.data_ptr(), self.E, self.M,
                              self.mbar)


def _fp(footprint):
    fp = np.ascontiguousarray(np.asarray(footprint, dtype=np.float32).reshape(-1, 2))
    return fp, fp.ctypes.data_as(ctypes.c_void_p), int(fp.shape[0])


def _poses(poses):
    assert poses.dtype == torch.float32 and poses.is_cuda and poses.dim() == 2 and poses.shape[1] == 3
    return poses.contiguous()


def psdf_eval(footprint, poses, edges: EdgeSet, params: Params | None = None):
    """phi, edge, obstacle and winner keys per stage (psdf_eval of the C ABI)."""
    params = params or Params()
    poses = _poses(poses)
    N = poses.shape[0]
    dev = poses.device
    d = torch.empty(N, dtype=torch.float32, device=dev)
    edge = torch.empty(N, dtype=torch.int32, device=dev)
    obst = torch.empty(N, dtype=torch.int32, device=dev)
    keys = torch.empty(N, dtype=torch.int64, device=dev)
    fp, fpp, m = _fp(footprint)
    ec, pc = edges.c(), params.c()
    _lib.check(_lib.lib().psdf_eval(fpp, m, poses.data_ptr(), N, ctypes.byref(ec),
                                    ctypes.byref(pc), d.data_ptr(), edge.data_ptr(),
                                    obst.data_ptr(), keys.data_ptr(), _lib.stream_handle()))
    return d, edge, obst, keys


def psdf_grad(footprint, poses, edges: EdgeSet, params: Params | None = None, out=None):
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
    fp, fpp, m = _fp(footprint)
    ec, pc = edges.c(), params.c()
    _lib.check(_lib.lib().psdf_grad(fpp, m, poses.data_ptr(), N, ctypes.byref(ec),
                                    ctypes.byref(pc), d.data_ptr(), edge.data_ptr(),
                                    obst.data_ptr(), grad.data_ptr(), keys.data_ptr(),
                                    _lib.stream_handle()))
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


def hard_min():
    return Params(eta=math.inf)
