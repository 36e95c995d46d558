"""ctypes binding of ``libpsdf.so`` (the C ABI declared in include/psdf.h).

Argument marshalling only: every step of the PSDF runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream.  There is no
fallback: if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (imported first so that the library binds to torch's HIP runtime)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsdf.so")

PSDF_OK = 0
PSDF_EINVAL = -1
PSDF_ENONCONVEX = -2
PSDF_EDEGENERATE = -3
PSDF_ETOOBIG = -4
PSDF_EWS = -5
PSDF_EHIP = -6
MAX_FP_VERTS = 16
MAX_OBST_EDGES = 16
MLP_PARAMS = 4545
NOALLOC_WS_BYTES = 4 << 20


class PsdfParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_float), ("eps_sat", ctypes.c_float), ("eta", ctypes.c_float)]


class PsdfStaged(ctypes.Structure):
    _fields_ = [("table", ctypes.c_void_p), ("bytes", ctypes.c_size_t), ("E", ctypes.c_int32),
                ("M", ctypes.c_int32), ("mi_class", ctypes.c_int32), ("eps", ctypes.c_float),
                ("src", ctypes.c_void_p * 5)]


class PsdfEdges(ctypes.Structure):
    _fields_ = [("ax", ctypes.c_void_p), ("ay", ctypes.c_void_p), ("bx", ctypes.c_void_p),
                ("by", ctypes.c_void_p), ("obst_off", ctypes.c_void_p), ("E", ctypes.c_int32),
                ("M", ctypes.c_int32), ("mbar", ctypes.c_int32),
                ("staged", ctypes.POINTER(PsdfStaged))]


class PsdfBatchDesc(ctypes.Structure):
    _fields_ = [("fp_off", ctypes.c_int32), ("m", ctypes.c_int32), ("pose_off", ctypes.c_int32),
                ("N", ctypes.c_int32), ("edge_off", ctypes.c_int32), ("E", ctypes.c_int32),
                ("obst_off", ctypes.c_int32), ("M", ctypes.c_int32)]


PSDF_BATCH_GRAPH = 1
PSDF_BATCH_AUTOTUNE = 2


class PsdfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"psdf error {code}: {msg}")
        self.code = code


_lib = None

_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_SIGS = {
    "psdf_last_error": (ctypes.c_char_p, []),
    "psdf_version": (ctypes.c_char_p, []),
    "psdf_workspace_bytes": (ctypes.c_size_t, [_I32, _I32]),
    "psdf_eval": (ctypes.c_int, [_VP, _I32, _VP, _I32, ctypes.POINTER(PsdfEdges),
                                 ctypes.POINTER(PsdfParams), _VP, _VP, _VP, _VP, _VP,
                                 ctypes.c_size_t, _VP]),
    "psdf_grad": (ctypes.c_int, [_VP, _I32, _VP, _I32, ctypes.POINTER(PsdfEdges),
                                 ctypes.POINTER(PsdfParams), _VP, _VP, _VP, _VP, _VP, _VP,
                                 ctypes.c_size_t, _VP]),
    "psdf_grad_noalloc": (ctypes.c_int, [_VP, _I32, _VP, _I32, ctypes.POINTER(PsdfEdges),
                                         ctypes.POINTER(PsdfParams), _VP, _VP, _VP, _VP, _VP,
                                         _VP]),
    "psdf_set_launch_shape": (ctypes.c_int, [_I32, _I32]),
    "psdf_batch_plan_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(PsdfBatchDesc),
                                              _I32, _VP, _I32, ctypes.POINTER(PsdfParams), _I32]),
    "psdf_batch_plan_destroy": (None, [_VP]),
    "psdf_batch": (ctypes.c_int, [_VP] + [_VP] * 11 + [_VP]),
    "psdf_batch_autotune": (ctypes.c_int, [_VP] + [_VP] * 11 + [_VP, ctypes.POINTER(ctypes.c_float)]),
    "psdf_batch_screened": (ctypes.c_int, [_VP, _VP, _I32, _I32] + [_VP] * 11 + [_VP] * 3 + [_VP]),
    "psdf_batch_screened_bound": (ctypes.c_int, [_VP] + [_VP] * 11 + [_VP] * 3 + [_VP]),
    "psdf_screen_labels": (ctypes.c_int, [_VP] + [_VP] * 5 + [_VP, _VP, _I32, _VP, _VP, _VP]),
    "psdf_mlp_forward": (ctypes.c_int, [_VP, _VP, _I32, _VP, _VP]),
    "psdf_mlp_ws_bytes": (ctypes.c_size_t, [_I32]),
    "psdf_mlp_grad": (ctypes.c_int, [_VP, _VP, _VP, _I32, _VP, _VP, ctypes.c_size_t, _VP]),
    "psdf_mlp_train_step": (ctypes.c_int, [_VP, _VP, _VP, _I32, ctypes.c_float, _VP, _VP, _I32,
                                           _VP, _VP, ctypes.c_size_t, _VP]),
    "psdf_batch_plan_info": (ctypes.c_int, [_VP] + [ctypes.POINTER(_I32)] * 5),
    "psdf_batch_set_shape": (ctypes.c_int, [_VP, _I32, _I32, _I32]),
    "psdf_bwd": (ctypes.c_int, [_VP, _I32, _VP, _I32, ctypes.POINTER(PsdfEdges),
                                ctypes.POINTER(PsdfParams), _VP, _VP, _VP, _VP]),
    "psdf_constraints": (ctypes.c_int, [_VP, _I32, _VP, _I32, ctypes.POINTER(PsdfEdges),
                                        ctypes.POINTER(PsdfParams), ctypes.c_float, _VP, _VP, _VP,
                                        _VP, ctypes.c_size_t, _VP]),
    "psdf_bwd_geometry": (ctypes.c_int, [_VP, _I32, _VP, _I32, ctypes.POINTER(PsdfEdges),
                                         ctypes.POINTER(PsdfParams), _VP, _VP, _VP, _VP, _VP]),
    "psdf_time_stage_min": (ctypes.c_int, [_VP, _I32, _VP, _I32, ctypes.POINTER(PsdfEdges),
                                           ctypes.POINTER(PsdfParams), _VP, ctypes.c_size_t, _I32,
                                           _VP, ctypes.POINTER(ctypes.c_float)]),
    "psdf_sd_matrix": (ctypes.c_int, [_VP, _I32, _VP, _I32, ctypes.POINTER(PsdfEdges),
                                      ctypes.POINTER(PsdfParams), _VP, _VP]),
    "psdf_encode_ws_bytes": (ctypes.c_size_t, [_I32]),
    "psdf_timer_enable": (ctypes.c_int, [_I32]),
    "psdf_timer_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "psdf_validate_edges": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "psdf_staged_bytes": (ctypes.c_size_t, [_I32, _I32]),
    "psdf_batch_stage": (ctypes.c_int, [ctypes.c_void_p] * 7),
    "psdf_batch_unstage": (ctypes.c_int, [ctypes.c_void_p]),
    "psdf_stage_edges": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]),
    "psdf_encode_padded": (ctypes.c_int, [_VP, _VP, _VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP,
                                          _VP, ctypes.c_size_t, _VP]),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(rc):
    if rc != PSDF_OK:
        raise PsdfError(rc, lib().psdf_last_error().decode())
    return rc


def stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def timer_enable(capacity):
    check(lib().psdf_timer_enable(int(capacity)))


def timer_read():
    """(summed ms, launches) of the dominant-kernel launches timed since the last read."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    check(lib().psdf_timer_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value
