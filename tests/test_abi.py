"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every entry point include/psdf.h declares, and its host validation returns
the documented error codes before anything is enqueued."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2607_04310_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "psdf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psdf_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    syms = declared_symbols()
    assert "psdf_eval" in syms and "psdf_grad" in syms and "psdf_bwd" in syms
    for name in syms:
        assert hasattr(lib, name), name
    assert lib.psdf_version().decode().startswith("psdf")


RECT = np.array([[-0.3, -0.2], [0.3, -0.2], [0.3, 0.2], [-0.3, 0.2]], np.float32)


def _call_eval(fp, m=None, N=0, edges=None, params=None, poses=1):
    fp = np.ascontiguousarray(fp, dtype=np.float32)
    m = fp.shape[0] if m is None else m
    e = edges if edges is not None else _lib.PsdfEdges(1, 1, 1, 1, 1, 4, 1, 4)
    p = params or _lib.PsdfParams(1e-12, 1e-6, 1000.0)
    d = ctypes.c_void_p(1)
    return _lib.lib().psdf_eval(fp.ctypes.data_as(ctypes.c_void_p), m, ctypes.c_void_p(poses), N,
                                ctypes.byref(e), ctypes.byref(p), d, d, d, d, d, 1 << 30, None)


def test_valid_footprint_with_no_stage_is_a_no_op():
    assert _call_eval(RECT) == _lib.PSDF_OK
    assert _call_eval(RECT[::-1]) == _lib.PSDF_OK        # clockwise accepted


@pytest.mark.parametrize("fp,code", [
    (RECT[:2], _lib.PSDF_ENONCONVEX),                                   # m = 2
    (np.zeros((17, 2)), _lib.PSDF_ENONCONVEX),                          # m = 17
    (np.array([[0, 0], [1, 0], [0.2, 0.2], [0, 1]]), _lib.PSDF_ENONCONVEX),   # reflex vertex
    (np.array([[0, 0], [1, 0], [1, 0], [0, 1]]), _lib.PSDF_EDEGENERATE),      # zero-length edge
    (np.array([[0, 0], [1, 0], [2, 0], [0, 1]]), _lib.PSDF_ENONCONVEX),       # collinear
    (np.array([[0, 0], [1, 0], [0, 1], [1, 1]]), _lib.PSDF_ENONCONVEX),       # bow tie
])
def test_footprint_validation(fp, code):
    assert _call_eval(fp) == code
    assert _lib.lib().psdf_last_error().decode() != ""


def test_self_intersecting_star_rejected():
    ang = np.deg2rad(144.0 * np.arange(5))                 # pentagram: every turn is left
    star = np.stack([np.cos(ang), np.sin(ang)], 1)
    assert _call_eval(star) == _lib.PSDF_ENONCONVEX


@pytest.mark.parametrize("mbar", [0, 17])
def test_mbar_bound(mbar):
    e = _lib.PsdfEdges(1, 1, 1, 1, 1, 4, 1, mbar)
    assert _call_eval(RECT, edges=e) == _lib.PSDF_ETOOBIG


def test_null_and_negative_arguments():
    assert _call_eval(RECT, N=-1) == _lib.PSDF_EINVAL
    assert _call_eval(RECT, N=3, poses=0) == _lib.PSDF_EINVAL
    assert _call_eval(RECT, edges=_lib.PsdfEdges(0, 1, 1, 1, 1, 4, 1, 4)) == _lib.PSDF_EINVAL
    assert _call_eval(RECT, edges=_lib.PsdfEdges(1, 1, 1, 1, 0, 4, 1, 4)) == _lib.PSDF_EINVAL
    assert _call_eval(RECT, edges=_lib.PsdfEdges(1, 1, 1, 1, 1, -4, 1, 4)) == _lib.PSDF_EINVAL
    nan_params = _lib.PsdfParams(1e-12, 1e-6, float("nan"))
    assert _call_eval(RECT, params=nan_params) == _lib.PSDF_EINVAL
    assert _call_eval(RECT, params=_lib.PsdfParams(-1.0, 1e-6, 1.0)) == _lib.PSDF_EINVAL


def test_workspace_query_and_check():
    lib = _lib.lib()
    assert lib.psdf_workspace_bytes(0, 10) == 0 and lib.psdf_workspace_bytes(10, 0) == 0
    assert lib.psdf_workspace_bytes(50, 4096) == 2 * 50 * 64 * 8
    # a too-small workspace is rejected before anything is enqueued
    fp = np.ascontiguousarray(RECT)
    e = _lib.PsdfEdges(1, 1, 1, 1, 1, 4, 1, 4)
    p = _lib.PsdfParams(1e-12, 1e-6, 1000.0)
    d = ctypes.c_void_p(1)
    rc = lib.psdf_eval(fp.ctypes.data_as(ctypes.c_void_p), 4, d, 3, ctypes.byref(e), ctypes.byref(p),
                       d, d, d, d, d, 8, None)
    assert rc == _lib.PSDF_EWS


def test_launch_shape_override_validation():
    lib = _lib.lib()
    assert lib.psdf_set_launch_shape(128, 1) == _lib.PSDF_EINVAL
    assert lib.psdf_set_launch_shape(64, 0) == _lib.PSDF_EINVAL
    assert lib.psdf_set_launch_shape(64, 65) == _lib.PSDF_EINVAL
    assert lib.psdf_set_launch_shape(256, 4) == _lib.PSDF_OK
    assert lib.psdf_set_launch_shape(0, 0) == _lib.PSDF_OK


def test_encode_workspace_query():
    assert _lib.lib().psdf_encode_ws_bytes(0) == 0
    assert _lib.lib().psdf_encode_ws_bytes(1000) >= 4000


def test_constraints_validation():
    fp = np.ascontiguousarray(RECT)
    e = _lib.PsdfEdges(1, 1, 1, 1, 1, 4, 1, 4)
    p = _lib.PsdfParams(1e-12, 1e-6, 1000.0)
    lib = _lib.lib()

    def call(dmin, hj, keys=1):
        return lib.psdf_constraints(fp.ctypes.data_as(ctypes.c_void_p), 4, ctypes.c_void_p(1), 1,
                                    ctypes.byref(e), ctypes.byref(p), dmin, hj, None,
                                    ctypes.c_void_p(keys) if keys else None, ctypes.c_void_p(1),
                                    1 << 30, None)
    assert call(0.01, None) == _lib.PSDF_EINVAL
    assert call(0.01, ctypes.c_void_p(1), keys=0) == _lib.PSDF_EINVAL
    assert call(float("nan"), ctypes.c_void_p(1)) == _lib.PSDF_EINVAL
    assert "d_min" in lib.psdf_last_error().decode()


def test_time_stage_min_validation():
    fp = np.ascontiguousarray(RECT)
    e = _lib.PsdfEdges(1, 1, 1, 1, 1, 4, 1, 4)
    p = _lib.PsdfParams(1e-12, 1e-6, 1000.0)
    ms = ctypes.c_float(1.0)
    lib = _lib.lib()
    assert lib.psdf_time_stage_min(fp.ctypes.data_as(ctypes.c_void_p), 4, ctypes.c_void_p(1), 1,
                                   ctypes.byref(e), ctypes.byref(p), ctypes.c_void_p(1), 1 << 30,
                                   0, None, ctypes.byref(ms)) == _lib.PSDF_EINVAL
    # no stage: nothing launched, zero time
    assert lib.psdf_time_stage_min(fp.ctypes.data_as(ctypes.c_void_p), 4, None, 0,
                                   ctypes.byref(e), ctypes.byref(p), None, 0, 5, None,
                                   ctypes.byref(ms)) == _lib.PSDF_OK and ms.value == 0.0


def test_misaligned_workspace_is_rejected():
    fp = np.ascontiguousarray(RECT)
    e = _lib.PsdfEdges(1, 1, 1, 1, 1, 4, 1, 4)
    p = _lib.PsdfParams(1e-12, 1e-6, 1000.0)
    d = ctypes.c_void_p(16)
    rc = _lib.lib().psdf_eval(fp.ctypes.data_as(ctypes.c_void_p), 4, ctypes.c_void_p(16), 1,
                              ctypes.byref(e), ctypes.byref(p), d, d, d, d, ctypes.c_void_p(8),
                              1 << 30, None)
    assert rc == _lib.PSDF_EINVAL
    assert "aligned" in _lib.lib().psdf_last_error().decode()


def test_validate_edges_argument_checks():
    lib = _lib.lib()
    assert lib.psdf_validate_edges(None, ctypes.c_void_p(16), None) == _lib.PSDF_EINVAL
    e = _lib.PsdfEdges(1, 1, 1, 1, 1, 4, 1, 4)
    assert lib.psdf_validate_edges(ctypes.byref(e), None, None) == _lib.PSDF_EINVAL
    bad_mbar = _lib.PsdfEdges(1, 1, 1, 1, 1, 4, 1, 17)
    assert lib.psdf_validate_edges(ctypes.byref(bad_mbar), ctypes.c_void_p(16), None) == _lib.PSDF_ETOOBIG


def _staged(E=4, M=1, cls=4, eps=1e-12, table=256, nbytes=1 << 20, src=(1, 1, 1, 1, 1)):
    return _lib.PsdfStaged(table, nbytes, E, M, cls, eps, (ctypes.c_void_p * 5)(*src))


def test_staged_table_size():
    lib = _lib.lib()
    assert lib.psdf_staged_bytes(0, 4) == 0 and lib.psdf_staged_bytes(10, 0) == 0
    assert lib.psdf_staged_bytes(10, 17) == 0 and lib.psdf_staged_bytes((1 << 28) + 1, 4) == 0
    # (40 * class + 16) bytes per row, rows = M rounded up to 64
    assert lib.psdf_staged_bytes(1, 4) == 64 * 176
    assert lib.psdf_staged_bytes(4096, 3) == 4096 * 176
    assert lib.psdf_staged_bytes(65, 5) == 128 * 336
    assert lib.psdf_staged_bytes(64, 16) == 64 * 656


def test_stage_edges_argument_checks():
    lib = _lib.lib()
    e = _lib.PsdfEdges(1, 1, 1, 1, 1, 4, 1, 4)
    p = _lib.PsdfParams(1e-12, 1e-6, 1000.0)
    out = _lib.PsdfStaged()
    need = lib.psdf_staged_bytes(1, 4)

    def stage(edges=e, params=p, table=256, nbytes=need, o=out):
        return lib.psdf_stage_edges(ctypes.byref(edges), ctypes.byref(params) if params else None,
                                    table, nbytes, ctypes.byref(o) if o is not None else None,
                                    None)
    assert stage(o=None) == _lib.PSDF_EINVAL
    assert stage(table=None) == _lib.PSDF_EINVAL
    assert stage(table=264) == _lib.PSDF_EINVAL                 # not 16-byte aligned
    assert stage(nbytes=need - 1) == _lib.PSDF_EWS
    assert stage(params=_lib.PsdfParams(float("nan"), 1e-6, 1.0)) == _lib.PSDF_EINVAL
    assert stage(edges=_lib.PsdfEdges(1, 1, 1, 1, 1, 4, 1, 0)) == _lib.PSDF_ETOOBIG
    assert stage(edges=_lib.PsdfEdges(1, 1, 1, 1, 1, 4, (1 << 28) + 1, 4)) == _lib.PSDF_ETOOBIG
    # an empty edge set needs no table and enqueues nothing
    empty = _lib.PsdfEdges(0, 0, 0, 0, 1, 0, 0, 4)
    assert stage(edges=empty, table=None, nbytes=0) == _lib.PSDF_OK
    assert (out.E, out.M, out.mi_class) == (0, 0, 4)
    assert list(out.src) == [None, None, None, None, 1]


@pytest.mark.parametrize("rows", [
    [(0, 3), (2, 2)],           # row 2 in both instances (row 4 in none)
    [(0, 3), (4, 2)],           # beyond the 5 packed rows
    [(3, 2), (0, 2), (2, 2)],   # row 3 twice
])
def test_batch_plan_rejects_stage_rows_that_do_not_tile(rows):
    # plan creation checks the descriptors before it touches the device, so
    # a rejected layout returns without a GPU
    n = len(rows)
    desc = (_lib.PsdfBatchDesc * n)(*[_lib.PsdfBatchDesc(0, 4, po, N, 0, 0, 0, 0) for po, N in rows])
    fp = np.ascontiguousarray(RECT)
    p = _lib.PsdfParams(1e-12, 1e-6, 1000.0)
    plan = ctypes.c_void_p()
    rc = _lib.lib().psdf_batch_plan_create(ctypes.byref(plan), desc, n,
                                           fp.ctypes.data_as(ctypes.c_void_p), 4, ctypes.byref(p), 0)
    assert rc == _lib.PSDF_EINVAL and not plan.value
    assert "stage row" in _lib.lib().psdf_last_error().decode()


def test_batch_stage_argument_checks():
    lib = _lib.lib()
    assert lib.psdf_batch_stage(None, 1, 1, 1, 1, 1, None) == _lib.PSDF_EINVAL
    assert lib.psdf_batch_unstage(None) == _lib.PSDF_EINVAL


@pytest.mark.parametrize("fields,ok", [
    (dict(), True),
    (dict(E=8), False),                      # made for another edge count
    (dict(M=2), False),                      # another obstacle count
    (dict(cls=8), False),                    # another edge class
    (dict(eps=1e-9), False),                 # another eps
    (dict(table=None), False),
    (dict(table=264), False),                # misaligned
    (dict(nbytes=100), False),               # too small
    (dict(src=(1, 1, 1, 2, 1)), False),      # made from other arrays
])
def test_staged_table_must_match_the_call(fields, ok):
    st = _staged(**fields)
    e = _lib.PsdfEdges(1, 1, 1, 1, 1, 4, 1, 4, ctypes.pointer(st))
    rc = _call_eval(RECT, edges=e)         # N = 0: only the host checks run
    assert rc == (_lib.PSDF_OK if ok else _lib.PSDF_EINVAL)
