"""GPU test of psdf_grad_noalloc, the psdf_grad form that allocates nothing:
called through the C ABI, its outputs must equal psdf_grad's (same kernels,
so bit for bit) on two consecutive calls, the second on a smaller problem,
and a problem too large for its static scratch must be refused before any
work is enqueued."""
import ctypes

import numpy as np
import pytest

from paper_2607_04310_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_04310_amd import api as _api
    return _api


def _outputs(N, dev):
    return (torch.full((N,), 7.0, device=dev), torch.full((N,), 7, dtype=torch.int32, device=dev),
            torch.full((N,), 7, dtype=torch.int32, device=dev),
            torch.full((N, 3), 7.0, device=dev), torch.full((N,), 7, dtype=torch.int64, device=dev))


def _noalloc(api, fp, poses, es, params=None):
    from paper_2607_04310_amd import _lib
    params = params or api.Params()
    fp = np.ascontiguousarray(np.asarray(fp, dtype=np.float32).reshape(-1, 2))
    N = int(poses.shape[0])
    d, edge, obst, grad, keys = _outputs(N, poses.device)
    ec, pc = es.c(), params.c()
    rc = _lib.lib().psdf_grad_noalloc(fp.ctypes.data_as(ctypes.c_void_p), fp.shape[0],
                                      poses.data_ptr(), N, ctypes.byref(ec), ctypes.byref(pc),
                                      d.data_ptr(), edge.data_ptr(), obst.data_ptr(),
                                      grad.data_ptr(), keys.data_ptr(), _lib.stream_handle())
    return rc, (d, edge, obst, grad, keys)


def _same(a, b):
    for x, y in zip(a, b):
        assert torch.equal(x, y) or (x.dtype.is_floating_point and
                                     torch.equal(torch.nan_to_num(x, 9.0), torch.nan_to_num(y, 9.0)))


def test_noalloc_equals_psdf_grad_twice(api):
    from paper_2607_04310_amd import _lib
    dev = torch.device("cuda:0")
    big = inputs.c2(0)                              # N = 50, M = 4096: two kernels, 64 partial columns
    rng = np.random.default_rng(31)
    small = inputs.random_small(rng, n_obst=1500, n_poses=23, segments=40, lo=-12, hi=12)
    for inst in (big, small):
        print(f"[noalloc] N={inst.N} M={inst.M}", flush=True)
        es = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device=dev)
        poses = torch.tensor(inst.poses, device=dev)
        rc, got = _noalloc(api, inst.footprint, poses, es)
        assert rc == _lib.PSDF_OK, _lib.lib().psdf_last_error().decode()
        ref = api.psdf_grad(inst.footprint, poses, es)
        torch.cuda.synchronize()
        _same(got, ref)


def test_noalloc_refuses_oversized_problem(api):
    from paper_2607_04310_amd import _lib
    dev = torch.device("cuda:0")
    inst = inputs.c2(0)
    es = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device=dev)
    # N stages whose partial rows exceed the static scratch; checked on the
    # host before anything is enqueued, so the poses are never read
    N = _lib.NOALLOC_WS_BYTES // (16 * ((inst.M + 63) // 64)) + 1
    poses = torch.zeros((N, 3), device=dev)
    assert _lib.lib().psdf_workspace_bytes(N, inst.M) > _lib.NOALLOC_WS_BYTES
    rc, _ = _noalloc(api, inst.footprint, poses, es)
    assert rc == _lib.PSDF_ETOOBIG
    assert "no-alloc" in _lib.lib().psdf_last_error().decode()
    # the largest N that fits still runs and matches psdf_grad
    N -= 1
    poses = torch.tensor(np.resize(inst.poses, (N, 3)), device=dev)
    rc, got = _noalloc(api, inst.footprint, poses, es)
    assert rc == _lib.PSDF_OK, _lib.lib().psdf_last_error().decode()
    ref = api.psdf_grad(inst.footprint, poses, es)
    torch.cuda.synchronize()
    _same(got, ref)
