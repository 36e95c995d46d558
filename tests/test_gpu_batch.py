"""GPU tests of psdf_batch (uneven batches in one persistent launch, graph
replay, autotuner) against the per-instance psdf_grad path and the FP64
oracle."""
import numpy as np
import pytest

from paper_2607_04310_amd import inputs
from parity import check_stages

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_04310_amd import api as _api
    return _api


@pytest.fixture(scope="module")
def c4():
    return inputs.c4(512)


def per_instance(api, b):
    """The per-instance launch loop: psdf_grad on views of the packed arrays."""
    outs = []
    for k in range(b.n_inst):
        fp, poses, es = b.instance_views(k)
        outs.append(api.psdf_grad(fp, poses, es))
    torch.cuda.synchronize()
    cat = [torch.cat([o[j] for o in outs]) for j in range(4)]
    return [x.cpu().numpy() for x in cat]


def batch_out(b):
    b.run()
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (b.d, b.edge, b.obst, b.grad)]


def assert_equal_outputs(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y, equal_nan=True)


def test_c4_batch_matches_loop_bitwise(api, c4):
    print(f"[batch] c4 512 instances, {sum(i.N * i.E for i in c4):.3e} pairs", flush=True)
    b = api.Batch(c4, graph=False)
    assert_equal_outputs(batch_out(b), per_instance(api, b))
    b.close()


def test_c4_batch_vs_oracle_full(api, c4):
    """Every stage of all 512 c4 instances (1.1e8 stage x edge pairs) against
    the oracle: value, tie-aware winner and edge, gradient."""
    b = api.Batch(c4, graph=True)
    d, e, o, g = batch_out(b)
    tot = dict(stages=0, obst_ties=0, edge_ties=0, kink_grads=0, pen=0)
    for k, inst in enumerate(c4):
        po = b.desc[k][2]
        sl = slice(po, po + inst.N)
        st = check_stages(inst.footprint, inst.poses, inst.edges, inst.obst_off, 1000.0,
                          d[sl], e[sl], o[sl], g[sl])
        for key in tot:
            tot[key] += st[key]
        if k % 64 == 63:
            print(f"[batch] c4 vs oracle: {k + 1} instances, {tot}", flush=True)
    assert tot["stages"] == sum(i.N for i in c4)
    b.close()


def test_graph_replay_after_inputs_change(api, c4):
    sub = c4[:40]
    b = api.Batch(sub, graph=True)
    first = batch_out(b)
    again = batch_out(b)          # replay of the captured graph
    assert_equal_outputs(first, again)
    # change the inputs in place; the captured pointers stay valid
    with torch.no_grad():
        b.poses[:, 0] += 0.37
        b.poses[:, 2] -= 0.5
        b.ax.mul_(1.01)
    torch.cuda.synchronize()
    replay = batch_out(b)
    loop = per_instance(api, b)
    assert_equal_outputs(replay, loop)
    assert not np.array_equal(replay[0], first[0])
    b.close()


def test_concurrent_groups_graph_replays(api, c4):
    """Several footprint sizes run as concurrent launches (forked streams,
    graph branches once captured): every replay, with eager work and host
    synchronisations between replays, equals the per-instance loop."""
    sub = c4[:60]
    assert len({len(i.footprint) for i in sub}) > 1     # more than one group
    ref = None
    for graph in (True, False):
        b = api.Batch(sub, graph=graph)
        for rep in range(4):
            out = batch_out(b)
            if ref is None:
                ref = per_instance(api, b)
            assert_equal_outputs(out, ref)
            x = torch.randn(1 << 20, device="cuda")       # eager work between replays
            (x * 2.0).sum().item()
        b.close()


def test_autotune_keeps_results(api, c4):
    sub = c4[:96]
    b = api.Batch(sub, graph=True, autotune=True)
    ref = batch_out(b)
    best = b.autotune()
    info = b.info()
    assert best > 0 and info["n_items"] > 0 and info["stages_per_item"] in (1, 2, 4, 8, 16)
    assert_equal_outputs(batch_out(b), ref)
    # a second plan of the same signature starts from the cached shape
    b2 = api.Batch(sub, graph=False)
    assert b2.info()["stages_per_item"] == info["stages_per_item"]
    assert b2.info()["obstacles_per_tile"] == info["obstacles_per_tile"]
    assert_equal_outputs(batch_out(b2), ref)
    b.close()
    b2.close()


def test_explicit_shapes_keep_results(api, c4):
    """psdf_batch_set_shape: every launch shape (stage blocks of any length,
    cut evenly; 64- or 256-obstacle tiles; persistent or direct) gives the
    same outputs bit for bit."""
    b = api.Batch(c4[:48], graph=False)
    ref = batch_out(b)
    for sb, tile, direct in ((3, 64, 0), (7, 256, 1), (25, 256, 0), (64, 64, 1), (64, 256, 0)):
        b.set_shape(sb, tile, direct)
        info = b.info()
        assert (info["stages_per_item"], info["obstacles_per_tile"], info["direct"]) == (sb, tile, direct)
        assert_equal_outputs(batch_out(b), ref)
    b.close()


def test_batch_mixed_shapes_and_nan(api):
    rng = np.random.default_rng(77)
    insts = []
    for k in range(20):
        inst = inputs.random_small(rng, n_obst=int(rng.integers(1, 90)), n_poses=int(rng.integers(1, 70)),
                                   segments=int(rng.integers(0, 9)), lo=-3, hi=3)
        insts.append(inst)
    insts[3].poses = insts[3].poses.copy()
    insts[3].poses[0, 1] = np.nan
    b = api.Batch(insts, graph=True)
    d, e, o, g = batch_out(b)
    assert_equal_outputs([d, e, o, g], per_instance(api, b))
    po = b.desc[3][2]
    assert np.isnan(d[po]) and e[po] == -1 and o[po] == -1
    for k in (0, 5, 11, 19):
        inst = insts[k]
        sl = slice(b.desc[k][2], b.desc[k][2] + inst.N)
        check_stages(inst.footprint, inst.poses, inst.edges, inst.obst_off, 1000.0,
                     d[sl], e[sl], o[sl], g[sl])
    b.close()


def test_batch_obstacle_free_instances(api):
    """Instances without obstacles give the empty-set result (d = +inf, no
    winner, zero gradient), the same as psdf_grad on an empty edge set, in a
    mixed batch and in a batch with no edge at all; graph replays included."""
    rng = np.random.default_rng(78)
    insts = [inputs.random_small(rng, n_obst=0 if k in (0, 2, 5) else 25, n_poses=15 + k,
                                 segments=0 if k in (0, 2, 5) else 3, lo=-3, hi=3) for k in range(7)]
    for only_empty in (False, True):
        sel = [insts[k] for k in (0, 2, 5)] if only_empty else insts
        b = api.Batch(sel, graph=True)
        for _ in range(2):
            d, e, o, g = batch_out(b)
            assert_equal_outputs([d, e, o, g], per_instance(api, b))
        for k, inst in enumerate(sel):
            if len(inst.obst_off) == 1:
                sl = slice(b.desc[k][2], b.desc[k][2] + inst.N)
                assert np.all(np.isposinf(d[sl])) and np.all(e[sl] == -1) and np.all(o[sl] == -1)
                assert np.all(g[sl] == 0)
        b.close()


def test_single_instance_batch_equals_plain(api):
    inst = inputs.c2(0)
    b = api.Batch([inst], graph=True)
    assert_equal_outputs(batch_out(b), per_instance(api, b))
    b.close()


def test_time_varying_edge_sets(api):
    """Per-stage edge sets (moving obstacles): every stage against its own
    set, in one batch launch, checked stage by stage against the oracle."""
    fp, poses, stage_edges, stage_off = inputs.moving_obstacles(0, N=30, R=200)
    print(f"[batch] horizon of {len(poses)} stages with per-stage edge sets", flush=True)
    b = api.horizon_batch(fp, poses, stage_edges, stage_off, graph=True)
    d, e, o, g = batch_out(b)
    checked = 0
    for s in range(len(poses)):
        st = check_stages(fp, poses[s:s + 1], stage_edges[s], stage_off[s], 1000.0,
                          d[s:s + 1], e[s:s + 1], o[s:s + 1], g[s:s + 1])
        checked += st["stages"]
    assert checked == len(poses)
    # the sets do differ: stage 0's set at the last pose gives another result
    last = len(poses) - 1
    ref0 = __import__("oracle").psdf(fp, poses[last:], stage_edges[0], stage_off[0])
    assert ref0["phi"][0] != pytest.approx(float(d[last]), abs=1e-4)
    b.close()


def test_stage_rows_in_any_order(api):
    """The instances' stage rows may tile the packed poses in any order: a plan
    whose rows run in reverse instance order gives every stage the outputs it
    gets in instance order, for the plain batch and the screened forms."""
    import ctypes
    from paper_2607_04310_amd import _lib
    rng = np.random.default_rng(91)
    insts = [inputs.random_small(rng, n_obst=40 + 30 * k, n_poses=10 + 3 * k, segments=3, lo=-3, hi=3)
             for k in range(6)]
    b = api.Batch(insts, graph=False)
    n = b.n_inst
    Ns = [dd[3] for dd in b.desc]
    new_off, acc = [0] * n, 0
    for k in reversed(range(n)):
        new_off[k] = acc
        acc += Ns[k]
    # rows[r] = the row that stage r (instance order) takes in the reversed plan
    rows = np.concatenate([np.arange(new_off[k], new_off[k] + Ns[k]) for k in range(n)])
    b2 = api.Batch(insts, graph=False)
    _lib.lib().psdf_batch_plan_destroy(b2.plan)
    b2.plan = None
    desc = [(dd[0], dd[1], new_off[k]) + tuple(dd[3:]) for k, dd in enumerate(b.desc)]
    arr = (_lib.PsdfBatchDesc * n)(*[_lib.PsdfBatchDesc(*dd) for dd in desc])
    plan, pc = ctypes.c_void_p(0), b2.params.c()
    _lib.check(_lib.lib().psdf_batch_plan_create(
        ctypes.byref(plan), arr, n, b2.footprints.ctypes.data_as(ctypes.c_void_p), b2.mbar,
        ctypes.byref(pc), 0))
    b2.plan, b2.desc = plan, desc
    back = torch.tensor(np.argsort(rows), device=b.poses.device)   # new row -> old row
    b2.poses = b.poses[back].contiguous()
    print(f"[batch] {n} instances, {len(rows)} stage rows in reverse instance order", flush=True)

    def outs(x):
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in (x.d, x.edge, x.obst, x.grad, x.keys)]

    for form in ("plain", "bound", "distance", "bound_staged"):
        if form == "bound_staged":
            b.stage()
            b2.stage()
        for x in (b, b2):
            if form == "plain":
                x.run()
            elif form == "distance":
                x.screened(None, pool=128, topk=256)
            else:
                x.screened_bound()
        ref, got = outs(b), outs(b2)
        for u, v in zip(got, ref):
            assert np.array_equal(u[rows], v, equal_nan=True), form
    for k, inst in enumerate(insts):
        sl = slice(b.desc[k][2], b.desc[k][2] + inst.N)
        check_stages(inst.footprint, inst.poses, inst.edges, inst.obst_off, 1000.0,
                     *[t[sl] for t in ref[:4]])
    b.close()
    b2.close()


def test_all_footprint_groups_share_four_lanes(api):
    """Footprints of 3..8 and 9..16 vertices: all seven footprint-size groups
    in one batch, more groups than the call's four streams, so some streams
    run two groups back to back.  Eager calls and graph replays equal the
    per-instance loop bit for bit; sampled instances match the oracle."""
    rng = np.random.default_rng(93)
    ms = [3, 4, 5, 6, 7, 8, 9, 12, 16] * 3
    insts = [inputs.random_small(rng, n_obst=int(rng.integers(20, 120)), n_poses=int(rng.integers(5, 40)),
                                 segments=int(rng.integers(0, 6)), lo=-3, hi=3, fp_m=m) for m in ms]
    ref = None
    for graph in (False, True):
        b = api.Batch(insts, graph=graph)
        if ref is None:
            ref = per_instance(api, b)
        for _ in range(2):
            assert_equal_outputs(batch_out(b), ref)
        b.close()
    d, e, o, g = ref
    b = api.Batch(insts, graph=False)
    for k in (0, 6, 7, 8, 17, 26):
        inst = insts[k]
        sl = slice(b.desc[k][2], b.desc[k][2] + inst.N)
        check_stages(inst.footprint, inst.poses, inst.edges, inst.obst_off, 1000.0,
                     d[sl], e[sl], o[sl], g[sl])
    b.close()
