"""GPU tests of the screener: MLP kernels against the FP64 MLP oracle, label
generation against the PSDF oracle, certified screened evaluation equal to
the full evaluation bit for bit (MLP ranking, distance ranking, the
bound-threshold form, forced fallback), the c5 workload (64 instances x 50
stages x 65536 edges) checked against the FP64 oracle on the plain batch and
on every screened form (the MLP trained on held-out instances), and a
comparison of the trained network with the screens that use no network:
certification rate, exact evaluations, winner recall and call time."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp_oracle as mo
from paper_2607_04310_amd import inputs
from parity import check_stages, oracle_reference

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_04310_amd import api as _api
    return _api


def _rand_theta(seed):
    rng = np.random.default_rng(seed)
    th = inputs.mlp_init_params(seed).astype(np.float64)
    th[mo.H * mo.N_IN:mo.H * mo.N_IN + mo.H] = rng.normal(0, 0.2, mo.H)
    th[-1 - 2 * mo.H:-1 - mo.H] = rng.normal(0, 0.2, mo.H)
    th[-1] = 0.3
    return th.astype(np.float32)


def _close(gpu, ref, rtol=2e-2):
    scale = max(1e-6, float(np.abs(ref).max()))
    return float(np.abs(gpu - ref).max()) <= rtol * scale


@pytest.mark.parametrize("B", [1, 15, 16, 17, 1000, 4096])
def test_mlp_forward_vs_oracle(api, B):
    th = _rand_theta(B)
    X = np.random.default_rng(B).uniform(-1.5, 1.5, (B, 4)).astype(np.float32)
    y = api.mlp_forward(torch.tensor(th, device="cuda"), torch.tensor(X, device="cuda")).cpu().numpy()
    ref, _ = mo.forward(th, X, bf16_on=True)
    assert _close(y, ref)


@pytest.mark.parametrize("B", [16, 33, 4096])
def test_mlp_grad_vs_oracle(api, B):
    th = _rand_theta(100 + B)
    rng = np.random.default_rng(B)
    X = rng.uniform(-1.5, 1.5, (B, 4)).astype(np.float32)
    T = rng.uniform(0, 2, B).astype(np.float32)
    g, loss = api.mlp_grad(torch.tensor(th, device="cuda"), torch.tensor(X, device="cuda"),
                           torch.tensor(T, device="cuda"))
    g = g.cpu().numpy()
    ref = mo.backward(th, X, T, bf16_on=True)
    W1, b1, W2, b2, w3, b3 = mo.unpack(g)
    R = mo.unpack(ref)
    for name, a, b in zip(["W1", "b1", "W2", "b2", "w3", "b3"], (W1, b1, W2, b2, w3, b3), R):
        assert _close(np.asarray(a), np.asarray(b), 3e-2), name
    assert abs(float(loss) - mo.loss(th, X, T, True)) <= 2e-2 * max(1e-6, mo.loss(th, X, T, True))


def test_mlp_train_step_is_adam(api):
    th = _rand_theta(7)
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, (512, 4)).astype(np.float32)
    T = rng.uniform(0, 2, 512).astype(np.float32)
    dth = torch.tensor(th, device="cuda")
    g, _ = api.mlp_grad(dth, torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda"))
    m = torch.zeros_like(dth)
    v = torch.zeros_like(dth)
    api.mlp_train_step(dth, m, v, 1, 1e-3, torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda"))
    new, _, _ = mo.adam(th.astype(np.float64), np.zeros(len(th)), np.zeros(len(th)),
                        g.cpu().numpy().astype(np.float64), 1, 1e-3)
    np.testing.assert_allclose(dth.cpu().numpy(), new, rtol=0, atol=2e-6)


def test_training_reduces_loss(api):
    from paper_2607_04310_amd import screener
    insts = inputs.c5(2, cfg=6)
    X, T = screener.training_set(insts, near=512, far=512, seed=1)
    theta, hist = screener.train(X, T, epochs=20, batch=1024, lr=3e-3, seed=0)
    print(f"[train] {X.shape[0]} pairs, loss by epoch {[round(h, 4) for h in hist]}", flush=True)
    assert hist[-1] < 0.25 * hist[0]
    y = api.mlp_forward(theta, X)
    ref, _ = mo.forward(theta.cpu().numpy(), X.cpu().numpy(), bf16_on=True)
    assert _close(y.cpu().numpy(), ref)


def test_training_checkpoint_resume(api, tmp_path):
    """Training saved after 4 epochs and resumed from the checkpoint continues
    the Adam step count and keeps reducing the loss."""
    from paper_2607_04310_amd import screener
    insts = inputs.c5(1, cfg=6)
    X, T = screener.training_set(insts, near=256, far=256, seed=2)
    st = {}
    theta, hist = screener.train(X, T, epochs=4, batch=1024, lr=3e-3, seed=0, state=st)
    path = tmp_path / "screener.safetensors"
    screener.save_checkpoint(path, theta, st["m"], st["v"], step=st["step"], seed=0, hist=hist)
    ck = screener.load_checkpoint(path, device="cuda")
    assert torch.equal(ck["theta"], theta)
    st2 = {}
    theta2, hist2 = screener.train(X, T, epochs=4, batch=1024, lr=1e-3, seed=1, resume=ck, state=st2)
    assert st2["step"] == st["step"] + 4 * (X.shape[0] // 1024)
    assert hist2[-1] < hist[0] and np.isfinite(hist2).all()
    assert not torch.equal(theta2, theta)


def test_labels_vs_oracle(api):
    inst = inputs.c5_instance(0)
    b = api.Batch([inst], graph=False)
    rng = np.random.default_rng(0)
    st = rng.integers(0, inst.N, 300).astype(np.int32)
    ed = rng.integers(0, inst.E, 300).astype(np.int32)
    X, T = b.labels(st, ed)
    X, T = X.cpu().numpy(), T.cpu().numpy()
    for k in range(300):
        pose = inst.poses[st[k]].astype(np.float64)
        e = inst.edges[ed[k]].astype(np.float64)
        c, s = math.cos(pose[2]), math.sin(pose[2])
        loc = [(c * (x - pose[0]) + s * (y - pose[1]), -s * (x - pose[0]) + c * (y - pose[1]))
               for x, y in ((e[0], e[1]), (e[2], e[3]))]
        np.testing.assert_allclose(X[k], np.ravel(loc) / 4.0, atol=2e-6)
        i = int(np.searchsorted(inst.obst_off, ed[k], side="right") - 1)
        e0, e1 = inst.obst_off[i], inst.obst_off[i + 1]
        det = oracle.obstacle(inst.footprint, pose, inst.edges[e0:e1])
        assert abs(T[k] - min(5.0, det["edge_pool"][ed[k] - e0])) <= 1e-5
    b.close()


def _run_plain(b):
    b.run()
    torch.cuda.synchronize()
    return [x.clone() for x in (b.d, b.edge, b.obst, b.grad, b.keys)]


def _assert_same(a, b):
    for x, y in zip(a, b):
        assert torch.equal(x, y) or (x.dtype.is_floating_point and
                                     torch.equal(torch.nan_to_num(x, 7.0), torch.nan_to_num(y, 7.0)))


@pytest.mark.parametrize("ranking", ["distance", "mlp"])
def test_screened_equals_full_c5(api, ranking):
    insts = inputs.c5(16)
    b = api.Batch(insts, graph=False)
    ref = _run_plain(b)
    theta = torch.tensor(_rand_theta(3), device="cuda") if ranking == "mlp" else None
    out, (cand, cert, ck) = b.screened(theta, pool=256, topk=256, stats=True)
    torch.cuda.synchronize()
    _assert_same([x.clone() for x in out], ref)
    print(f"[screen {ranking}] certified {cert.float().mean().item():.3f}, "
          f"mean candidates {cand.float().mean().item():.1f}", flush=True)
    b.close()


def test_screened_forced_fallback(api):
    insts = inputs.c5(4)
    b = api.Batch(insts, graph=False)
    ref = _run_plain(b)
    out, (cand, cert, ck) = b.screened(None, pool=1, topk=1, stats=True)
    torch.cuda.synchronize()
    assert cert.float().mean().item() < 0.5          # most stages fall back
    _assert_same([x.clone() for x in out], ref)
    zero = torch.zeros(inputs.MLP_PARAMS, device="cuda")   # every score ties
    out = b.screened(zero, pool=64, topk=4)
    torch.cuda.synchronize()
    _assert_same([x.clone() for x in out], ref)
    b.close()


def test_screened_uneven_batch(api):
    insts = inputs.c4(64)
    b = api.Batch(insts, graph=False)
    ref = _run_plain(b)
    out = b.screened(None, pool=128, topk=128)
    torch.cuda.synchronize()
    _assert_same([x.clone() for x in out], ref)
    rng = np.random.default_rng(9)
    mixed = [inputs.random_small(rng, n_obst=40, n_poses=30, segments=6, lo=-3, hi=3) for _ in range(8)]
    mixed[2].poses = mixed[2].poses.copy()
    mixed[2].poses[4, 0] = np.nan
    b2 = api.Batch(mixed, graph=False)
    ref2 = _run_plain(b2)
    out2 = b2.screened(torch.tensor(_rand_theta(5), device="cuda"), pool=16, topk=8)
    torch.cuda.synchronize()
    _assert_same([x.clone() for x in out2], ref2)
    # the bound-threshold form on both batches (free segments, a NaN pose)
    for bb, rr in ((b, ref), (b2, ref2)):
        out3 = bb.screened_bound()
        torch.cuda.synchronize()
        _assert_same([x.clone() for x in out3], rr)
    b.close()
    b2.close()


def _assert_empty_rows(out, rows):
    d, edge, obst, grad, keys = (x.cpu() for x in out)
    assert bool(torch.isinf(d[rows]).all()) and bool((d[rows] > 0).all())
    assert bool((edge[rows] == -1).all()) and bool((obst[rows] == -1).all())
    assert bool((grad[rows] == 0).all()) and bool((keys[rows] == -1).all())


def test_screened_obstacle_free_instances(api):
    """Instances without obstacles, alone in a batch (no edges at all) and
    mixed with populated ones: their stages get the empty-set result (min
    over no obstacle is +inf) on the plain and the screened path, and every
    such stage certifies."""
    rng = np.random.default_rng(21)
    b = api.Batch([inputs.random_small(rng, n_obst=0, n_poses=10) for _ in range(3)], graph=False)
    ref = _run_plain(b)
    _assert_empty_rows(ref, slice(None))
    out, (cand, cert, ck) = b.screened(None, pool=16, topk=8, stats=True)
    torch.cuda.synchronize()
    _assert_same([x.clone() for x in out], ref)
    assert bool(cert.bool().all())
    b.close()
    mixed = [inputs.random_small(rng, n_obst=0 if k % 2 else 30, n_poses=20, segments=0 if k % 2 else 5)
             for k in range(6)]
    b2 = api.Batch(mixed, graph=False)
    ref2 = _run_plain(b2)
    rows = torch.tensor(np.concatenate([np.full(20, k % 2 == 1) for k in range(6)]))
    _assert_empty_rows(ref2, rows)
    out2, (cand, cert, ck) = b2.screened(None, pool=16, topk=8, stats=True)
    torch.cuda.synchronize()
    _assert_same([x.clone() for x in out2], ref2)
    assert bool(cert.bool().cpu()[rows].all())
    out3, (cand, cert, ck) = b2.screened_bound(stats=True)
    torch.cuda.synchronize()
    _assert_same([x.clone() for x in out3], ref2)
    assert bool(cert.bool().cpu()[rows].all())
    b2.close()


def test_screened_repeated_calls(api):
    """Back-to-back screened calls with and without fallback work: the
    screening counters start from zero on every call."""
    insts = inputs.c5(4)
    b = api.Batch(insts, graph=False)
    ref = _run_plain(b)
    for pool, topk in ((1, 1), (128, 256), (0, 0), (1, 1), (1, 1), (0, 0), (128, 256)):
        out = b.screened_bound() if pool == 0 else b.screened(None, pool=pool, topk=topk)
        torch.cuda.synchronize()
        _assert_same([x.clone() for x in out], ref)
    b.close()


# ---------------------------------------------------------------- c5 against the oracle

@pytest.fixture(scope="module")
def c5(api):
    """The c5 batch, its plain outputs, a network trained on held-out c5
    instances (other seeds) and the oracle's reference for the checked
    stages: every stage of instances 0 and 1, and three stages of each of
    the 64 instances."""
    from paper_2607_04310_amd import screener
    insts = inputs.c5(64)
    print(f"[c5] {sum(i.N * i.E for i in insts):.3e} stage x edge pairs", flush=True)
    b = api.Batch(insts, graph=False)
    plain = _run_plain(b)
    X, T = screener.training_set(inputs.c5(6, cfg=6), near=1024, far=1024, seed=1)
    theta, hist = screener.train(X, T, epochs=10, batch=4096, lr=2e-3, seed=0)
    print(f"[c5] trained on {X.shape[0]} held-out pairs, loss {hist[0]:.4f} -> {hist[-1]:.4f}",
          flush=True)
    rng = np.random.default_rng(11)
    checked = {}
    for k, inst in enumerate(insts):
        stages = np.arange(inst.N) if k < 2 else np.sort(rng.choice(inst.N, 3, replace=False))
        checked[k] = (stages, oracle_reference(inst.footprint, inst.poses, inst.edges,
                                               inst.obst_off, 1000.0, stages))
    print("[c5] oracle reference ready", flush=True)
    yield dict(insts=insts, b=b, plain=plain, theta=theta, checked=checked)
    b.close()


def _check_c5(c5, outs, label):
    d, e, o, g, _ = (x.cpu().numpy() for x in outs)
    tot = dict(stages=0, obst_ties=0, edge_ties=0, kink_grads=0, pen=0)
    for k, inst in enumerate(c5["insts"]):
        po = c5["b"].desc[k][2]
        sl = slice(po, po + inst.N)
        stages, ref = c5["checked"][k]
        st = check_stages(inst.footprint, inst.poses, inst.edges, inst.obst_off, 1000.0, d[sl],
                          e[sl], o[sl], g[sl], stages=stages, reference=ref)
        for key in tot:
            tot[key] += st[key]
    print(f"[c5 {label}] vs oracle: {tot}", flush=True)
    assert tot["stages"] == sum(len(v[0]) for v in c5["checked"].values())


def test_c5_plain_batch_vs_oracle(api, c5):
    _check_c5(c5, c5["plain"], "plain")


def _screen(c5, mode, theta=None):
    b = c5["b"]
    if mode == "bound":
        return b.screened_bound(stats=True)
    return b.screened(theta, pool=128, topk=256, stats=True)


@pytest.mark.parametrize("mode", ["distance", "trained_mlp", "bound"])
def test_c5_screened_vs_oracle(api, c5, mode):
    out, (cand, cert, ck) = _screen(c5, mode, c5["theta"] if mode == "trained_mlp" else None)
    torch.cuda.synchronize()
    out = [x.clone() for x in out]
    _assert_same(out, c5["plain"])
    _check_c5(c5, out, mode)
    print(f"[c5 {mode}] certified {cert.float().mean().item():.4f}, exact evaluations per "
          f"stage {cand.float().mean().item():.1f}", flush=True)


def _time_ms(fn, reps=10, warm=5):
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    z.record()
    torch.cuda.synchronize()
    return a.elapsed_time(z) / reps


def test_trained_network_against_screens_without_it(api, c5):
    """What the trained network gains over the method without it, on c5
    instances held out from its training set.  Every form is exact (bitwise
    the plain batch).  Reported per form: certification rate, exact
    (stage, obstacle) evaluations per stage, winner recall (the candidates'
    minimum is already the answer) and the call time.  Asserted: the trained
    network ranks better than an untrained one (higher winner recall, at
    least as many certified stages), and the bound-threshold form, which needs
    no ranking, certifies every stage with the fewest exact evaluations."""
    rows = {}
    forms = [("trained_mlp", c5["theta"]), ("untrained_mlp", torch.tensor(_rand_theta(3), device="cuda")),
             ("distance", None), ("bound", None)]
    for name, th in forms:
        mode = "bound" if name == "bound" else "ranked"
        out, (cand, cert, ck) = _screen(c5, mode, th)
        torch.cuda.synchronize()
        _assert_same([x.clone() for x in out], c5["plain"])
        t = _time_ms(lambda: _screen(c5, mode, th))
        keys = out[4]
        rows[name] = dict(certified=cert.float().mean().item(), exact=cand.float().mean().item(),
                          recall=(ck == keys).float().mean().item(), ms=t)
    t_plain = _time_ms(lambda: c5["b"].run())
    print(f"[gain] plain batch {t_plain:.3f} ms", flush=True)
    for name, r in rows.items():
        print(f"[gain] {name:>13}: certified {r['certified']:.4f}  exact/stage {r['exact']:7.1f}  "
              f"winner recall {r['recall']:.4f}  {r['ms']:.3f} ms", flush=True)
    tr, un = rows["trained_mlp"], rows["untrained_mlp"]
    print(f"[gain] trained network vs distance ranking: time x{rows['distance']['ms'] / tr['ms']:.2f}, "
          f"exact evaluations x{rows['distance']['exact'] / tr['exact']:.2f}; vs bound threshold: "
          f"time x{rows['bound']['ms'] / tr['ms']:.2f}", flush=True)
    assert tr["recall"] > un["recall"] and tr["certified"] >= un["certified"]
    assert tr["certified"] >= 0.95 and tr["recall"] >= 0.95
    assert rows["bound"]["certified"] == 1.0
    assert rows["bound"]["exact"] <= min(r["exact"] for r in rows.values())


@pytest.mark.parametrize("mode", ["ranked", "bound"])
def test_screened_open_chain_around_pose(api, mode):
    """An open chain of two edges whose convex hull holds the footprint (the
    axis test finds no separating axis, so its sd is negative) while the
    chain itself is 1 m from the pose: no certificate may exclude it (its
    bounds are -inf), so the screened result is the plain one even when the
    ranking picks a nearer rectangle as the only candidate."""
    fp = inputs.hexagon_footprint(inputs.rng_for(2, 0))
    poses = np.array([[3.0, 1.0, 0.0], [3.0, 1.0, 0.4]], np.float32)
    chain = np.array([[0, 0, 4, 0], [4, 0, 4, 4]], np.float32)
    rect = inputs.rect_edges(np.array([[3.0, 1.8]]), np.array([[0.2, 0.2]]), np.zeros(1))
    edges = np.concatenate([chain, rect]).astype(np.float32)
    off = np.array([0, 2, 6], np.int32)
    inst = inputs.Instance(fp, poses, edges, off, 4, dict(workload="open_chain"))
    ref = oracle.psdf(fp, poses, edges, off)
    assert np.all(ref["obst"] == 0) and np.all(ref["phi"] < 0)   # the chain wins, penetrating
    b = api.Batch([inst], graph=False)
    plain = _run_plain(b)
    out = b.screened_bound() if mode == "bound" else b.screened(None, pool=2, topk=1)
    torch.cuda.synchronize()
    _assert_same([x.clone() for x in out], plain)
    d, e, o, g, _ = (x.cpu().numpy() for x in plain)
    check_stages(fp, poses, edges, off, 1000.0, d, e, o, g)
    b.close()


def _copies_instance(n_obst, at, side, n_poses, seed):
    """n_obst copies of one square at `at` and a short horizon near the
    origin: every copy has the same horizon bound bit for bit (a tie block
    the horizon pass cannot split)."""
    edges = inputs.rect_edges(np.array([at], np.float64), np.array([[side, side]]), np.zeros(1))
    edges = np.tile(edges, (n_obst, 1))
    rng = np.random.default_rng(seed)
    poses = np.concatenate([rng.uniform(-0.2, 0.2, (n_poses, 2)),
                            rng.uniform(-np.pi, np.pi, (n_poses, 1))], 1).astype(np.float32)
    fp = inputs.hexagon_footprint(inputs.rng_for(2, 0))
    return inputs.Instance(fp, poses, edges.astype(np.float32), inputs.csr_offsets([4] * n_obst), 4,
                           dict(workload="copies"))


def test_screened_fallback_triggers(api):
    """The stages that no certificate may cover go to the full evaluation and
    still equal the plain batch: (a) more than 512 obstacles under the
    bound-threshold form's bar (600 squares stacked on the pose), (b) a
    horizon list longer than 2048 from a tie block of 2500 equal bounds
    (copies of one square),
    (c) an ordinary instance beside them that certifies."""
    rng = np.random.default_rng(4)
    fp = inputs.hexagon_footprint(inputs.rng_for(2, 0))
    stacked = inputs.rect_edges(rng.uniform(-0.3, 0.3, (600, 2)), np.full((600, 2), 0.2),
                                rng.uniform(-np.pi, np.pi, 600))
    dense = inputs.Instance(fp, np.array([[0.0, 0.0, 0.3], [0.1, -0.1, 1.0]], np.float32),
                            stacked.astype(np.float32), inputs.csr_offsets([4] * 600), 4,
                            dict(workload="stacked"))
    ring = _copies_instance(2500, (10.0, 0.0), 0.3, 6, 5)
    normal = inputs.c5_instance(3)
    b = api.Batch([dense, ring, normal], graph=False)
    ref = _run_plain(b)
    for form in ("bound", "distance"):
        if form == "bound":
            out, (cand, cert, ck) = b.screened_bound(stats=True)
        else:
            out, (cand, cert, ck) = b.screened(None, pool=512, topk=256, stats=True)
        torch.cuda.synchronize()
        _assert_same([x.clone() for x in out], ref)
        cert = cert.cpu().numpy()
        print(f"[fallback {form}] certified per row {cert.tolist()[:8]} ..., "
              f"normal instance {cert[8:].mean():.3f}", flush=True)
        if form == "bound":
            assert cert[:2].sum() == 0          # more than 512 candidates under the bar
        assert cert[2:8].sum() == 0             # the tied horizon list is unusable
        assert cert[8:].mean() > 0.9
    d, e, o, g, _ = (x.cpu().numpy() for x in ref)
    for k, inst in enumerate((dense, ring)):
        po = b.desc[k][2]
        sl = slice(po, po + inst.N)
        check_stages(inst.footprint, inst.poses, inst.edges, inst.obst_off, 1000.0, d[sl], e[sl],
                     o[sl], g[sl])
    b.close()


def test_screened_graph_replays(api):
    """Screened calls captured in a HIP graph and replayed three times, with
    eager plain and screened calls (and synchronisations) between the
    replays: every replay gives the plain batch's outputs.  The batch has
    stages that fail the certificate, so the replays run the fallback, and
    in the bound form its finishing tiles and the reopening of the horizon
    lists, from the graph."""
    rng = np.random.default_rng(14)
    fp = inputs.hexagon_footprint(inputs.rng_for(2, 0))
    stacked = inputs.rect_edges(rng.uniform(-0.3, 0.3, (600, 2)), np.full((600, 2), 0.2),
                                rng.uniform(-np.pi, np.pi, 600))
    dense = inputs.Instance(fp, np.array([[0.0, 0.0, 0.3], [0.1, -0.1, 1.0]], np.float32),
                            stacked.astype(np.float32), inputs.csr_offsets([4] * 600), 4,
                            dict(workload="stacked"))
    b = api.Batch([dense, inputs.c5_instance(5), _copies_instance(2500, (10.0, 0.0), 0.3, 6, 7)],
                  graph=False)
    ref = _run_plain(b)
    for form in ("bound", "distance"):
        call = (lambda: b.screened_bound()) if form == "bound" else \
            (lambda: b.screened(None, pool=128, topk=256))
        _, (cand, cert, _) = b.screened_bound(stats=True) if form == "bound" else \
            b.screened(None, pool=128, topk=256, stats=True)
        torch.cuda.synchronize()
        assert int((cert == 0).sum()) > 0        # the fallback has work
        call()
        torch.cuda.synchronize()
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cap):
            call()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=cap):
            call()
        for rep in range(3):
            for x in (b.d, b.edge, b.obst, b.grad, b.keys):
                x.zero_()
            g.replay()
            torch.cuda.synchronize()
            print(f"[graph {form}] replay {rep}", flush=True)
            _assert_same([x.clone() for x in (b.d, b.edge, b.obst, b.grad, b.keys)], ref)
            b.run()                              # eager work between the replays
            b.screened(None, pool=1, topk=1)     # an eager screened call (pool 1, top-1)
            torch.cuda.synchronize()
            _assert_same([x.clone() for x in (b.d, b.edge, b.obst, b.grad, b.keys)], ref)
        del g
    b.close()


def test_screened_all_footprint_groups(api):
    """Footprints of 3..16 vertices (all seven footprint-size groups, the
    16-slot screen kernels included): the bound-threshold, distance-ranked,
    network-ranked (untrained weights) and forced-fallback screened calls,
    on the edges and on staged circles, give the plain batch's outputs bit
    for bit, twice in a row."""
    rng = np.random.default_rng(94)
    ms = [3, 4, 5, 6, 7, 8, 9, 12, 16] * 2
    insts = [inputs.random_small(rng, n_obst=int(rng.integers(20, 150)), n_poses=int(rng.integers(5, 30)),
                                 segments=int(rng.integers(0, 6)), lo=-3, hi=3, fp_m=m) for m in ms]
    b = api.Batch(insts, graph=False)
    ref = _run_plain(b)
    theta = torch.tensor(_rand_theta(5), device="cuda")
    for staged in (False, True):
        if staged:
            b.stage()
        for name, fn in (("bound", lambda: b.screened_bound()),
                         ("distance", lambda: b.screened(None, pool=64, topk=64)),
                         ("network", lambda: b.screened(theta, pool=64, topk=64)),
                         ("fallback", lambda: b.screened(None, pool=1, topk=1))):
            for _ in range(2):
                out = fn()
                torch.cuda.synchronize()
                _assert_same([x.clone() for x in out], ref)
            print(f"[groups] {name} staged={staged} ok", flush=True)
    b.close()


# ---------------------------------------------------------------- staged circles

def _all_forms(b, theta):
    outs = {}
    for name, fn in (("bound", lambda: b.screened_bound()),
                     ("distance", lambda: b.screened(None, pool=128, topk=256)),
                     ("mlp", lambda: b.screened(theta, pool=128, topk=256)),
                     ("fallback", lambda: b.screened(None, pool=1, topk=1))):
        out = fn()
        torch.cuda.synchronize()
        outs[name] = [x.clone() for x in out]
    return outs


def test_staged_circles_same_results(api):
    """psdf_batch_stage: every screened form reads the circles taken once per
    edge set and gives the unstaged call's outputs bit for bit, on c5
    instances, an uneven mixed batch (free segments, a NaN pose, an open
    chain, empty instances) and the fallback-trigger batch."""
    rng = np.random.default_rng(31)
    mixed = [inputs.random_small(rng, n_obst=40, n_poses=30, segments=6, lo=-3, hi=3) for _ in range(5)]
    mixed[1].poses = mixed[1].poses.copy()
    mixed[1].poses[4, 0] = np.nan
    mixed.append(inputs.random_small(rng, n_obst=0, n_poses=10))
    fp = inputs.hexagon_footprint(inputs.rng_for(2, 0))
    chain = inputs.Instance(fp, np.array([[3.0, 1.0, 0.0], [3.0, 1.0, 0.4]], np.float32),
                            np.array([[0, 0, 4, 0], [4, 0, 4, 4]], np.float32),
                            np.array([0, 2], np.int32), 4, dict(workload="open_chain"))
    batches = [inputs.c5(8), mixed + [chain], [_copies_instance(2500, (10.0, 0.0), 0.3, 6, 5),
                                             inputs.c5_instance(5)]]
    theta = torch.tensor(_rand_theta(7), device="cuda")
    for insts in batches:
        b = api.Batch(insts, graph=False)
        print(f"[staged circles] {len(insts)} instances, {sum(i.M for i in insts)} obstacles",
              flush=True)
        plain = _run_plain(b)
        ref = _all_forms(b, theta)
        b.stage()
        got = _all_forms(b, theta)
        for name in ref:
            _assert_same(got[name], ref[name])
            _assert_same(got[name], plain)
        b.unstage()
        _assert_same(_all_forms(b, theta)["bound"], plain)
        b.close()


def test_staged_circles_checks_and_restage(api):
    """A screened call with other edge tensors than the staged ones is
    refused; after an in-place change of the edges, staging again gives the
    new edge set's outputs."""
    from paper_2607_04310_amd import _lib
    insts = inputs.c5(4)
    b = api.Batch(insts, graph=False).stage()
    old_ax = b.ax
    b.ax = b.ax.clone()
    with pytest.raises(_lib.PsdfError):
        b.screened_bound()
    b.ax = old_ax
    b.screened_bound()
    for col in (b.ax, b.bx):
        col.add_(0.61)
    b.stage()
    plain = _run_plain(b)
    out = b.screened_bound()
    torch.cuda.synchronize()
    _assert_same([x.clone() for x in out], plain)
    out = b.screened(None, pool=128, topk=256)
    torch.cuda.synchronize()
    _assert_same([x.clone() for x in out], plain)
    b.close()


@pytest.mark.parametrize("eta", [50.0, 1000.0, math.inf])
def test_staged_bound_quads_bitwise(api, eta):
    """The bound screen on staged rows evaluates its seed and a few candidates
    one obstacle per quad of lanes, and larger candidate sets one obstacle
    per lane: both give the plain batch's outputs bit for bit, at a soft, the
    default and the hard minimum, on penetrating stages, free segments, an
    open chain, an obstacle with a NaN coordinate and candidate sets on both
    sides of the quad path's limit (32)."""
    rng = np.random.default_rng(57)
    mixed = [inputs.random_small(rng, n_obst=60, n_poses=24, segments=8, lo=-2, hi=2)
             for _ in range(4)]
    bad = mixed[2]
    bad.edges = bad.edges.copy()
    bad.edges[5, 1] = np.nan             # an edge of the second rectangle
    fp = inputs.hexagon_footprint(inputs.rng_for(2, 0))
    chain = inputs.Instance(fp, np.array([[3.0, 1.0, 0.0], [3.0, 1.0, 0.4]], np.float32),
                            np.array([[0, 0, 4, 0], [4, 0, 4, 4]], np.float32),
                            np.array([0, 2], np.int32), 4, dict(workload="open_chain"))
    insts = mixed + [chain, _copies_instance(40, (0.5, 0.0), 0.3, 6, 5), inputs.c5_instance(3)]
    p = api.Params(eta=eta)
    b = api.Batch(insts, graph=False, params=p)
    print(f"[quads] eta={eta} {len(insts)} instances", flush=True)
    plain = _run_plain(b)
    lanes = [x.clone() for x in b.screened_bound()]
    b.stage()
    out, (cand, cert, _) = b.screened_bound(stats=True)
    torch.cuda.synchronize()
    _assert_same([x.clone() for x in out], plain)
    _assert_same(lanes, plain)
    n = cand.cpu().numpy()
    assert (n <= 33).any() and (n > 33).any(), "both evaluation paths taken"
    b.close()
