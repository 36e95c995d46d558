"""Benchmark of the PSDF hot path on one MI355X.

A step is one psdf_batch call (value, winning obstacle and edge, and the pose
gradient of every stage) on the 'c5' workload: 64 independent instances,
each a hexagonal footprint (circumradius 0.5 m, vertex radii jittered
+-10 %) at N = 50 stage poses along a random smooth path, against 65536 edges
from 16384 rectangles (sides U[0.1, 0.8] m) whose centres follow a
32-component Gaussian mixture (sigma = 2 m) in a 60 x 60 m square;
2.10e8 stage x edge pairs per step.  Inputs are resident in HBM before the
timed region.

Prints one JSON line:
  value        stage x edge evaluations per second of whole psdf_batch calls
               (K calls, each a replay of the plan's HIP graph, between one
               event pair);
  screened     the same outputs (bit for bit) from the certified screened
               forms on the same inputs: the bound-threshold form, and the
               top-K forms ranked by the edge distance and by the screener
               network trained on held-out instances; rate, certification,
               exact evaluations per stage, winner recall; and each form again
               with the obstacles' bounding circles taken once per edge set;
  roofline     the persistent batch kernel: algorithmic FLOP per launch over
               its mean duration from HIP events that each dispatch records
               on its launch stream; VALU issue and HBM bytes from the
               rocprofv3 counter summaries in profiles/ while the kernel's
               sources are unchanged;
  cpu_baseline the FP64 oracle on the host's cores (all, and one), built for
               the host (-O3 -march=native), on a bounded c5 sample;
  extras       c2 latency (one psdf_grad call, on the edges and on the staged
               edge set), c2 x 256, the uneven batch c4
               against its per-instance loop, one pose against growing edge
               sets, the paper's Table I query shapes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stage×edge PSDF+grad evals/s (plain vs screened, exact) and % FP32 VALU peak"
PEAK_FP32_TFLOPS = 157.3
# The published FP32 peak counts packed FP32 (two results per lane and
# instruction).  The kernels are built without packed FP32, so one FMA per
# lane and cycle, 78.6 TFLOP/s, is the ceiling they can reach.
REACHABLE_FP32_TFLOPS = 78.6
SIMDS, CLOCK_GHZ = 1024, 2.4

CSRC = os.path.join("paper_2607_04310_amd", "csrc")
# each kernel's own sources (code, instantiation, launch choice, build flags)
KERNELS = {
    # the batch kernel's code and its work items; its launch shape is hashed with it
    "batch_kernel": dict(
        sources=[os.path.join(CSRC, f) for f in (
            "psdf_device.hpp", "psdf_winner.hpp", "psdf_batch.hpp", "psdf_batch.hip",
            "psdf_host.hpp")]
        + [os.path.join("paper_2607_04310_amd", "build.py")],
        valu=os.path.join(ROOT, "profiles", "batch_kernel_c5_valu_counters.md"),
        hbm=os.path.join(ROOT, "profiles", "batch_kernel_c5_hbm_counters.md")),
    "main_kernel": dict(
        sources=[os.path.join(CSRC, f) for f in (
            "psdf_device.hpp", "psdf_kernels.hpp", "psdf_winner.hpp", "psdf_inst_mf6.hip",
            "psdf_host.cpp", "psdf_host.hpp")]
        + [os.path.join("paper_2607_04310_amd", "build.py")],
        valu=os.path.join(ROOT, "profiles", "main_kernel_c2_valu_counters.md"),
        hbm=os.path.join(ROOT, "profiles", "main_kernel_c2_hbm_counters.md")),
    # the same per-stage minimum reading a staged edge set
    "main_staged_kernel": dict(
        sources=[os.path.join(CSRC, f) for f in (
            "psdf_device.hpp", "psdf_kernels.hpp", "psdf_staged.hpp", "psdf_winner.hpp",
            "psdf_inst_mf6.hip", "psdf_host.cpp", "psdf_host.hpp")]
        + [os.path.join("paper_2607_04310_amd", "build.py")],
        valu=os.path.join(ROOT, "profiles", "main_staged_kernel_c2_valu_counters.md"),
        hbm=os.path.join(ROOT, "profiles", "main_staged_kernel_c2_hbm_counters.md")),
}


def source_hash(kernel, shape=None):
    """Hash of the kernel's sources (and of its launch shape, when given)."""
    h = hashlib.sha256()
    for f in KERNELS[kernel]["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if shape is not None:
        h.update(json.dumps(shape, sort_keys=True).encode())
    return h.hexdigest()[:16]


def counted(kernel, what, field, shape=None):
    """A figure recorded in a counter summary, or (None, why not) when the
    summary is missing or the kernel (or its launch shape) has changed since
    it was taken."""
    try:
        text = open(KERNELS[kernel][what]).read()
    except OSError:
        return None, "no counter summary"
    mh = re.search(r"source_sha256:\s*([0-9a-f]+)", text)
    mv = re.search(field + r":\s*([0-9.eE+]+)", text)
    if not mh or not mv:
        return None, "counter summary incomplete"
    if mh.group(1) != source_hash(kernel, shape):
        return None, "kernel changed since the counters were taken"
    return float(mv.group(1)), "rocprofv3 counters"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the GPU's clock ramps up under load: the batch kernel runs ~15 % slower
    # during the first ~40 launches (30 ms), so the default warmup covers that
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=24.0,
                    help="bound on the CPU-oracle sample (0 disables it)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--counters", choices=["", "c5", "c2", "screen", "single"], default="",
                    help="only launch the workload's dominant call `steps` times (eagerly) and a "
                         "256 MiB device copy (the calibration of the HBM byte counters); "
                         "screen: c5's bound-threshold and distance-ranked screened calls on "
                         "staged circles, `steps` times each; single: one pose against 4194304 "
                         "rectangles (16.7 M edges)")
    ap.add_argument("--extras", type=int, default=1, help="also measure the secondary workloads")
    ap.add_argument("--screened", type=int, default=1, help="also measure the screened forms")
    return ap.parse_args()


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def timed_calls(torch, fn, reps, warm):
    """Mean ms per call of `reps` calls between one event pair, after `warm`."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a, b = _events(torch)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def graph_calls(torch, fn, reps, outs, rtol=None):
    """Mean ms per call of `reps` calls captured into one HIP graph (outside
    the timed region) and replayed once between an event pair, after an
    untimed replay whose outputs must equal the eager call's bit for bit
    (with rtol: within rtol of the largest magnitude, for outputs summed with
    float atomics in no fixed order)."""
    fn()
    torch.cuda.synchronize()
    ref = [x.clone() for x in outs]
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cap):
        for _ in range(reps):
            fn()
    for x in outs:
        x.zero_()
    g.replay()
    torch.cuda.synchronize()
    for x, y in zip(outs, ref):
        if rtol is not None:
            scale = float(y.abs().max()) if y.numel() else 0.0
            if not torch.allclose(x, y, rtol=0.0, atol=rtol * scale, equal_nan=True):
                raise RuntimeError("graph replay differs from the eager call")
        elif not (torch.equal(x, y) or torch.equal(torch.nan_to_num(x, 7.0), torch.nan_to_num(y, 7.0))):
            raise RuntimeError("graph replay differs from the eager call")
    a, b = _events(torch)
    a.record()
    g.replay()
    b.record()
    torch.cuda.synchronize()
    del g
    return a.elapsed_time(b) / reps


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(oracle, insts, nthreads, budget, stages=None):
    """stage x edge pairs per second of the FP64 oracle over `insts` (cycled
    until `budget` seconds are spent), all stages or the first `stages`."""
    t0 = time.perf_counter()
    pairs, k, used = 0, 0, 0
    while True:
        i = insts[k % len(insts)]
        n = i.N if stages is None else min(stages, i.N)
        r = oracle.psdf(i.footprint, i.poses[:n], i.edges, i.obst_off, nthreads=nthreads)
        used = r["threads"]
        pairs += n * i.E
        k += 1
        done = time.perf_counter() - t0
        if done >= budget:
            return pairs / done, k, done, int(used)


def cpu_baseline(c5, seconds, inputs):
    """The FP64 oracle (value, winner, gradient) timed on this host, on all
    cores and on one core: the headline on c5 (a third of the budget each),
    and c1, c2 and a c4 sample (the last third)."""
    import oracle
    oracle.use_native_build()
    inst = c5[0]
    oracle.psdf(inst.footprint, inst.poses[:1], inst.edges, inst.obst_off)   # load / warm
    v, k, done, used = _oracle_rate(oracle, c5, 0, seconds / 3)
    v1, k1, done1, _ = _oracle_rate(oracle, c5[:1], 1, seconds / 3, stages=4)
    others = {}
    small = dict(c1=[inputs.c1(s) for s in range(4)], c2=[inputs.c2(s) for s in range(2)],
                 c4=[inputs.c4_instance(k) for k in range(16)])
    share = seconds / 3 / (2 * len(small))
    for name, insts in small.items():
        a, ka, _, ua = _oracle_rate(oracle, insts, 0, share)
        b, kb, _, _ = _oracle_rate(oracle, insts, 1, share)
        others[name] = dict(value=a, one_core_value=b, threads=ua,
                            sample=f"{len(insts)} instances cycled, {ka} / {kb} calls")
    return dict(value=v, unit="stage×edge evals/s", cores=used, kind="oracle",
                sample=f"{k} whole c5 instances (N={inst.N}, E={inst.E}, value+winner+gradient, "
                       f"FP64) in {done:.1f} s on {used} threads",
                one_core_value=v1,
                one_core_sample=f"{k1} x the first 4 stages of c5 instance 0 in {done1:.1f} s",
                other_configs=others,
                cpu_model=cpu_model(), nproc=os.cpu_count(),
                build="g++ -O3 -march=native -ffp-contract=off -fopenmp")


def extras(torch, api, flops, inputs):
    """c2 latency with its kernel's roofline, c2 x 256, the uneven batch c4
    against its per-instance loop, one pose against growing edge sets, and
    the Table I query shapes."""
    from paper_2607_04310_amd import _lib
    out = {}
    inst = inputs.c2(0)
    es = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device="cuda")
    poses = torch.tensor(inst.poses, device="cuda")
    ws = api.workspace(inst.N, inst.M, "cuda")
    o = api.psdf_grad(inst.footprint, poses, es, ws=ws)

    def c2_step():
        api.psdf_grad(inst.footprint, poses, es, out=o, ws=ws)
    t_graph = graph_calls(torch, c2_step, 200, list(o))
    t_eager = timed_calls(torch, c2_step, 200, 20)
    kms = api.time_stage_min(inst.footprint, poses, es, 200, ws=ws)
    fl = flops.flops_instance(len(inst.footprint), inst.N, inst.edges, inst.obst_off)
    valu, _ = counted("main_kernel", "valu", "valu_insts_per_launch")
    out["c2_latency"] = dict(
        workload="c2: hexagon (m=6), N=50 path poses, E=16384 (4096 rectangles, 40x40 m), psdf_grad",
        us_per_call=t_graph * 1e3, eager_us_per_call=t_eager * 1e3,
        evals_per_s=inst.N * inst.E / (t_graph * 1e-3),
        main_kernel_us=kms * 1e3, main_kernel_tflops=fl / (kms * 1e-3) / 1e12,
        main_kernel_frac=fl / (kms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
        main_kernel_valu_busy=None if valu is None else valu * 4 / (SIMDS * kms * 1e-3 * CLOCK_GHZ * 1e9))
    log(f"c2: {t_graph * 1e3:.2f} us per call (graph), {t_eager * 1e3:.2f} eager, main kernel "
        f"{kms * 1e3:.2f} us")
    # the same call on the staged edge set (the obstacles' pose-independent
    # constants taken once, when the environment changes)
    ref = [x.clone() for x in o]
    es.stage()
    t_graph_s = graph_calls(torch, c2_step, 200, list(o))
    if not all(torch.equal(x, y) for x, y in zip(o, ref)):
        raise RuntimeError("psdf_grad on the staged edge set differs from the plain call")
    t_eager_s = timed_calls(torch, c2_step, 200, 20)
    kms_s = api.time_stage_min(inst.footprint, poses, es, 200, ws=ws)
    valu_s, _ = counted("main_staged_kernel", "valu", "valu_insts_per_launch")
    out["c2_latency"]["staged"] = dict(
        us_per_call=t_graph_s * 1e3, eager_us_per_call=t_eager_s * 1e3,
        evals_per_s=inst.N * inst.E / (t_graph_s * 1e-3),
        main_kernel_us=kms_s * 1e3, main_kernel_tflops=fl / (kms_s * 1e-3) / 1e12,
        main_kernel_frac=fl / (kms_s * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
        main_kernel_valu_busy=None if valu_s is None
        else valu_s * 4 / (SIMDS * kms_s * 1e-3 * CLOCK_GHZ * 1e9))
    log(f"c2 staged: {t_graph_s * 1e3:.2f} us per call (graph), {t_eager_s * 1e3:.2f} eager, "
        f"main kernel {kms_s * 1e3:.2f} us")
    del es, poses, ws, o, ref

    log("c4: building 512 instances")
    c4 = inputs.c4(512)
    pairs4 = sum(i.N * i.E for i in c4)
    b = api.Batch(c4, graph=True, autotune=True)
    b.autotune()
    t_batch = timed_calls(torch, b.run, 20, 3)
    views = [b.instance_views(k) for k in range(b.n_inst)]

    def loop():
        for fp, ps, e in views:
            api.psdf_grad(fp, ps, e)
    t_loop = timed_calls(torch, loop, 3, 1)
    f4 = sum(flops.flops_instance(len(i.footprint), i.N, i.edges, i.obst_off) for i in c4)
    out["c4_batch"] = dict(pairs=pairs4, batch_ms=t_batch, loop_ms=t_loop,
                           batch_evals_per_s=pairs4 / (t_batch * 1e-3),
                           loop_evals_per_s=pairs4 / (t_loop * 1e-3),
                           batch_tflops=f4 / (t_batch * 1e-3) / 1e12, shape=b.info())
    log(f"c4: batch {t_batch:.3f} ms, loop {t_loop:.3f} ms")
    b.close()
    del c4, views

    c2b = inputs.c2_batch(256)
    pairs2 = sum(i.N * i.E for i in c2b)
    b = api.Batch(c2b, graph=True, autotune=True)
    b.autotune()
    t = timed_calls(torch, b.run, 20, 3)
    f2 = sum(flops.flops_instance(len(i.footprint), i.N, i.edges, i.obst_off) for i in c2b)
    out["c2x256_batch"] = dict(pairs=pairs2, ms=t, evals_per_s=pairs2 / (t * 1e-3),
                               tflops=f2 / (t * 1e-3) / 1e12, shape=b.info())
    log(f"c2x256: {t:.3f} ms")
    b.close()
    del c2b

    sweep = []
    for rects in (1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22):
        inst = inputs.single_pose(rects)
        es = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device="cuda")
        poses = torch.tensor(inst.poses, device="cuda")
        ws = api.workspace(1, inst.M, "cuda")
        o = api.psdf_grad(inst.footprint, poses, es, ws=ws)
        t = timed_calls(torch, lambda: api.psdf_grad(inst.footprint, poses, es, out=o, ws=ws), 20, 3)
        nbytes = flops.bytes_instance(1, inst.E, inst.M)
        sweep.append(dict(E=inst.E, ms=t, evals_per_s=inst.E / (t * 1e-3),
                          gbytes_per_s=nbytes / (t * 1e-3) / 1e9))
        del es, poses, ws, o
    out["single_pose_sweep"] = sweep
    log("single pose: " + ", ".join(f"E={r['E']}: {r['gbytes_per_s']:.0f} GB/s" for r in sweep))

    table = []
    for M in (1, 10, 100):
        for B in (1, 10, 100):
            inst = inputs.table_i(M, B)
            es = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device="cuda")
            poses = torch.tensor(inst.poses, device="cuda")
            ws = api.workspace(B, M, "cuda")
            o = api.psdf_grad(inst.footprint, poses, es, ws=ws)
            t_fwd = timed_calls(torch, lambda: api.psdf_eval(inst.footprint, poses, es, ws=ws), 200, 20)
            step = lambda: api.psdf_grad(inst.footprint, poses, es, out=o, ws=ws)  # noqa: E731
            t_grad = timed_calls(torch, step, 200, 20)
            t_g = graph_calls(torch, step, 100, list(o))
            table.append(dict(M=M, B=B, fwd_us=t_fwd * 1e3, grad_us=t_grad * 1e3,
                              grad_graph_us=t_g * 1e3))
            del es, poses, ws, o
    out["table_i_latency"] = table
    log("table I: " + ", ".join(f"{r['M']}x{r['B']}: {r['grad_graph_us']:.1f} us" for r in table))
    return out


def next_rows(torch, api, flops, inputs):
    """The rows beyond the per-stage minimum, on c2's shapes: per-stage
    (time-varying) edge sets in one batch launch, the geometry adjoint, the
    constraint export (with and without its copy to pinned host memory) and
    the per-obstacle sd matrix (also on one c5 instance); each timed as K
    calls captured in one HIP graph and replayed."""
    import ctypes

    import numpy as np

    from paper_2607_04310_amd import _lib
    lib = _lib.lib()
    out = {}
    fp, poses_h, stage_edges, stage_off = inputs.moving_obstacles(0, N=50, R=4096, half=20.0)
    b = api.horizon_batch(fp, poses_h, stage_edges, stage_off, graph=False)
    t = graph_calls(torch, b.run, 100, [b.d, b.edge, b.obst, b.grad, b.keys])
    pairs = sum(len(e) for e in stage_edges)
    out["per_stage_edge_sets"] = dict(
        workload="50 stages, each against its own set of 4096 moving rectangles (c2's density)",
        us_per_call=t * 1e3, evals_per_s=pairs / (t * 1e-3), shape=b.info())
    log(f"per-stage edge sets: {t * 1e3:.1f} us per call")
    b.close()
    del b, stage_edges, stage_off

    inst = inputs.c2(0)
    es = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device="cuda")
    poses = torch.tensor(inst.poses, device="cuda")
    ws = api.workspace(inst.N, inst.M, "cuda")
    d, edge, obst, grad, keys = api.psdf_grad(inst.footprint, poses, es, ws=ws)
    fpa = np.ascontiguousarray(np.asarray(inst.footprint, dtype=np.float32))
    fpp, m = fpa.ctypes.data_as(ctypes.c_void_p), int(fpa.shape[0])
    ec, pc = es.c(), api.Params().c()
    gout = torch.ones(inst.N, device="cuda")
    ge = torch.empty((inst.E, 4), device="cuda")
    gf = torch.empty((m, 2), device="cuda")

    def geometry():
        _lib.check(lib.psdf_bwd_geometry(fpp, m, poses.data_ptr(), inst.N, ctypes.byref(ec),
                                         ctypes.byref(pc), keys.data_ptr(), gout.data_ptr(),
                                         ge.data_ptr(), gf.data_ptr(), _lib.stream_handle()))
    t = graph_calls(torch, geometry, 200, [ge, gf], rtol=1e-5)
    out["geometry_adjoint"] = dict(
        workload="c2: sum over the 50 stages of dphi/d(edge endpoints) and dphi/d(footprint "
                 "vertices), from psdf_grad's keys", us_per_call=t * 1e3)
    log(f"geometry adjoint: {t * 1e3:.1f} us per call")

    hj = torch.empty((inst.N, 4), device="cuda")
    kk = torch.empty(inst.N, dtype=torch.int64, device="cuda")
    host = torch.empty((inst.N, 4), dtype=torch.float32, pin_memory=True)
    res = {}
    for name, hp in (("device", None), ("with_pinned_copy", host)):
        def export(hp=hp):
            _lib.check(lib.psdf_constraints(fpp, m, poses.data_ptr(), inst.N, ctypes.byref(ec),
                                            ctypes.byref(pc), 0.1, hj.data_ptr(),
                                            None if hp is None else hp.data_ptr(), kk.data_ptr(),
                                            ws.data_ptr(), ws.numel(), _lib.stream_handle()))
        res[name] = graph_calls(torch, export, 200, [hj, kk]) * 1e3
    if not torch.equal(host, hj.cpu()):
        raise RuntimeError("the pinned copy of the constraint rows differs from the device rows")
    out["constraint_export"] = dict(
        workload="c2: (phi - d_min, -grad phi) per stage, d_min = 0.1 m", us_per_call=res)
    log(f"constraint export: {res['device']:.1f} us per call, {res['with_pinned_copy']:.1f} with "
        f"the pinned copy")
    del es, poses, ws, d, edge, obst, grad, keys, ge, gf, hj, kk

    rows = []
    for name, inst in (("c2", inputs.c2(0)), ("c5 instance 0", inputs.c5_instance(0))):
        es = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device="cuda")
        poses = torch.tensor(inst.poses, device="cuda")
        sd = api.psdf_sd_matrix(inst.footprint, poses, es)
        t = graph_calls(torch, lambda: api.psdf_sd_matrix(inst.footprint, poses, es, out=sd), 100,
                        [sd])
        fl = flops.flops_instance(len(inst.footprint), inst.N, inst.edges, inst.obst_off)
        rows.append(dict(workload=f"{name}: N={inst.N} x M={inst.M} sd values", us_per_call=t * 1e3,
                         evals_per_s=inst.N * inst.E / (t * 1e-3),
                         out_gbytes_per_s=inst.N * inst.M * 4 / (t * 1e-3) / 1e9,
                         tflops=fl / (t * 1e-3) / 1e12,
                         frac=fl / (t * 1e-3) / 1e12 / PEAK_FP32_TFLOPS))
        log(f"sd matrix {name}: {t * 1e3:.1f} us per call, {rows[-1]['tflops']:.1f} TFLOP/s")
        del es, poses, sd
    out["sd_matrix"] = rows
    return out


def screened_forms(torch, api, inputs, c5, b, ref, steps):
    """The certified screened forms on the c5 batch: each timed as `steps`
    calls in one HIP graph replay, its outputs equal to the plain batch's."""
    from paper_2607_04310_amd import screener
    log("c5: training the screener on held-out instances")
    X, T = screener.training_set(inputs.c5(10, cfg=6), near=1024, far=1024, seed=1)
    theta, hist = screener.train(X, T, epochs=12, batch=4096, lr=2e-3, seed=0, log=log)
    pairs = sum(i.N * i.E for i in c5)
    forms = {"bound": lambda: b.screened_bound(),
             "distance": lambda: b.screened(None, pool=128, topk=256),
             "trained_mlp": lambda: b.screened(theta, pool=128, topk=256)}
    res = dict(train_pairs=int(X.shape[0]), train_loss=hist[-1])
    outs = [b.d, b.edge, b.obst, b.grad, b.keys]
    for name, fn in forms.items():
        ms = graph_calls(torch, fn, steps, outs)
        if name == "bound":
            _, (cand, cert, ck) = b.screened_bound(stats=True)
        else:
            _, (cand, cert, ck) = b.screened(None if name == "distance" else theta, pool=128,
                                             topk=256, stats=True)
        torch.cuda.synchronize()
        exact = all(torch.equal(x, y) or torch.equal(torch.nan_to_num(x, 7.0), torch.nan_to_num(y, 7.0))
                    for x, y in zip(outs, ref))
        if not exact:
            raise RuntimeError(f"screened ({name}) outputs differ from the plain batch")
        res[name] = dict(ms=ms, evals_per_s=pairs / (ms * 1e-3), exact=exact,
                         certified=float(cert.float().mean()),
                         exact_evals_per_stage=float(cand.float().mean()),
                         winner_recall=float((ck == b.keys).float().mean()))
        log(f"c5 screened {name}: {ms:.4f} ms, certified {res[name]['certified']:.4f}, "
            f"{res[name]['exact_evals_per_stage']:.1f} exact per stage")
    # the same forms with the bounding circles taken once per edge set
    # (psdf_batch_stage), as when the environment is static between calls
    b.stage()
    res["staged_circles"] = {}
    for name, fn in forms.items():
        ms = graph_calls(torch, fn, steps, outs)
        torch.cuda.synchronize()
        if not all(torch.equal(x, y) or torch.equal(torch.nan_to_num(x, 7.0), torch.nan_to_num(y, 7.0))
                   for x, y in zip(outs, ref)):
            raise RuntimeError(f"screened ({name}, staged circles) outputs differ from the plain batch")
        res["staged_circles"][name] = dict(ms=ms, evals_per_s=pairs / (ms * 1e-3), exact=True)
        log(f"c5 screened {name}, staged circles: {ms:.4f} ms")
    b.unstage()
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the PSDF hot path has no multi-GPU path "
              "(independent instances would shard across GPUs with no exchange; one huge "
              "instance would shard its obstacles and all-reduce the per-stage minimum keys)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2607_04310_amd import _lib, api, flops, inputs

    if args.counters == "single":
        inst = inputs.single_pose(1 << 22)
        es = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device="cuda")
        poses = torch.tensor(inst.poses, device="cuda")
        ws = api.workspace(1, inst.M, "cuda")
        for _ in range(args.steps):
            api.psdf_grad(inst.footprint, poses, es, ws=ws)
        torch.cuda.synchronize()
        del es
    if args.counters == "c2":
        inst = inputs.c2(0)
        es = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device="cuda")
        poses = torch.tensor(inst.poses, device="cuda")
        ws = api.workspace(inst.N, inst.M, "cuda")
        for _ in range(args.steps):
            api.psdf_grad(inst.footprint, poses, es, ws=ws)
        es.stage()      # then as many calls on the staged edge set
        for _ in range(args.steps):
            api.psdf_grad(inst.footprint, poses, es, ws=ws)
    log("c5: building 64 instances")
    c5 = inputs.c5(64)
    pairs = sum(i.N * i.E for i in c5)
    if args.counters:
        if args.counters == "c5":
            b = api.Batch(c5, graph=False)
            for _ in range(args.steps):
                b.run()
            b.close()
        if args.counters == "screen":
            b = api.Batch(c5, graph=False)
            b.stage()
            for _ in range(args.steps):
                b.screened_bound()
            for _ in range(args.steps):
                b.screened(None, pool=128, topk=256)
            b.close()
        src = torch.ones(64 << 20, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(counters_run=args.counters, steps=args.steps,
                              copy_bytes=src.numel() * 4)))
        return

    bg = api.Batch(c5, graph=True)       # replays the plan's own HIP graph
    be = api.Batch(c5, graph=False)      # eager launches (kernel timing, screened forms)
    if bg.info() != be.info():
        raise RuntimeError("the two plans of the same batch chose different launch shapes")
    be.run()
    bg.run()
    torch.cuda.synchronize()
    ref = [x.clone() for x in (be.d, be.edge, be.obst, be.grad, be.keys)]
    got = [bg.d, bg.edge, bg.obst, bg.grad, bg.keys]
    if not all(torch.equal(x, y) or torch.equal(torch.nan_to_num(x, 7.0), torch.nan_to_num(y, 7.0))
               for x, y in zip(got, ref)):
        raise RuntimeError("graph replay of psdf_batch differs from the eager call")
    # warm-up straight into the timed region: the GPU's clock drops when it
    # idles (a host-side check here cost the first ~40 timed calls up to 25 %)
    for _ in range(args.warmup):
        bg.run()

    # timed region: K whole psdf_batch calls between one event pair
    a, z = _events(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record()
    for _ in range(args.steps):
        bg.run()
    z.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = a.elapsed_time(z) / args.steps
    value = pairs / (ms_step * 1e-3)
    log(f"c5 plain psdf_batch: {ms_step:.4f} ms per call, {value:.3e} evals/s")

    # the persistent batch kernel alone: events recorded by each dispatch on
    # its launch stream, over K eager calls
    _lib.timer_enable(args.steps)
    for _ in range(args.steps):
        be.run()
    torch.cuda.synchronize()
    kms_total, launches = _lib.timer_read()
    _lib.timer_enable(0)
    kernel_ms = kms_total / max(1, launches)
    flop = sum(flops.flops_instance(len(i.footprint), i.N, i.edges, i.obst_off) for i in c5)
    achieved = flop / (kernel_ms * 1e-3) / 1e12
    info = be.info()
    traffic, traffic_note = counted("batch_kernel", "hbm", "traffic_bytes_per_launch", info)
    valu, _ = counted("batch_kernel", "valu", "valu_insts_per_launch", info)
    fp32_insts, _ = counted("batch_kernel", "valu", "fp32_insts_per_launch", info)
    fp32_flop, _ = counted("batch_kernel", "valu", "fp32_flop_per_launch", info)
    cycles = SIMDS * kernel_ms * 1e-3 * CLOCK_GHZ * 1e9
    kname = f"batch_kernel<6, 4, {info['obstacles_per_tile'] // 64}>"
    res = dict(
        metric=METRIC, value=value, unit="stage×edge evals/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=ms_step, higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        timing="K psdf_batch calls (each a replay of the plan's HIP graph) between one event pair",
        config=dict(workload="c5: 64 instances x N=50 path poses x E=65536 edges (16384 rectangles, "
                             "32-component Gaussian mixture, sigma 2 m, 60x60 m), hexagon footprint "
                             "(m=6), psdf_batch (value+winner+gradient)",
                    instances=len(c5), N=50, E=65536, M=16384, m=6, eta=1000.0, pairs=pairs,
                    launch_shape=info),
        roofline=dict(bound="alu", achieved=achieved, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                      frac=achieved / PEAK_FP32_TFLOPS,
                      frac_of_unpacked=achieved / REACHABLE_FP32_TFLOPS,
                      traffic=traffic, traffic_note=traffic_note,
                      algorithmic_bytes=sum(flops.bytes_instance(i.N, i.E, i.M) for i in c5),
                      fp32_issue=None if fp32_insts is None else fp32_insts * 4 / cycles,
                      valu_insts_x4_over_simd_cycles=None if valu is None else valu * 4 / cycles,
                      executed_fp32_tflops=None if fp32_flop is None else fp32_flop / (kernel_ms * 1e-3) / 1e12,
                      valu_insts_per_launch=valu, fp32_insts_per_launch=fp32_insts,
                      kernel=kname, kernel_us=kernel_ms * 1e3,
                      kernel_launches_timed=launches, flop_per_launch=flop,
                      source_sha256=source_hash("batch_kernel", info)),
        wall_s=wall,
    )
    if args.screened:
        res["screened"] = screened_forms(torch, api, inputs, c5, be, ref, args.steps)
    bg.close()
    be.close()
    if args.extras:
        res["extras"] = extras(torch, api, flops, inputs)
        res["extras"]["next_rows"] = next_rows(torch, api, flops, inputs)
    if not args.no_cpu and args.cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(c5, args.cpu_seconds, inputs)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
