"""Benchmark of the PSDF hot path on one MI355X.

A step is one psdf_grad call (per-stage minimum over obstacles, winning
obstacle and edge, and the pose gradient) on the 'c2' workload: hexagonal
footprint (circumradius 0.5 m, radii jittered +-10 %), N = 50 stage poses
along a random smooth path, 16384 edges from 4096 random rectangles in a
40 x 40 m square.  Inputs are resident in HBM before the timed region.

Prints one JSON line: value = stage x edge evaluations per second of whole
psdf_grad calls, K calls captured into one HIP graph and replayed (the eager
per-call rate, host launch cost included, is reported beside it); roofline of the dominant (per-stage minimum) kernel from HIP
events on its launch stream (K back-to-back launches between one event pair;
the per-launch event-bracketed figure, which adds the dispatch overhead, is
reported beside it); cpu_baseline = the FP64 oracle on host cores.
"""
from __future__ import annotations

import argparse
import json
import os
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

# HBM bytes per launch of the dominant kernel, from the FETCH_SIZE / WRITE_SIZE
# counter runs recorded in this file (each scaled by the same counter's reading
# for a copy kernel of known size), valid only while the kernel's sources
# hash to the value recorded beside it.
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "main_kernel_c2_hbm_counters.md")
VALU_SUMMARY = os.path.join(ROOT, "profiles", "main_kernel_c2_valu_counters.md")
SIMDS, CLOCK_GHZ = 1024, 2.4
# The per-stage-minimum kernel's own sources: its code and instantiation, the
# launch-shape choice, the build flags.
KERNEL_SOURCES = [os.path.join("paper_2607_04310_amd", "csrc", f) for f in (
    "psdf_device.hpp", "psdf_kernels.hpp", "psdf_winner.hpp", "psdf_inst_mf6.hip",
    "psdf_host.cpp", "psdf_host.hpp")] + [os.path.join("paper_2607_04310_amd", "build.py")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counted_valu_insts():
    """VALU wave-instructions per launch from the VALU counter summary, or
    None when it is missing or the kernel has changed since."""
    import re
    try:
        text = open(VALU_SUMMARY).read()
    except OSError:
        return None
    mh = re.search(r"source_sha256:\s*([0-9a-f]+)", text)
    mv = re.search(r"valu_insts_per_launch:\s*([0-9.eE+]+)", text)
    if not mh or not mv or mh.group(1) != kernel_source_hash():
        return None
    return float(mv.group(1))


def counted_traffic():
    """(bytes per launch, note) from the counter summary, or (None, why not)."""
    import re
    try:
        text = open(COUNTER_SUMMARY).read()
    except OSError:
        return None, "no counter summary"
    mh = re.search(r"source_sha256:\s*([0-9a-f]+)", text)
    mb = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not mh or not mb:
        return None, "counter summary incomplete"
    if mh.group(1) != kernel_source_hash():
        return None, "kernel changed since the counters were taken"
    return float(mb.group(1)), "rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="bound on the CPU-oracle sample (0 disables it)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--counters", action="store_true",
                    help="only launch the c2 psdf_grad call `steps` times and a 256 MiB "
                         "device copy (the calibration of the HBM byte counters)")
    ap.add_argument("--extras", type=int, default=1,
                    help="also measure the uneven batch (c4) and the screened path (c5)")
    return ap.parse_args()


def cpu_baseline(inst, seconds):
    """The FP64 oracle (value, winner, gradient) on all host cores, repeated on
    the same workload until `seconds` of wall time have passed."""
    import oracle
    oracle.psdf(inst.footprint, inst.poses[:1], inst.edges, inst.obst_off)   # load / warm
    done, reps, used = 0.0, 0, 0
    t0 = time.perf_counter()
    while True:
        r = oracle.psdf(inst.footprint, inst.poses, inst.edges, inst.obst_off)
        used = r["threads"]
        reps += 1
        done = time.perf_counter() - t0
        if done >= seconds:
            break
    value = reps * inst.N * inst.E / done
    return dict(value=value, unit="stage×edge evals/s", cores=int(used), kind="oracle",
                sample=f"{reps} full c2 evaluations (N={inst.N}, E={inst.E}, value+winner+gradient, "
                       f"FP64) in {done:.1f} s")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timeit(torch, fn, reps, warm, blocks=1):
    """Mean ms per call over `reps` calls after `warm` untimed ones; with
    blocks > 1, the median over that many such timed blocks."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(blocks):
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b) / reps)
    return sorted(times)[len(times) // 2]


def extras(torch, api, flops, inputs):
    """Secondary lines: the uneven batch (c4: persistent graph vs the
    per-instance loop), c2 at throughput size (256 draws in one batch), one
    pose against growing edge sets, the latency of the paper's Table I query
    shapes, and certified screening (c5: plain batch vs screened with the
    trained MLP and with distance ranking)."""
    from paper_2607_04310_amd import screener
    out = {}
    log("c4: building 512 instances")
    c4 = inputs.c4(512)
    pairs4 = sum(i.N * i.E for i in c4)
    b = api.Batch(c4, graph=True, autotune=True)
    b.autotune()
    log(f"c4: autotuned {b.info()}")
    t_batch = _timeit(torch, b.run, 20, 3)
    views = [b.instance_views(k) for k in range(b.n_inst)]

    def loop():
        for fp, poses, es in views:
            api.psdf_grad(fp, poses, es)
    t_loop = _timeit(torch, loop, 3, 1)
    f4 = sum(flops.flops_instance(len(i.footprint), i.N, i.edges, i.obst_off) for i in c4)
    out["c4_batch"] = dict(pairs=pairs4, batch_ms=t_batch, loop_ms=t_loop,
                           batch_evals_per_s=pairs4 / (t_batch * 1e-3),
                           loop_evals_per_s=pairs4 / (t_loop * 1e-3),
                           batch_tflops=f4 / (t_batch * 1e-3) / 1e12, shape=b.info())
    b.close()

    # c2 at throughput size: 256 independent c2 draws in one batch launch
    log("c2x256: building")
    c2b = inputs.c2_batch(256)
    pairs2 = sum(i.N * i.E for i in c2b)
    b = api.Batch(c2b, graph=True, autotune=True)
    b.autotune()
    t = _timeit(torch, b.run, 20, 3)
    f2 = sum(flops.flops_instance(len(i.footprint), i.N, i.edges, i.obst_off) for i in c2b)
    out["c2x256_batch"] = dict(pairs=pairs2, ms=t, evals_per_s=pairs2 / (t * 1e-3),
                               tflops=f2 / (t * 1e-3) / 1e12, shape=b.info())
    log(f"c2x256: {t:.3f} ms, {pairs2 / (t * 1e-3):.3e} evals/s")
    b.close()
    del c2b

    # one stage pose against growing edge sets: every edge is read once per
    # call, the HBM end of the workload
    sweep = []
    for rects in (1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22):
        inst = inputs.single_pose(rects)
        es = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device="cuda")
        poses = torch.tensor(inst.poses, device="cuda")
        ws = api.workspace(1, inst.M, "cuda")
        o = api.psdf_grad(inst.footprint, poses, es, ws=ws)
        t = _timeit(torch, lambda: api.psdf_grad(inst.footprint, poses, es, out=o, ws=ws), 20, 3)
        nbytes = flops.bytes_instance(1, inst.E, inst.M)
        fl = flops.flops_instance(len(inst.footprint), 1, inst.edges, inst.obst_off)
        sweep.append(dict(E=inst.E, ms=t, evals_per_s=inst.E / (t * 1e-3),
                          gbytes_per_s=nbytes / (t * 1e-3) / 1e9, tflops=fl / (t * 1e-3) / 1e12))
        log(f"single pose E={inst.E}: {t * 1e3:.1f} us, {nbytes / (t * 1e-3) / 1e9:.0f} GB/s")
        del es, poses, ws, o
    out["single_pose_sweep"] = sweep

    # the query shapes of the paper's Table I: latency of one value call
    # (psdf_eval) and one value + gradient call (psdf_grad) for B poses
    # against M obstacles, eager from Python as a per-query caller issues
    # them, and the value + gradient call replayed from a HIP graph
    table = []
    for M in (1, 10, 100):
        for B in (1, 10, 100):
            inst = inputs.table_i(M, B)
            es = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device="cuda")
            poses = torch.tensor(inst.poses, device="cuda")
            ws = api.workspace(B, M, "cuda")
            o = api.psdf_grad(inst.footprint, poses, es, ws=ws)
            t_fwd = _timeit(torch, lambda: api.psdf_eval(inst.footprint, poses, es, ws=ws), 200, 20)
            t_grad = _timeit(torch, lambda: api.psdf_grad(inst.footprint, poses, es, out=o, ws=ws),
                             200, 20)
            cap = torch.cuda.Stream()
            cap.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(cap):
                api.psdf_grad(inst.footprint, poses, es, out=o, ws=ws)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cap):
                for _ in range(100):
                    api.psdf_grad(inst.footprint, poses, es, out=o, ws=ws)
            t_graph = _timeit(torch, g.replay, 5, 1) / 100
            del g
            table.append(dict(M=M, B=B, fwd_us=t_fwd * 1e3, grad_us=t_grad * 1e3,
                              grad_graph_us=t_graph * 1e3))
            del es, poses, ws, o
    log("table I shapes: " + ", ".join(f"M={r['M']} B={r['B']}: {r['grad_us']:.1f} us"
                                       for r in table))
    out["table_i_latency"] = table

    # screener trained on held-out instances (different seeds from the test batch)
    log("c5: training set")
    X, T = screener.training_set(inputs.c5(10, cfg=6), near=1024, far=1024, seed=1)
    log(f"c5: training on {X.shape[0]} pairs")
    theta, hist = screener.train(X, T, epochs=12, batch=4096, lr=2e-3, seed=0, log=log)
    c5 = inputs.c5(64)
    pairs5 = sum(i.N * i.E for i in c5)
    b = api.Batch(c5, graph=True)
    # the first blocks of ten calls of this workload run up to 15 % slower
    # than the later ones (measured: 0.73, 0.68, 0.65, 0.62, 0.62 ms), so
    # these c5 lines warm up for 30 calls and report the median of five blocks
    t_plain = _timeit(torch, b.run, 10, 30, blocks=5)
    res = dict(pairs=pairs5, train_pairs=int(X.shape[0]), train_loss=hist[-1], plain_ms=t_plain,
               plain_evals_per_s=pairs5 / (t_plain * 1e-3))
    ref = [x.clone() for x in (b.d, b.keys)]
    for name, th in (("mlp", theta), ("distance", None)):
        log(f"c5: screened, {name} ranking")
        t = _timeit(torch, lambda: b.screened(th, pool=128, topk=256), 10, 30, blocks=5)
        (d, _, _, _, keys), (cand, cert, ck) = b.screened(th, pool=128, topk=256, stats=True)
        torch.cuda.synchronize()
        exact = bool(torch.equal(keys, ref[1]))
        res[name] = dict(ms=t, evals_per_s=pairs5 / (t * 1e-3), exact=exact,
                         certified=float(cert.float().mean()), mean_candidates=float(cand.float().mean()),
                         winner_recall=float((ck == keys).float().mean()))
    out["c5_screen"] = res
    b.close()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the PSDF hot path has no multi-GPU path "
              "(independent instances would shard across GPUs with no exchange; one huge "
              "instance would shard its obstacles and all-reduce the per-stage minimum keys)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2607_04310_amd import _lib, api, flops, inputs

    dev = torch.device("cuda:0")
    inst = inputs.c2(0)
    edges = api.EdgeSet(inst.edges, inst.obst_off, inst.mbar, device=dev)
    poses = torch.tensor(inst.poses, device=dev)
    N, E, M = inst.N, inst.E, inst.M
    out = (torch.empty(N, device=dev), torch.empty(N, dtype=torch.int32, device=dev),
           torch.empty(N, dtype=torch.int32, device=dev), torch.empty((N, 3), device=dev),
           torch.empty(N, dtype=torch.int64, device=dev))
    params = api.Params()
    ws = api.workspace(N, M, dev)

    def step():
        api.psdf_grad(inst.footprint, poses, edges, params, out=out, ws=ws)

    if args.counters:
        src = torch.ones(64 << 20, device=dev)
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            step()
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(counters_run=True, steps=args.steps, copy_bytes=src.numel() * 4)))
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ref = [x.clone() for x in out]

    # Eager calls from Python, for reference: each call pays the binding's and
    # the HIP runtime's host-side launch cost, which can exceed the GPU time
    # of a call of this size.
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    eager_ms = start.elapsed_time(stop) / args.steps

    # Timed region: the same K whole psdf_grad calls, captured once (outside
    # the timed region) into a HIP graph and replayed once, as a launch-bound
    # loop of small calls is run in deployment.  An untimed replay first, then
    # a check that the replayed calls reproduce the eager outputs bit for bit.
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        step()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=cap):
        for _ in range(args.steps):
            step()
    for x in out:
        x.zero_()
    graph.replay()
    torch.cuda.synchronize()
    if not all(torch.equal(a, b) for a, b in zip(out, ref)):
        raise RuntimeError("graph replay of psdf_grad differs from the eager call")
    t0 = time.perf_counter()
    start.record()
    graph.replay()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = start.elapsed_time(stop) / args.steps
    del graph

    # The dominant kernel alone: the same steps' per-stage-minimum launches
    # with an event pair around each (dispatch overhead included), and
    # back-to-back launches between one event pair on the launch stream.
    _lib.timer_enable(args.steps)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    kms, launches = _lib.timer_read()
    _lib.timer_enable(0)
    kernel_ms_bracketed = kms / max(1, launches)
    kernel_ms = api.time_stage_min(inst.footprint, poses, edges, args.steps, params, ws=ws)

    flop = flops.flops_instance(len(inst.footprint), N, inst.edges, inst.obst_off)
    achieved = flop / (kernel_ms * 1e-3) / 1e12
    traffic, traffic_note = counted_traffic()
    valu = counted_valu_insts()
    valu_busy = None if valu is None else valu * 4 / (SIMDS * kernel_ms * 1e-3 * CLOCK_GHZ * 1e9)
    value = N * E / (ms_step * 1e-3)
    res = dict(
        metric=METRIC, value=value, unit="stage×edge evals/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=ms_step, eager_ms_per_step=eager_ms,
        eager_value=N * E / (eager_ms * 1e-3), timing="one HIP graph replay of the K calls",
        higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="c2: hexagon footprint (m=6), N=50 path poses, E=16384 edges "
                             "(4096 rectangles, 40x40 m), psdf_grad (value+winner+gradient)",
                    N=N, E=E, M=M, m=len(inst.footprint), eta=params.eta),
        roofline=dict(bound="alu", achieved=achieved, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                      frac=achieved / PEAK_FP32_TFLOPS,
                      frac_of_unpacked=achieved / REACHABLE_FP32_TFLOPS, traffic=traffic,
                      traffic_note=traffic_note,
                      algorithmic_bytes=flops.bytes_instance(N, E, M),
                      valu_busy=valu_busy, valu_insts_per_launch=valu,
                      kernel="main_kernel (per-stage minimum)", kernel_us=kernel_ms * 1e3,
                      kernel_us_event_bracketed=kernel_ms_bracketed * 1e3,
                      flop_per_launch=flop, source_sha256=kernel_source_hash()),
        wall_s=wall,
    )
    log(f"c2: {value:.3e} evals/s, {ms_step * 1e3:.2f} us per call (graph replay), "
        f"{eager_ms * 1e3:.2f} us per eager call")
    if args.extras:
        res["extras"] = extras(torch, api, flops, inputs)
    if not args.no_cpu and args.cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
