"""Benchmark of the PSDF hot path on one MI355X.

A step is one psdf_grad call (per-stage minimum over obstacles, winning
obstacle and edge, and the pose gradient) on the 'c2' workload: hexagonal
footprint (circumradius 0.5 m, radii jittered +-10 %), N = 50 stage poses
along a random smooth path, 16384 edges from 4096 random rectangles in a
40 x 40 m square.  Inputs are resident in HBM before the timed region.

Prints one JSON line: value = stage x edge evaluations per second of whole
psdf_grad calls; roofline of the dominant (per-stage minimum) kernel from HIP
events on its launch stream; cpu_baseline = the FP64 oracle on host cores.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="bound on the CPU-oracle sample (0 disables it)")
    ap.add_argument("--no-cpu", action="store_true")
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


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the PSDF hot path has no multi-GPU "
              "path in this build (see DESIGN.md for how it would shard)", file=sys.stderr)
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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # Timed region: K whole psdf_grad calls.
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = start.elapsed_time(stop) / args.steps

    # Same launches again with the library's event pairs around the dominant kernel.
    _lib.timer_enable(args.steps)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    kms, launches = _lib.timer_read()
    _lib.timer_enable(0)
    kernel_ms = kms / max(1, launches)

    flop = flops.flops_instance(len(inst.footprint), N, inst.edges, inst.obst_off)
    achieved = flop / (kernel_ms * 1e-3) / 1e12
    value = N * E / (ms_step * 1e-3)
    res = dict(
        metric=METRIC, value=value, unit="stage×edge evals/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=ms_step, higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="c2: hexagon footprint (m=6), N=50 path poses, E=16384 edges "
                             "(4096 rectangles, 40x40 m), psdf_grad (value+winner+gradient)",
                    N=N, E=E, M=M, m=len(inst.footprint), eta=params.eta),
        roofline=dict(bound="alu", achieved=achieved, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                      frac=achieved / PEAK_FP32_TFLOPS, traffic=None,
                      kernel="main_kernel (per-stage minimum)", kernel_us=kernel_ms * 1e3,
                      flop_per_launch=flop),
        wall_s=wall,
    )
    if not args.no_cpu and args.cpu_seconds > 0:
        res["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
