"""Compile the HIP sources of the package into ``libpsdf.so`` (gfx950).

Each translation unit is compiled to an object in parallel, then linked.
Flags: -O3, -ffp-contract=off (every fused multiply-add is explicit in the
source, so all kernels that share the device arithmetic agree bit for bit),
and packed FP32 instructions disabled for the device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpsdf.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = (["psdf_host.cpp", "psdf_plain.hip", "psdf_batch.hip", "psdf_mlp.hip", "psdf_geom.hip"]
           + [f"psdf_inst_mf{m}.hip" for m in (3, 4, 5, 6, 7, 8, 16)]
           + [f"psdf_batch_mf{m}.hip" for m in (3, 4, 5, 6, 7, 8, 16)]
           + [f"psdf_screen_mf{m}.hip" for m in (3, 4, 5, 6, 7, 8, 16)])

ARCH = os.environ.get("PSDF_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", f"-I{INCLUDE}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return exe


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc()] + COMMON + DEVICE
    if src.endswith(".hip"):
        cmd += ["-x", "hip"]
    cmd += ["-c", path, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = jobs or min(8, len(SOURCES))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
