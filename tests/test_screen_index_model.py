"""The screening kernels' work-group index arithmetic (the reductions, the
threshold search with its alternating halves, the pool and candidate
compactions of both screened forms, the horizon list append), restated for
a 256-lane work-group on the host with arrays of the kernels' sizes, under
the host address and undefined-behaviour sanitizers: every pool size the
ABI allows, top-K from 1 to past the slot count, horizon lists of 0..2048
entries, the three edge classes, keys with ties, unused slots, -inf and NaN.
Every index must stay in its array, every threshold search must end, every
compaction must write each slot once."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_screen_index_arithmetic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "screen_index_model")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "sanitize", "screen_index_model.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok "), r.stdout + r.stderr
