"""Every workgroup barrier of the library's kernels sits in lane-uniform control flow.

A barrier inside a loop whose exit the compiler implements with exec masks
(a lane-divergent loop) can be executed a different number of times by the
wavefronts of one workgroup, which deadlocks the workgroup.  The kernels are
written so that every loop holding a barrier is steered by wave-uniform
values; this test compiles them for gfx950 and checks the generated code
(no GPU needed).
"""
import os
import shutil
import subprocess

import pytest

from barrier_check import report

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_1201_4060_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", ["eval.hip", "hessian.hip", "batch.hip", "fft.hip"])
def test_barriers_only_in_uniform_loops(src, tmp_path):
    asm = tmp_path / (src + ".s")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", str(asm)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    rows = report(str(asm))
    assert rows, "no kernel with a barrier found"
    bad = [(name, nb, nbad) for name, nb, nbad in rows if nbad]
    assert not bad, f"barriers in lane-divergent loops: {bad}"
