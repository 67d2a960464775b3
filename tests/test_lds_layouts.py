"""The LDS layout arithmetic of the streamed kernels, checked on the host:
tests/lds_layout_check.cpp (built with hipcc; only its host code runs) checks
every exchange of the fused transforms of 256..2048 points: the
base-plus-offset addressing equals the position of the full index, the
padded layouts are injective within their row length, and the chosen pads
keep each pass's writes free of bank conflicts."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1810_02821_amd", "csrc")


def test_lds_layouts_hold(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "lds_layout_check")
    cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", CSRC, os.path.join(HERE, "lds_layout_check.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-2000:]
    assert " 0 failures" in r.stdout
