"""Build libmf.so for gfx950 with hipcc (in-tree, next to this file).

Every source is compiled to an object in parallel (one hipcc per file), then
the objects are linked into the shared library."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libmf.so")

# Packed FP32 instructions are disabled for every HIP translation unit.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    c = os.path.join(HERE, "csrc")
    return sorted(glob.glob(os.path.join(c, "*.hip"))) + sorted(glob.glob(os.path.join(c, "*.cpp")))


def _jobs() -> int:
    try:
        n = int(os.environ.get("MAX_JOBS", "0"))
    except ValueError:
        n = 0
    return max(1, min(16, n if n > 0 else (os.cpu_count() or 4)))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
    return r.returncode


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = "-I" + os.path.join(ROOT, "include")
    with tempfile.TemporaryDirectory(prefix="mf_build_") as tmpd:
        srcs = sources()
        objs = [os.path.join(tmpd, os.path.basename(s) + ".o") for s in srcs]
        lang = lambda s: ["-x", "hip"] if s.endswith(".hip") else []
        cmds = [[hipcc, *HIP_FLAGS, inc, *lang(s), "-c", s, "-o", o] for s, o in zip(srcs, objs)]
        with ThreadPoolExecutor(_jobs()) as ex:
            rcs = list(ex.map(lambda c: _run(c, verbose), cmds))
        if any(rcs):
            raise RuntimeError("hipcc failed to compile a source of libmf.so")
        tmp = OUT + ".tmp"
        if _run([hipcc, *HIP_FLAGS, "-shared", *objs, "-o", tmp], verbose):
            raise RuntimeError("hipcc failed to link libmf.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
