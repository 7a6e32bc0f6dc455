"""Build the HIP library libpencilfft.so in-tree for gfx950 with hipcc.

Usage: python -m paper_1905_02803_amd.build   (or build() from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpencilfft.so")
SOURCES = ["capi.hip", "kernels.hip", "kernels_p2.hip", "kernels_mr.hip",
           "kernels_mr_p0.hip", "kernels_mr_p1.hip", "kernels_mr_p2.hip", "kernels_mr_p3.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, out: str = LIB, extra=()) -> str:
    """Compile every source to an object, link the shared library, return its path."""
    objs = []
    bdir = os.path.join(os.path.dirname(out), "_build")
    os.makedirs(bdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    procs = []
    for src in SOURCES:  # the sources compile concurrently
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = [HIPCC] + FLAGS + list(extra) + inc + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
