"""Build the gfx950 shared library librbns.so in-tree with hipcc.

    python -m paper_1807_11866_amd.build

Every HIP translation unit under csrc/ is compiled for gfx950 only, with packed-FP32
instructions disabled, and linked into paper_1807_11866_amd/librbns.so.
"""

from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librbns.so")
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, extra=()):
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-mllvm", "-pragma-unroll-threshold=1000000",
           "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
           "-I", os.path.join(HERE, "..", "include"), "-o", tmp, *srcs, *extra]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
