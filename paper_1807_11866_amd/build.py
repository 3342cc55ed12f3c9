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


FLAGS = ["-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-pragma-unroll-threshold=1000000",
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def build(verbose=False, extra=(), jobs=None, incremental=False):
    """Compile every csrc/*.hip translation unit (in parallel) and link librbns.so.

    incremental=True keeps the objects under _build/ and recompiles only the translation
    units older than their source or any header (a development shortcut; the default
    rebuilds everything).
    """
    from concurrent.futures import ThreadPoolExecutor

    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    headers = (glob.glob(os.path.join(CSRC, "*.hpp")) +
               glob.glob(os.path.join(HERE, "..", "include", "*.h")))
    newest_header = max(os.path.getmtime(h) for h in headers)
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(HERE, "..", "include")]

    def compile_one(src):
        name = os.path.basename(src)
        if incremental:
            obj = os.path.join(objdir, name + ".o")
            if (os.path.exists(obj) and
                    os.path.getmtime(obj) > max(os.path.getmtime(src), newest_header)):
                return obj
        else:
            obj = os.path.join(objdir, name + f".{os.getpid()}.o")
        tmp = obj + ".tmp"
        cmd = [hipcc(), f"--offload-arch={ARCH}", *FLAGS, *inc, *extra, "-c", src, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, obj)
        return obj

    jobs = jobs or min(len(srcs), max(1, os.cpu_count() or 1), 16)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                   check=True)
    if not incremental:
        for o in objs:
            os.remove(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
