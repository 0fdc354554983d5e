"""Build the HIP library ``libpcfr.so`` in-tree for gfx950.

``python -m paper_2605_19928_amd.build`` compiles every source under
``csrc/`` with hipcc (one object per source, compiled in parallel, then
linked).  Packed-FP32 instructions are disabled for all device code
(``-packed-fp32-ops``).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libpcfr.so")
ARCH = os.environ.get("PCFR_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.cpp", "cards.cpp", "tree.cpp", "equity.cpp", "iso.cpp", "solver.hip", "leafnet.hip", "prune.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    inc = os.path.join(HERE, "..", "include")

    def compile_one(src: str) -> str:
        obj = os.path.join(OBJ, src + ".o")
        cmd = [hipcc, *FLAGS, "-I", inc, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
