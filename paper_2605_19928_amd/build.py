"""Build the HIP library ``libpcfr.so`` in-tree for gfx950.

``python -m paper_2605_19928_amd.build`` compiles every source under
``csrc/`` with hipcc.  Packed-FP32 instructions are disabled for all device
code (``-packed-fp32-ops``).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpcfr.so")
ARCH = os.environ.get("PCFR_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.cpp", "cards.cpp", "tree.cpp", "equity.cpp", "iso.cpp", "solver.hip", "leafnet.hip", "prune.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = OUT + ".tmp"
    cmd = [hipcc, *FLAGS, "-I", os.path.join(HERE, "..", "include"), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
