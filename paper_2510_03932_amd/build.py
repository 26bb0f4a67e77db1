"""Build the gfx950 evaluation library in-tree: ``libocpeval.so`` next to this file.

    python -m paper_2510_03932_amd.build

Compiles the HIP kernels and the host index layer with hipcc for gfx950 only.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libocpeval.so")
SOURCES = [os.path.join(CSRC, "ocp_eval.hip"), os.path.join(CSRC, "ocp_batch.hip"),
           os.path.join(CSRC, "ocp_diff.hip"), os.path.join(CSRC, "ocp_host.cpp"),
           os.path.join(CSRC, "ocp_quad.hip"), os.path.join(CSRC, "ocp_quad_host.cpp"),
           os.path.join(CSRC, "ocp_mapped.hip"), os.path.join(CSRC, "ocp_order_host.cpp"),
           os.path.join(CSRC, "ocp_fused.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
    "-I", CSRC,
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
