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
COMPILE_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
    "-I", CSRC,
]
# kept for callers that want the single-command form
FLAGS = [*COMPILE_FLAGS, "-shared"]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source to an object (in parallel, one hipcc per source),
    then link the shared library.  Always recompiles."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(src) + ".o") for src in SOURCES]
    cmds = [[HIPCC, *COMPILE_FLAGS, "-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1, 16))

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd).returncode

    with ThreadPoolExecutor(max_workers=jobs) as pool:
        codes = list(pool.map(run, cmds))
    bad = [os.path.basename(src) for src, rc in zip(SOURCES, codes) if rc != 0]
    if bad:
        raise RuntimeError(f"hipcc failed for {', '.join(bad)}")
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
