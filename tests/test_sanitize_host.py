"""The host index layer and the C oracle under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

``sanitize_host.cpp`` links the library's host sources (sizes, patterns, KKT
structure, stage orderings, symmetric reordering, argument validation) and the
oracle's C source, all compiled with ``-fsanitize=address,undefined``, and
compares the closed-form builders with the oracle's generic ones over a grid
of shapes, both schemes, every boundary option and the quadrotor model; it
also runs the oracle's value functions on small instances.  A sanitizer report
aborts the run, and so does any mismatch.  The host layer makes no HIP call,
so this needs no GPU; it is compiled by g++/gcc against the HIP headers only.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_03932_amd", "csrc")
HOST_SOURCES = ["ocp_host.cpp", "ocp_order_host.cpp", "ocp_quad_host.cpp"]
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
INC = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
       "-I" + CSRC]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs g++ and gcc")


def _build(tmp_path):
    objs = []
    for src in HOST_SOURCES:
        obj = str(tmp_path / (src + ".o"))
        subprocess.check_call(["g++", "-std=c++17", *SAN, *INC, "-c", os.path.join(CSRC, src),
                               "-o", obj])
        objs.append(obj)
    orc = str(tmp_path / "ocp_oracle.o")
    subprocess.check_call(["gcc", "-std=c11", *SAN, "-fopenmp", "-ffp-contract=off", "-c",
                           os.path.join(ROOT, "oracle", "ocp_oracle.c"), "-o", orc])
    drv = str(tmp_path / "sanitize_host.o")
    subprocess.check_call(["g++", "-std=c++17", *SAN, *INC, "-c",
                           os.path.join(ROOT, "tests", "sanitize_host.cpp"), "-o", drv])
    exe = str(tmp_path / "sanitize_host")
    subprocess.check_call(["g++", *SAN, "-fopenmp", drv, *objs, orc, "-o", exe, "-lpthread", "-lm"])
    return exe


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    return env


def test_host_layer_and_oracle_clean_under_asan_ubsan(tmp_path):
    exe = _build(tmp_path)
    res = subprocess.run([exe], capture_output=True, text=True, env=_env(), timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "ok: 102 structure cases" in res.stdout, out[-2000:]


def test_sanitizer_flags_catch_a_planted_overflow(tmp_path):
    """The same flags do report a one-past-the-end heap write, so a clean run
    above means something."""
    src = tmp_path / "oob.cpp"
    src.write_text("#include <vector>\nint main(){std::vector<int> v(8);"
                   " int *p = v.data(); volatile int i = 8; p[i] = 1; return 0;}\n")
    exe = str(tmp_path / "oob")
    subprocess.check_call(["g++", "-std=c++17", *SAN, str(src), "-o", exe])
    res = subprocess.run([exe], capture_output=True, text=True, env=_env(), timeout=60)
    assert res.returncode != 0
    assert "heap-buffer-overflow" in res.stderr
