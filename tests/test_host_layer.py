"""The library's host side, without a GPU: it loads, exports every declared
entry point, validates arguments before any HIP call, and its closed-form
pattern and KKT index builders equal the oracle's generic sort-based build
bit for bit."""
from __future__ import annotations

import ctypes
import os
import re
import sys

import numpy as np
import pytest

import paper_2510_03932_amd as ocp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

GRID = [(1, 1, 0), (1, 1, 1), (2, 1, 0), (3, 2, 0), (2, 2, 1), (5, 3, 0), (4, 3, 1), (3, 4, 2),
        (7, 5, 3), (10, 6, 3), (1, 16, 8), (33, 16, 8), (17, 32, 32), (1000, 4, 2), (999, 8, 4)]


def test_library_exports_every_declared_symbol():
    L = ocp.lib()
    names = ocp.exported_names()
    assert len(names) == 54, names
    for name in names:
        assert hasattr(L, name), name
    text = open(ocp.HEADER).read()
    # every entry point documents its arguments in a comment right above it
    for name in names:
        assert re.search(r"\*/\s*\n(?:[^\n]*\n)?[^\n]*\b" + name + r"\s*\(", text), name


@pytest.mark.parametrize("N,n,m", GRID)
def test_sizes_match_oracle(orc, N, n, m):
    s = ocp.sizes(N, n, m)
    o = orc.sizes(N, n, m)
    for k in ("nvar", "ncon", "nnzj", "nnzh", "dim", "npair", "T", "S"):
        assert s[k] == o[k], k
    assert s["nnzk"] == o["nnzh"] + o["nnzj"] + o["ncon"]


@pytest.mark.parametrize("N,n,m", GRID)
def test_pattern_bit_exact(orc, N, n, m):
    got = ocp.pattern(N, n, m)
    want = orc.pattern(N, n, m)
    for g, w in zip(got, want):
        assert g.dtype == np.int32
        assert np.array_equal(g, w)


@pytest.mark.parametrize("N,n,m", GRID)
def test_kkt_bit_exact(orc, N, n, m):
    got = ocp.kkt_pattern(N, n, m)
    want = orc.kkt(N, n, m)
    for name, g, w in zip(("rowptr", "colind", "perm_j", "perm_h"), got, want):
        assert g.dtype == np.int32
        assert np.array_equal(g, w), name


@pytest.mark.slow
def test_kkt_bit_exact_ipm_loop_size(orc):
    """The 1e5-interval, n = 8, m = 4 workload: 2.2e7 KKT entries."""
    N, n, m = 100_000, 8, 4
    got = ocp.kkt_pattern(N, n, m)
    want = orc.kkt(N, n, m)
    for name, g, w in zip(("rowptr", "colind", "perm_j", "perm_h"), got, want):
        assert np.array_equal(g, w), name


def test_kkt_partial_outputs():
    N, n, m = 50, 3, 1
    full = ocp.kkt_pattern(N, n, m)
    part = ocp.kkt_pattern(N, n, m, rowptr=False, colind=False)
    assert part[0] is None and part[1] is None
    assert np.array_equal(part[2], full[2]) and np.array_equal(part[3], full[3])


@pytest.mark.parametrize("N,n,m,code", [
    (0, 4, 2, ocp.OCP_ERR_ARG), (-5, 4, 2, ocp.OCP_ERR_ARG), (10, 0, 2, ocp.OCP_ERR_ARG),
    (10, 33, 2, ocp.OCP_ERR_ARG), (10, 4, -1, ocp.OCP_ERR_ARG), (10, 4, 33, ocp.OCP_ERR_ARG),
    (2**31, 1, 0, ocp.OCP_ERR_OVERFLOW), (10_000_000, 16, 8, ocp.OCP_ERR_OVERFLOW),
    (2_700_000, 16, 8, ocp.OCP_ERR_OVERFLOW),
])
def test_size_errors(N, n, m, code):
    with pytest.raises(ocp.OcpError) as e:
        ocp.sizes(N, n, m)
    assert e.value.code == code
    assert str(e.value).strip()
    # the builders validate on their own, before touching any output
    assert ocp.lib().ocp_build_kkt(N, n, m, None, None, None, None) == code
    assert ocp.lib().ocp_build_pattern(N, n, m, None, None, None, None) == code


def test_largest_workload_fits_int32():
    s = ocp.sizes(1_000_000, 16, 8)
    assert s["nnzk"] == 824_000_040 and s["nnzj"] == 768_000_000 and s["nnzh"] == 40_000_040
    assert s["dim"] == 40_000_024


def test_create_rejects_bad_arguments_before_any_hip_call():
    """These fail validation on the host, so they are safe without a GPU."""
    L = ocp.lib()
    h = ctypes.c_void_p()
    A = np.zeros((4, 4))
    g = np.zeros(4)
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
    assert L.ocp_create(0, 4, 2, ptr(A), None, ptr(g), ptr(g), None, ctypes.byref(h)) == ocp.OCP_ERR_ARG
    assert b"N must be" in L.ocp_last_error()
    assert L.ocp_create(10, 4, 2, ptr(A), None, ptr(g), ptr(g), None, ctypes.byref(h)) == ocp.OCP_ERR_ARG
    assert b"NULL" in L.ocp_last_error()
    assert L.ocp_create(10, 4, 0, None, None, ptr(g), ptr(g), None, ctypes.byref(h)) == ocp.OCP_ERR_ARG
    assert L.ocp_create(10, 4, 0, ptr(A), None, ptr(g), ptr(g), None, None) == ocp.OCP_ERR_ARG
    bad = A.copy()
    bad[1, 2] = np.nan
    assert L.ocp_create(10, 4, 0, ptr(bad), None, ptr(g), ptr(g), None, ctypes.byref(h)) == ocp.OCP_ERR_ARG
    assert h.value is None
    # every evaluation rejects a NULL handle
    for name in ("ocp_eval_obj", "ocp_eval_grad", "ocp_eval_cons", "ocp_eval_jac"):
        assert getattr(L, name)(None, None, None, None) == ocp.OCP_ERR_ARG
    assert L.ocp_eval_hess(None, None, None, 1.0, None, None) == ocp.OCP_ERR_ARG
    assert L.ocp_assemble_kkt(None, None, None, None, None, None, None, None, None) == ocp.OCP_ERR_ARG
    L.ocp_destroy(None)  # NULL-safe


def test_batch_create_rejects_bad_arguments_before_any_hip_call():
    L = ocp.lib()
    h = ctypes.c_void_p()
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
    A = np.zeros((2, 3, 3))
    g = np.zeros((2, 3))
    Ns = np.array([10, 20], np.int64)
    assert L.ocp_batch_create(0, ptr(Ns), 3, 0, ptr(A), None, ptr(g), ptr(g), None, ctypes.byref(h)) == ocp.OCP_ERR_ARG
    assert L.ocp_batch_create(2, None, 3, 0, ptr(A), None, ptr(g), ptr(g), None, ctypes.byref(h)) == ocp.OCP_ERR_ARG
    assert L.ocp_batch_create(2, ptr(Ns), 3, 1, ptr(A), None, ptr(g), ptr(g), None, ctypes.byref(h)) == ocp.OCP_ERR_ARG
    assert L.ocp_batch_create(2, ptr(Ns), 0, 0, ptr(A), None, ptr(g), ptr(g), None, ctypes.byref(h)) == ocp.OCP_ERR_ARG
    bad = np.array([10, 0], np.int64)
    assert L.ocp_batch_create(2, ptr(bad), 3, 0, ptr(A), None, ptr(g), ptr(g), None, ctypes.byref(h)) == ocp.OCP_ERR_ARG
    assert b"instance 1" in L.ocp_last_error()
    huge = np.array([10, 10_000_000], np.int64)
    assert L.ocp_batch_create(2, ptr(huge), 16, 8, ptr(np.zeros((2, 16, 16))), ptr(np.zeros((2, 16, 8))),
                              ptr(np.zeros((2, 16))), ptr(np.zeros((2, 16))), ptr(np.zeros((2, 8))),
                              ctypes.byref(h)) == ocp.OCP_ERR_OVERFLOW
    assert h.value is None
    cfg = ocp.BatchConfig(256, 1, 8, 0)
    assert L.ocp_batch_set_config(None, ctypes.byref(cfg)) == ocp.OCP_ERR_ARG
    assert L.ocp_batch_eval(None, 3, 0, None, None, 1.0, None, None, None) == ocp.OCP_ERR_ARG
    assert L.ocp_graph_launch(None, None) == ocp.OCP_ERR_ARG
    L.ocp_batch_destroy(None)
    L.ocp_graph_destroy(None)


EX_GRID = [(1, 1, 0), (2, 1, 1), (3, 2, 0), (4, 3, 1), (7, 5, 3), (1, 16, 8), (33, 16, 8),
           (17, 32, 32), (1000, 4, 2), (999, 8, 4)]


@pytest.mark.parametrize("scheme,bnd", [(s, b) for s in (0, 1) for b in (0, 1, 2)])
@pytest.mark.parametrize("N,n,m", EX_GRID)
def test_ex_sizes_patterns_kkt_bit_exact(orc, N, n, m, scheme, bnd):
    s = ocp.sizes(N, n, m, scheme, bnd)
    o = orc.sizes_ex(N, n, m, scheme, bnd)
    for k in ("nvar", "ncon", "nnzj", "nnzh", "dim", "npair", "T", "S"):
        assert s[k] == o[k], k
    for g, w in zip(ocp.pattern(N, n, m, scheme=scheme, boundary=bnd), orc.pattern_ex(N, n, m, scheme, bnd)):
        assert np.array_equal(g, w)
    got = ocp.kkt_pattern(N, n, m, scheme=scheme, boundary=bnd)
    want = orc.kkt_ex(N, n, m, scheme, bnd)
    for name, g, w in zip(("rowptr", "colind", "perm_j", "perm_h"), got, want):
        assert np.array_equal(g, w), name


def test_ex_rejects_unknown_options():
    for scheme, bnd in ((2, 0), (-1, 0), (0, 3), (0, -1)):
        with pytest.raises(ocp.OcpError) as e:
            ocp.sizes(10, 3, 1, scheme, bnd)
        assert e.value.code == ocp.OCP_ERR_ARG


# ---- the quadrotor model -------------------------------------------------------

@pytest.mark.parametrize("bnd", [0, 1, 2])
@pytest.mark.parametrize("N", [1, 2, 3, 64, 255, 1000, 4097])
def test_quad_sizes_patterns_kkt_bit_exact(orc, N, bnd):
    s = ocp.quad_sizes(N, bnd)
    o = orc.quad_sizes(N, bnd)
    for k in ("nvar", "ncon", "nnzj", "nnzh", "dim"):
        assert s[k] == o[k], k
    assert s["nnzk"] == s["nnzh"] + s["nnzj"] + s["ncon"]
    assert (s["T"], s["S"], s["npair"]) == (68, 23, 0)
    for g, w in zip(ocp.quad_pattern(N, bnd), orc.quad_pattern(N, bnd)):
        assert np.array_equal(g, w)
    got = ocp.quad_kkt_pattern(N, bnd)
    want = orc.quad_kkt(N, bnd)
    for name, g, w in zip(("rowptr", "colind", "perm_j", "perm_h"), got, want):
        assert np.array_equal(g, w), name


def test_quad_kkt_bit_exact_paper_grid(orc):
    """The paper's largest quadrotor grid, N = 2e5, with the initial-state rows."""
    got = ocp.quad_kkt_pattern(200_000, 1)
    want = orc.quad_kkt(200_000, 1)
    for name, g, w in zip(("rowptr", "colind", "perm_j", "perm_h"), got, want):
        assert np.array_equal(g, w), name


def test_quad_partial_outputs():
    full = ocp.quad_kkt_pattern(50, 2)
    part = ocp.quad_kkt_pattern(50, 2, rowptr=False, perm_h=False)
    assert part[0] is None and part[3] is None
    assert np.array_equal(part[1], full[1]) and np.array_equal(part[2], full[2])
    jr, jc, hr, hc = ocp.quad_pattern(50, 2, hess=False)
    assert hr is None and np.array_equal(jc, ocp.quad_pattern(50, 2)[1])


def test_quad_rejects_bad_arguments_before_any_hip_call():
    L = ocp.lib()
    h = ctypes.c_void_p()
    for N, bnd in ((0, 1), (-5, 0), (10, 3), (10, -1)):
        with pytest.raises(ocp.OcpError) as e:
            ocp.quad_sizes(N, bnd)
        assert e.value.code == ocp.OCP_ERR_ARG
        assert L.ocp_quad_create(N, bnd, 9.8, 0.1, ctypes.byref(h)) == ocp.OCP_ERR_ARG
    assert L.ocp_quad_create(10, 1, float("nan"), 0.1, ctypes.byref(h)) == ocp.OCP_ERR_ARG
    assert L.ocp_quad_create(10, 1, 9.8, float("inf"), ctypes.byref(h)) == ocp.OCP_ERR_ARG
    assert L.ocp_quad_create(10, 1, 9.8, 0.1, None) == ocp.OCP_ERR_ARG
    assert h.value is None
    with pytest.raises(ocp.OcpError) as e:
        ocp.quad_sizes(400_000_000, 1)
    assert e.value.code == ocp.OCP_ERR_OVERFLOW


# ---- symmetric reordering ---------------------------------------------------------

def _symbolic_fill(rowptr, colind):
    """Entries of L in an LDL^T factorization without pivoting, by symbolic
    elimination of the symmetric pattern (the definition of fill)."""
    dim = len(rowptr) - 1
    M = np.zeros((dim, dim), bool)
    rows = np.repeat(np.arange(dim), np.diff(rowptr))
    M[rows, colind] = True
    M[colind, rows] = True
    total = 0
    for k in range(dim):
        nb = np.flatnonzero(M[k, k + 1:]) + k + 1
        total += len(nb)
        if len(nb):
            M[np.ix_(nb, nb)] = True
    return total


@pytest.mark.parametrize("n,m,scheme,bnd", [(3, 2, 0, 0), (3, 2, 1, 2), (4, 1, 0, 1), (2, 0, 0, 2)])
def test_stage_order_is_fill_reducing(n, m, scheme, bnd):
    """Under the node-grouped ordering the LDL^T fill grows linearly in N
    (equal increments per doubling step once N is past the boundary effects),
    while in the natural order it grows faster."""
    fills, natural = [], []
    for N in (8, 16, 32):
        rp, ci, pj, ph = ocp.kkt_pattern(N, n, m, scheme=scheme, boundary=bnd)
        order = ocp.stage_order(N, n, m, scheme, bnd)
        assert np.array_equal(np.sort(order), np.arange(len(rp) - 1))
        rp2, ci2, _, _, _ = ocp.kkt_permute(rp, ci, pj, ph, order)
        fills.append(_symbolic_fill(rp2, ci2))
        natural.append(_symbolic_fill(rp, ci))
    per_node = [(fills[1] - fills[0]) / 8, (fills[2] - fills[1]) / 16]
    assert per_node[0] == per_node[1], fills
    # linear growth would add twice as much from 16 to 32 nodes as from 8 to 16
    assert (natural[2] - natural[1]) / (natural[1] - natural[0]) > 2.5, natural
    assert fills[2] < natural[2]


@pytest.mark.parametrize("N", [10, 100, 1000])
def test_stage_order_bandwidth_independent_of_N(N):
    n, m = 4, 2
    rp, ci, pj, ph = ocp.kkt_pattern(N, n, m, boundary=2)
    rp2, ci2, _, _, _ = ocp.kkt_permute(rp, ci, pj, ph, ocp.stage_order(N, n, m, 0, 2))
    rows = np.repeat(np.arange(len(rp2) - 1), np.diff(rp2))
    # a node block has n + m + n rows (plus n boundary rows at the ends); an
    # entry reaches at most into the previous block
    assert int((rows - ci2).max()) < 2 * (2 * n + m) + n


@pytest.mark.parametrize("N,n,m,scheme,bnd", [(1, 1, 0, 0, 0), (2, 3, 1, 1, 2), (7, 5, 3, 0, 1),
                                              (33, 16, 8, 1, 0), (1000, 4, 2, 0, 2)])
def test_kkt_permute_bit_exact(orc, N, n, m, scheme, bnd):
    rp, ci, pj, ph = ocp.kkt_pattern(N, n, m, scheme=scheme, boundary=bnd)
    orders = [ocp.stage_order(N, n, m, scheme, bnd),
              np.random.default_rng(N).permutation(len(rp) - 1).astype(np.int32)]
    for order in orders:
        got = ocp.kkt_permute(rp, ci, pj, ph, order)
        want = orc.kkt_permute(rp, ci, pj, ph, order)
        for name, g, w in zip(("rowptr", "colind", "perm_j", "perm_h", "diag"), got, want):
            assert np.array_equal(g, w), name


@pytest.mark.parametrize("N,bnd", [(1, 0), (5, 2), (300, 1)])
def test_quad_stage_order_and_permute(orc, N, bnd):
    order = ocp.quad_stage_order(N, bnd)
    rp, ci, pj, ph = ocp.quad_kkt_pattern(N, bnd)
    assert np.array_equal(np.sort(order), np.arange(len(rp) - 1))
    got = ocp.kkt_permute(rp, ci, pj, ph, order)
    want = orc.kkt_permute(rp, ci, pj, ph, order)
    for name, g, w in zip(("rowptr", "colind", "perm_j", "perm_h", "diag"), got, want):
        assert np.array_equal(g, w), name


def test_kkt_permute_rejects_bad_input():
    rp, ci, pj, ph = ocp.kkt_pattern(6, 3, 1)
    dim = len(rp) - 1
    bad = np.arange(dim, dtype=np.int32)
    bad[2] = bad[4]
    for order in (bad, np.arange(1, dim + 1, dtype=np.int32)):
        with pytest.raises(ocp.OcpError) as e:
            ocp.kkt_permute(rp, ci, pj, ph, order)
        assert e.value.code == ocp.OCP_ERR_ARG
    ident = np.arange(dim, dtype=np.int32)
    pj_bad = pj.copy()
    pj_bad[3] = rp[-1]
    with pytest.raises(ocp.OcpError) as e:
        ocp.kkt_permute(rp, ci, pj_bad, ph, ident)
    assert e.value.code == ocp.OCP_ERR_ARG
    ci_bad = ci.copy()
    ci_bad[0] = dim - 1  # above the diagonal of row 0
    with pytest.raises(ocp.OcpError) as e:
        ocp.kkt_permute(rp, ci_bad, pj, ph, ident)
    assert e.value.code == ocp.OCP_ERR_ARG
    with pytest.raises(ocp.OcpError):
        ocp.stage_order(0, 3, 1)


def test_newer_entry_points_reject_null_handles_before_any_hip_call():
    L = ocp.lib()
    c = ctypes.c_int64()
    assert L.ocp_mapped_plan_size(None, ctypes.byref(c)) == ocp.OCP_ERR_ARG
    assert L.ocp_mapped_plan(None, None, None, None, None, None) == ocp.OCP_ERR_ARG
    assert L.ocp_assemble_kkt_mapped(None, None, None, None, None, None, None, None, None, None) == ocp.OCP_ERR_ARG
    assert L.ocp_eval_kkt(None, None, None, 1.0, None, None, None) == ocp.OCP_ERR_ARG
    for name in ("ocp_eval_obj", "ocp_eval_grad", "ocp_eval_cons", "ocp_eval_jac"):
        assert getattr(L, name)(None, None, None, None) == ocp.OCP_ERR_ARG
    assert L.ocp_stage_order(10, 3, 1, None, None) == ocp.OCP_ERR_ARG
    assert L.ocp_quad_stage_order(10, 1, None) == ocp.OCP_ERR_ARG
    assert L.ocp_quad_sizes(10, 1, None) == ocp.OCP_ERR_ARG
    assert L.ocp_kkt_permute(0, None, None, 0, None, 0, None, None, None, None, None, None, None) == ocp.OCP_ERR_ARG
    assert b"ocp_kkt_permute" in L.ocp_last_error()


def test_quad_pattern_and_kkt_partial_outputs_match_full():
    """NULL outputs are skipped without touching the others (host only)."""
    full = ocp.quad_pattern(40, 1)
    jr, jc, hr, hc = ocp.quad_pattern(40, 1, jac=True, hess=False)
    assert np.array_equal(jr, full[0]) and np.array_equal(jc, full[1]) and hr is None and hc is None
    rp, ci, pj, ph = ocp.quad_kkt_pattern(40, 1, colind=False, perm_h=False)
    full = ocp.quad_kkt_pattern(40, 1)
    assert ci is None and ph is None
    assert np.array_equal(rp, full[0]) and np.array_equal(pj, full[2])


def test_verbose_errors_go_to_stderr(tmp_path):
    """OCP_VERBOSE=1 echoes every recorded error to stderr; unset, nothing is
    printed (a child process, since the variable is read once)."""
    import subprocess
    import textwrap
    script = textwrap.dedent("""
        import ctypes, sys
        sys.path.insert(0, %r)
        import paper_2510_03932_amd as ocp
        s = ocp.Sizes()
        rc = ocp.lib().ocp_sizes(0, 4, 2, ctypes.byref(s))
        print("rc", rc)
    """ % ROOT)
    env = dict(os.environ, OCP_VERBOSE="1")
    on = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=120)
    assert "rc 1" in on.stdout and "[ocp] error 1: N must be >= 1" in on.stderr, on.stderr
    env.pop("OCP_VERBOSE")
    off = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=120)
    assert "rc 1" in off.stdout and "[ocp]" not in off.stderr
