"""The one-time host symbolic step (paper Sec. 6) at the sizes the benchmarks
run: the library's closed-form COO patterns, KKT CSR structure and slot maps
equal the oracle's generic sort-based build bit for bit, in full, for

* the 1e6-interval, n = 16, m = 8 trapezoidal problem (768,000,000 Jacobian
  and 40,000,040 Hessian entries, 824,000,040 KKT slots), which the headline
  evaluation and assembly use;
* the same grid under forward Euler with initial and final boundary rows;
* the quadrotor model at 1e6 intervals with initial-state rows.

Without these, the GPU tests at those sizes could only check the maps
against themselves (kkt[perm_j[e]] == jac[e]), which a wrong but injective
map would pass.  CPU only; the trapezoidal case peaks at about 27 GB of host
memory and takes about a minute in the oracle's single-threaded build.
"""
from __future__ import annotations

import gc

import numpy as np
import pytest

import paper_2510_03932_amd as ocp

pytestmark = pytest.mark.slow


def _same(got, want, names):
    for name, g, w in zip(names, got, want):
        assert g.dtype == np.int32 and w.dtype == np.int32, name
        assert g.shape == w.shape, name
        assert np.array_equal(g, w), name


def test_full_size_trapezoidal_structure(orc):
    N, n, m = 1_000_000, 16, 8
    s = ocp.sizes(N, n, m)
    assert (s["nnzj"], s["nnzh"], s["nnzk"]) == (768_000_000, 40_000_040, 824_000_040)
    pat = orc.pattern(N, n, m)
    got = ocp.pattern(N, n, m)
    _same(got, pat, ("jrow", "jcol", "hrow", "hcol"))
    del got
    gc.collect()
    want = orc.kkt(N, n, m, pat=pat)
    del pat
    gc.collect()
    got = ocp.kkt_pattern(N, n, m)
    _same(got, want, ("rowptr", "colind", "perm_j", "perm_h"))


def test_full_size_euler_boundary_structure(orc):
    N, n, m = 1_000_000, 16, 8
    scheme, bnd = 1, 2
    pat = orc.pattern_ex(N, n, m, scheme, bnd)
    got = ocp.pattern(N, n, m, scheme=scheme, boundary=bnd)
    _same(got, pat, ("jrow", "jcol", "hrow", "hcol"))
    del got, pat
    gc.collect()
    want = orc.kkt_ex(N, n, m, scheme, bnd)
    gc.collect()
    got = ocp.kkt_pattern(N, n, m, scheme=scheme, boundary=bnd)
    _same(got, want, ("rowptr", "colind", "perm_j", "perm_h"))


def test_full_size_quadrotor_structure(orc):
    N, bnd = 1_000_000, 1
    pat = orc.quad_pattern(N, bnd)
    got = ocp.quad_pattern(N, bnd)
    _same(got, pat, ("jrow", "jcol", "hrow", "hcol"))
    del got, pat
    gc.collect()
    want = orc.quad_kkt(N, bnd)
    gc.collect()
    got = ocp.quad_kkt_pattern(N, bnd)
    _same(got, want, ("rowptr", "colind", "perm_j", "perm_h"))
