"""Pins of the oracle's symmetric KKT reordering (paper Sec. 6: a one-time
host reordering precedes the LDL^T factorization) and of the assembly through
slot maps alone:
- the permuted structure equals scipy's tril(K[order][:, order]).tocsr();
- every carried-over slot sits at the permuted (row, col) of its entry;
- assembled values equal the dense P K P^T of the naturally assembled K;
- the identity ordering reproduces the original structure;
- orderings that are not permutations are rejected."""
from __future__ import annotations

import numpy as np
import pytest


def _structure(orc, N, n, m, scheme, bnd):
    s = orc.sizes_ex(N, n, m, scheme, bnd)
    jr, jc, hr, hc = orc.pattern_ex(N, n, m, scheme, bnd)
    rp, ci, pj, ph = orc.kkt_ex(N, n, m, scheme, bnd)
    return s, (jr, jc, hr, hc), (rp, ci, pj, ph)


def _orders(dim, seed):
    rng = np.random.default_rng(seed)
    return {"random": rng.permutation(dim), "reversed": np.arange(dim)[::-1].copy()}


@pytest.mark.parametrize("scheme,bnd", [(0, 0), (1, 2), (0, 1)])
@pytest.mark.parametrize("N,n,m", [(5, 3, 2), (8, 1, 1), (4, 4, 0)])
def test_permuted_structure_matches_scipy(orc, N, n, m, scheme, bnd):
    import scipy.sparse as sp
    s, (jr, jc, hr, hc), (rp, ci, pj, ph) = _structure(orc, N, n, m, scheme, bnd)
    nv, dim = s["nvar"], s["dim"]
    rows = np.concatenate([hr, nv + jr, np.arange(dim)])
    cols = np.concatenate([hc, jc, np.arange(dim)])
    K = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(dim, dim)).tocsr()
    K = K + K.T
    for name, order in _orders(dim, 100 + N).items():
        rp2, ci2, pj2, ph2, dg2 = orc.kkt_permute(rp, ci, pj, ph, order)
        M = sp.tril(K[order][:, order]).tocsr()
        M.sort_indices()
        assert np.array_equal(M.indptr, rp2), name
        assert np.array_equal(M.indices, ci2), name
        pos = np.empty(dim, np.int64)
        pos[order] = np.arange(dim)
        slot_row = np.repeat(np.arange(dim), np.diff(rp2))
        a, b = pos[nv + jr], pos[jc]
        assert np.array_equal(slot_row[pj2], np.maximum(a, b)) and np.array_equal(ci2[pj2], np.minimum(a, b))
        a, b = pos[hr], pos[hc]
        assert np.array_equal(slot_row[ph2], np.maximum(a, b)) and np.array_equal(ci2[ph2], np.minimum(a, b))
        assert np.array_equal(slot_row[dg2], pos) and np.array_equal(ci2[dg2], pos)
        assert len(set(pj2.tolist()) | set(ph2.tolist()) | set(dg2.tolist())) == len(ci2)


@pytest.mark.parametrize("N,n,m,scheme,bnd", [(6, 3, 2, 0, 0), (5, 2, 1, 1, 2)])
def test_mapped_assembly_equals_dense_reordering(orc, N, n, m, scheme, bnd):
    s, _, (rp, ci, pj, ph) = _structure(orc, N, n, m, scheme, bnd)
    dim = s["dim"]
    rng = np.random.default_rng(7)
    jv, hv, reg = rng.normal(size=s["nnzj"]), rng.normal(size=s["nnzh"]), rng.normal(size=dim)
    kkt = orc.assemble(rp, pj, jv, ph, hv, reg)
    K = np.zeros((dim, dim))
    rows = np.repeat(np.arange(dim), np.diff(rp))
    K[rows, ci] = kkt
    K[ci, rows] = kkt
    order = rng.permutation(dim)
    rp2, ci2, pj2, ph2, dg2 = orc.kkt_permute(rp, ci, pj, ph, order)
    kkt2 = orc.assemble_mapped(rp2[-1], dg2, pj2, jv, ph2, hv, reg)
    K2 = np.zeros((dim, dim))
    rows2 = np.repeat(np.arange(dim), np.diff(rp2))
    K2[rows2, ci2] = kkt2
    K2[ci2, rows2] = kkt2
    assert np.array_equal(K2, K[np.ix_(order, order)])


def test_identity_ordering_reproduces_structure(orc):
    s, _, (rp, ci, pj, ph) = _structure(orc, 9, 4, 2, 0, 1)
    rp2, ci2, pj2, ph2, dg2 = orc.kkt_permute(rp, ci, pj, ph, np.arange(s["dim"]))
    for a, b in ((rp, rp2), (ci, ci2), (pj, pj2), (ph, ph2), (rp[1:] - 1, dg2)):
        assert np.array_equal(a, b)
    # and the mapped assembly then equals the rowptr-based one
    rng = np.random.default_rng(8)
    jv, hv, reg = rng.normal(size=s["nnzj"]), rng.normal(size=s["nnzh"]), rng.normal(size=s["dim"])
    a = orc.assemble(rp, pj, jv, ph, hv, reg)
    b = orc.assemble_mapped(rp[-1], dg2, pj, jv, ph, hv, reg)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_rejects_non_permutations(orc):
    s, _, (rp, ci, pj, ph) = _structure(orc, 4, 2, 1, 0, 0)
    dim = s["dim"]
    bad = np.arange(dim)
    bad[3] = bad[5]
    for order in (bad, np.arange(1, dim + 1), np.arange(-1, dim - 1)):
        with pytest.raises(ValueError):
            orc.kkt_permute(rp, ci, pj, ph, order)


def test_quadrotor_permutation(orc):
    """The same build serves any model's KKT: the quadrotor's, reversed."""
    import scipy.sparse as sp
    N = 6
    s = orc.quad_sizes(N, 1)
    jr, jc, hr, hc = orc.quad_pattern(N, 1)
    rp, ci, pj, ph = orc.quad_kkt(N, 1)
    nv, dim = s["nvar"], s["dim"]
    order = np.random.default_rng(9).permutation(dim)
    rp2, ci2, pj2, ph2, dg2 = orc.kkt_permute(rp, ci, pj, ph, order)
    rows = np.concatenate([hr, nv + jr, np.arange(dim)])
    cols = np.concatenate([hc, jc, np.arange(dim)])
    K = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(dim, dim)).tocsr()
    M = sp.tril((K + K.T)[order][:, order]).tocsr()
    M.sort_indices()
    assert np.array_equal(M.indptr, rp2) and np.array_equal(M.indices, ci2)
