"""GPU parity of the fused evaluation into the KKT matrix (ocp_eval_kkt), under
both schemes and every boundary option:
against the oracle's Jacobian and Hessian assembled by the oracle (values
within 1e-12 * mu, the magnitudes assembled the same way), and against the
separate path eval_jac + eval_hess + assemble_kkt (same expressions; the
compiler may contract them into FMAs differently, so within rounding); at the
N = 1e6, n = 16, m = 8 benchmark size on the device."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import check_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(1000, 4, 2, 0), (777, 5, 3, 1), (1, 1, 0, 0), (1, 1, 1, 2), (2, 2, 1, 0), (3, 3, 0, 1),
          (255, 2, 0, 0), (256, 3, 1, 2), (257, 16, 8, 0), (63, 6, 3, 1), (65, 7, 2, 0),
          (513, 32, 32, 2), (300, 9, 4, 0), (4097, 8, 4, 1)]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ocp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_03932_amd as ocp
    ocp.lib()
    return ocp


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


EULER_SHAPES = [(1000, 4, 2, 0), (777, 5, 3, 2), (1, 1, 0, 0), (1, 1, 1, 1), (2, 2, 1, 2), (3, 3, 0, 1),
                (257, 16, 8, 0), (65, 7, 2, 1), (513, 32, 32, 2), (4097, 8, 4, 0)]


@pytest.mark.parametrize("N,n,m,bnd,scheme", [s + (0,) for s in SHAPES] + [s + (1,) for s in EULER_SHAPES])
def test_fused_matches_oracle_and_separate_path(ocp, N, n, m, bnd, scheme):
    _say(f"[fused] N={N} n={n} m={m} bnd={bnd} scheme={scheme}")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=41, bnd=bnd, scheme=scheme)
    prob = ocp.Problem.from_instance(inst, dev)
    s = prob.sizes
    z, y = _t(inst.z), _t(inst.y)
    rp, ci, pj, ph = ocp.kkt_pattern(N, n, m, scheme=scheme, boundary=bnd)
    reg = np.random.default_rng(5).normal(size=s["dim"])
    for r in (None, reg):
        rt = None if r is None else _t(r)
        out = torch.full((s["nnzk"],), float("nan"), dtype=torch.float64, device=dev)
        fused = prob.eval_kkt(z, y, 0.7, rt, out=out).cpu().numpy()
        jv, hv = prob.jac(z), prob.hess(z, y, 0.7)
        sep = prob.assemble_kkt(_t(pj), _t(ph), _t(rp), jv, hv, rt).cpu().numpy()
        oj, mj = oracle.jac_ex(inst, scheme, bnd)
        oh, mh = oracle.hess_ex(inst, scheme, bnd, sigma=0.7)
        want = oracle.assemble(rp, pj, oj, ph, oh, r)
        mu = oracle.assemble(rp, pj, mj, ph, mh, None if r is None else np.abs(r))
        differ = np.flatnonzero(fused.view(np.uint64) != sep.view(np.uint64))
        if len(differ):
            rows = np.searchsorted(rp, differ, side="right") - 1
            _say(f"  bits differ from the separate path at {len(differ)} slots; rows "
                 f"{np.unique(np.minimum(rows // (N + 1), 99))[:8]} (row // (N+1)); "
                 f"max |diff|/mu {np.max(np.abs(fused[differ] - sep[differ]) / mu[differ]):.2e}")
        check_close(fused, want, mu, what=f"kkt reg={r is not None}")
        check_close(fused, sep, mu, what=f"fused vs separate reg={r is not None}")
    prob.close()


def test_fused_large_equals_separate_path(ocp):
    """N = 1e6, n = 16, m = 8 with a regularization diagonal: the fused KKT
    agrees with the separate path (itself checked against the oracle) to
    1e-12 relative, plus an absolute 1e-18 for the O(h) Hessian entries that
    can cancel, compared on the device."""
    _say("[fused] large")
    N, n, m = synth.LARGE
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=0)
    prob = ocp.Problem.from_instance(inst, dev)
    s = prob.sizes
    z, y = _t(inst.z), _t(inst.y)
    reg = torch.full((s["dim"],), 1e-8, dtype=torch.float64, device=dev)
    fused = prob.eval_kkt(z, y, 1.0, reg)
    rp, _, pj, ph = ocp.kkt_pattern(N, n, m, colind=False)
    tpj = _t(pj)
    del pj
    jv = prob.jac(z)
    hv = prob.hess(z, y, 1.0)
    sep = prob.assemble_kkt(tpj, _t(ph), _t(rp), jv, hv, reg)
    del jv, hv, tpj
    diff = (fused - sep).abs()
    bound = 1e-12 * (fused.abs() + sep.abs()) + 1e-18
    assert bool((diff <= bound).all())
    prob.close()
    del fused, sep
    torch.cuda.empty_cache()


QUAD_SHAPES = [(1, 0), (1, 2), (2, 1), (255, 1), (256, 0), (257, 2), (1000, 1), (4097, 1)]


@pytest.mark.parametrize("N,bnd", QUAD_SHAPES)
def test_fused_quadrotor_matches_oracle_and_separate_path(ocp, N, bnd):
    """The quadrotor model's fused KKT against the oracle's Jacobian and
    Hessian assembled by the oracle, and against the separate path."""
    _say(f"[fused quad] N={N} bnd={bnd}")
    dev = torch.device("cuda", 0)
    q = synth.make_quadrotor(N, seed=44, bnd=bnd)
    prob = ocp.QuadrotorProblem.from_instance(q, dev)
    s = prob.sizes
    z, y = _t(q.z), _t(q.y)
    rp, ci, pj, ph = ocp.quad_kkt_pattern(N, bnd)
    reg = np.random.default_rng(6).normal(size=s["dim"])
    for r in (None, reg):
        rt = None if r is None else _t(r)
        out = torch.full((s["nnzk"],), float("nan"), dtype=torch.float64, device=dev)
        fused = prob.eval_kkt(z, y, 0.7, rt, out=out).cpu().numpy()
        sep = prob.assemble_kkt(_t(pj), _t(ph), _t(rp), prob.jac(z), prob.hess(z, y, 0.7), rt).cpu().numpy()
        oj, mj = oracle.quad_jac(q)
        oh, mh = oracle.quad_hess(q, sigma=0.7)
        want = oracle.assemble(rp, pj, oj, ph, oh, r)
        mu = oracle.assemble(rp, pj, mj, ph, mh, None if r is None else np.abs(r))
        check_close(fused, want, mu, what=f"quad kkt reg={r is not None}")
        check_close(fused, sep, mu, what=f"quad fused vs separate reg={r is not None}")
    prob.close()


def test_fused_quadrotor_large_equals_separate_path(ocp):
    """The quadrotor at N = 1e6 with reg: the fused KKT against the separate
    path on the device (1e-12 relative plus 1e-18 absolute)."""
    _say("[fused quad] large")
    N = synth.QUAD_LARGE
    dev = torch.device("cuda", 0)
    q = synth.make_quadrotor(N, seed=0, bnd=1)
    prob = ocp.QuadrotorProblem.from_instance(q, dev)
    s = prob.sizes
    z, y = _t(q.z), _t(q.y)
    reg = torch.full((s["dim"],), 1e-8, dtype=torch.float64, device=dev)
    fused = prob.eval_kkt(z, y, 1.0, reg)
    rp, _, pj, ph = ocp.quad_kkt_pattern(N, 1, colind=False)
    sep = prob.assemble_kkt(_t(pj), _t(ph), _t(rp), prob.jac(z), prob.hess(z, y, 1.0), reg)
    diff = (fused - sep).abs()
    assert bool((diff <= 1e-12 * (fused.abs() + sep.abs()) + 1e-18).all())
    prob.close()
    del fused, sep
    torch.cuda.empty_cache()
