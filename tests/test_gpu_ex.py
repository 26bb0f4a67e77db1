"""GPU parity of the forward-Euler scheme and the boundary rows (through the
C ABI's *_ex entry points) against the CPU oracle's _ex family: values within
1e-12 * mu, assembly bit-exact, paired and single Jacobian stores bitwise
equal."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import check_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [(s, b) for s in (0, 1) for b in (0, 1, 2)]
SHAPES = [(1000, 4, 2), (777, 5, 3), (1, 1, 0), (2, 2, 1), (3, 3, 0), (257, 16, 8), (513, 32, 32),
          (4096, 8, 4), (60, 2, 9)]


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


@pytest.mark.parametrize("scheme,bnd", CASES)
@pytest.mark.parametrize("N,n,m", SHAPES)
def test_values_and_assembly(ocp, N, n, m, scheme, bnd):
    _say(f"[ex] N={N} n={n} m={m} scheme={scheme} bnd={bnd}")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=11, scheme=scheme, bnd=bnd)
    prob = ocp.Problem.from_instance(inst, dev)
    s = prob.sizes
    assert s["nvar"] == len(inst.z) and s["ncon"] == len(inst.y)
    z = torch.from_numpy(inst.z).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    got = dict(obj=prob.obj(z), grad=prob.grad(z), cons=prob.cons(z), jac=prob.jac(z),
               hess=prob.hess(z, y, 1.1))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    f, fm = oracle.obj_ex(inst, scheme, bnd)
    check_close(got["obj"], np.array([f]), np.array([fm]), what="obj")
    for name, (want, mu) in (("grad", oracle.grad_ex(inst, scheme, bnd)),
                             ("cons", oracle.cons_ex(inst, scheme, bnd)),
                             ("jac", oracle.jac_ex(inst, scheme, bnd)),
                             ("hess", oracle.hess_ex(inst, scheme, bnd, sigma=1.1))):
        check_close(got[name], want, mu, what=name)
    rowptr, _, perm_j, perm_h = ocp.kkt_pattern(N, n, m, colind=False, scheme=scheme, boundary=bnd)
    reg = np.random.default_rng(3).normal(size=s["dim"])
    kkt = prob.assemble_kkt(*(torch.from_numpy(a).to(dev) for a in (perm_j, perm_h, rowptr)),
                            torch.from_numpy(got["jac"]).to(dev), torch.from_numpy(got["hess"]).to(dev),
                            torch.from_numpy(reg).to(dev))
    want = oracle.assemble(rowptr, perm_j, got["jac"], perm_h, got["hess"], reg)
    assert np.array_equal(kkt.cpu().numpy().view(np.uint64), want.view(np.uint64))
    prob.close()


@pytest.mark.parametrize("bnd", [0, 2])
def test_euler_paired_and_single_stores_agree(ocp, bnd):
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(2000, 6, 3, seed=12, scheme=1, bnd=bnd)
    prob = ocp.Problem.from_instance(inst, dev)
    z = torch.from_numpy(inst.z).to(dev)
    a = prob.jac(z)
    buf = torch.empty(a.numel() + 1, dtype=torch.float64, device=dev)
    b = prob.jac(z, out=buf[1:])
    assert b.data_ptr() % 16 == 8
    assert torch.equal(a.view(torch.int64), b.view(torch.int64))
    c = prob.jac(z)
    assert torch.equal(a.view(torch.int64), c.view(torch.int64))
    prob.close()


def test_euler_large_full_arrays(ocp):
    """A 2e5-interval, n = 16, m = 8 instance under forward Euler with both
    boundary groups: defects, Jacobian and Hessian values as full arrays."""
    N, n, m = 200_000, 16, 8
    _say("[ex] large Euler")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=0, scheme=1, bnd=2)
    prob = ocp.Problem.from_instance(inst, dev)
    z = torch.from_numpy(inst.z).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    for name, fn, want in (("cons", lambda: prob.cons(z), oracle.cons_ex(inst, 1, 2)),
                           ("hess", lambda: prob.hess(z, y, 1.0), oracle.hess_ex(inst, 1, 2))):
        check_close(fn().cpu().numpy(), want[0], want[1], what=name)
    got = prob.jac(z).cpu().numpy()
    want, mu = oracle.jac_ex(inst, 1, 2)
    check_close(got, want, mu, what="jac")
    del got, want, mu
    prob.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("scheme,bnd", [(0, 0), (1, 2), (0, 1)])
def test_problem_pattern_methods(ocp, scheme, bnd):
    """Problem.pattern() and Problem.kkt_pattern() give the handle's own
    structure: bit-exact against the oracle's pattern and KKT build for the
    problem's sizes, scheme and boundary option; the same for the quadrotor."""
    N, n, m = 37, 5, 2
    inst = synth.make_instance(N, n, m, seed=3, scheme=scheme, bnd=bnd)
    prob = ocp.Problem.from_instance(inst, torch.device("cuda", 0))
    got = prob.pattern()
    want = oracle.pattern_ex(N, n, m, scheme, bnd)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    got = prob.kkt_pattern()
    rowptr, colind, perm_j, perm_h = oracle.kkt_ex(N, n, m, scheme, bnd)[:4]
    for g, w in zip(got, (rowptr, colind, perm_j, perm_h)):
        assert np.array_equal(g, w)
    prob.close()
    q = synth.make_quadrotor(21, seed=0, bnd=bnd)
    qp = ocp.QuadrotorProblem.from_instance(q, torch.device("cuda", 0))
    for g, w in zip(qp.pattern(), oracle.quad_pattern(21, bnd)):
        assert np.array_equal(g, w)
    for g, w in zip(qp.kkt_pattern(), oracle.quad_kkt(21, bnd)[:4]):
        assert np.array_equal(g, w)
    qp.close()
