"""GPU parity of the quadrotor model (paper Appendix A) against the CPU
oracle, through the C ABI: objective, gradient, defects, Jacobian and
Hessian values within 1e-12 * mu; the KKT assembly bit-exact (closed-form
slot maps, with and without reg, and shuffled maps that force the direct-store
path); paired and single Jacobian stores bitwise equal; full arrays at the
paper's largest grid (N = 2e5) and at N = 1e6, the benchmark's launch
configuration."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import check_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# ragged N around the 256-lane workgroup and the assembly tiles; N = 1, 2
# (both end nodes in one interval); every boundary option
CASES = [(1, 0), (1, 1), (2, 2), (3, 1), (255, 1), (256, 0), (257, 2), (511, 1), (1000, 1),
         (1023, 2), (4097, 1)]


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


def _evaluate(ocp, q, sigma=1.0):
    dev = torch.device("cuda", 0)
    prob = ocp.QuadrotorProblem.from_instance(q, dev)
    s = prob.sizes
    assert s["nvar"] == len(q.z) and s["ncon"] == len(q.y)
    z = torch.from_numpy(q.z).to(dev)
    y = torch.from_numpy(q.y).to(dev)
    got = dict(obj=prob.obj(z), grad=prob.grad(z), cons=prob.cons(z), jac=prob.jac(z),
               hess=prob.hess(z, y, sigma))
    torch.cuda.synchronize()
    return prob, {k: v.cpu().numpy() for k, v in got.items()}


def _check_values(q, got, sigma=1.0):
    f, fm = oracle.quad_obj(q)
    check_close(got["obj"], np.array([f]), np.array([fm]), what="obj")
    for name, (want, mu) in (("grad", oracle.quad_grad(q)), ("cons", oracle.quad_cons(q)),
                             ("jac", oracle.quad_jac(q)), ("hess", oracle.quad_hess(q, sigma=sigma))):
        check_close(got[name], want, mu, what=name)


@pytest.mark.parametrize("N,bnd", CASES)
def test_values_and_assembly(ocp, N, bnd):
    _say(f"[quad] N={N} bnd={bnd}")
    dev = torch.device("cuda", 0)
    q = synth.make_quadrotor(N, seed=21, bnd=bnd)
    prob, got = _evaluate(ocp, q, sigma=0.8)
    _check_values(q, got, sigma=0.8)
    rowptr, _, perm_j, perm_h = ocp.quad_kkt_pattern(N, bnd, colind=False)
    args = [torch.from_numpy(a).to(dev) for a in (perm_j, perm_h, rowptr, got["jac"], got["hess"])]
    reg = np.random.default_rng(3).normal(size=prob.sizes["dim"])
    for r in (None, reg):
        out = torch.full((prob.sizes["nnzk"],), float("nan"), dtype=torch.float64, device=dev)
        kkt = prob.assemble_kkt(*args, None if r is None else torch.from_numpy(r).to(dev), out=out)
        want = oracle.assemble(rowptr, perm_j, got["jac"], perm_h, got["hess"], r)
        assert np.array_equal(kkt.cpu().numpy().view(np.uint64), want.view(np.uint64))
    prob.close()


@pytest.mark.parametrize("scope", ["within_rows", "global"])
def test_assemble_generic_slot_map(ocp, scope):
    """Shuffled slot maps (constraint diagonals fixed): within CSR rows every
    tile still covers its range exactly; over the whole matrix the tiles fall
    back to direct stores.  Without reg the result equals the plain scatter."""
    _say(f"[quad assemble-generic] {scope}")
    dev = torch.device("cuda", 0)
    N, bnd = 3001, 2
    q = synth.make_quadrotor(N, seed=22, bnd=bnd)
    prob, got = _evaluate(ocp, q)
    rowptr, _, perm_j, perm_h = ocp.quad_kkt_pattern(N, bnd, colind=False)
    s = prob.sizes
    rng = np.random.default_rng(12)
    movable = np.concatenate([perm_h, perm_j])
    pi = np.arange(s["nnzk"], dtype=np.int64)
    if scope == "global":
        pi[movable] = movable[rng.permutation(len(movable))]
    else:
        rows = np.repeat(np.arange(s["dim"]), np.diff(rowptr))
        for d in rng.choice(s["dim"], size=3000, replace=False):
            slots = np.arange(rowptr[d], rowptr[d + 1])
            slots = slots[np.isin(slots, movable)]
            pi[slots] = rng.permutation(slots)
        assert np.all(rows[pi] == rows)
    pj2 = pi[perm_j].astype(np.int32)
    ph2 = pi[perm_h].astype(np.int32)
    kkt = prob.assemble_kkt(torch.from_numpy(pj2).to(dev), torch.from_numpy(ph2).to(dev),
                            torch.from_numpy(rowptr).to(dev), torch.from_numpy(got["jac"]).to(dev),
                            torch.from_numpy(got["hess"]).to(dev))
    want = oracle.assemble(rowptr, pj2, got["jac"], ph2, got["hess"], None)
    assert np.array_equal(kkt.cpu().numpy().view(np.uint64), want.view(np.uint64))
    prob.close()


def test_paired_and_single_stores_agree_and_deterministic(ocp):
    dev = torch.device("cuda", 0)
    q = synth.make_quadrotor(2000, seed=23, bnd=1)
    prob = ocp.QuadrotorProblem.from_instance(q, dev)
    z = torch.from_numpy(q.z).to(dev)
    y = torch.from_numpy(q.y).to(dev)
    a = prob.jac(z)
    buf = torch.empty(a.numel() + 1, dtype=torch.float64, device=dev)
    b = prob.jac(z, out=buf[1:])
    assert b.data_ptr() % 16 == 8
    assert torch.equal(a.view(torch.int64), b.view(torch.int64))
    for fn in (lambda: prob.jac(z), lambda: prob.hess(z, y, 1.0), lambda: prob.cons(z),
               lambda: prob.obj(z), lambda: prob.grad(z)):
        u, v = fn(), fn()
        assert torch.equal(u.view(torch.int64), v.view(torch.int64))
    prob.close()


def test_hover_defects_are_zero(ocp):
    """Level attitude, thrust g, no rates or velocities: every defect is 0."""
    dev = torch.device("cuda", 0)
    N = 777
    q = synth.make_quadrotor(N, seed=24, bnd=1)
    X = np.zeros((9, N + 1))
    X[0], X[2], X[4] = 1.5, -0.25, 3.0
    U = np.zeros((4, N + 1))
    U[0] = synth.QUAD_G
    q.z = np.concatenate([X.ravel(), U.ravel()])
    prob = ocp.QuadrotorProblem.from_instance(q, dev)
    c = prob.cons(torch.from_numpy(q.z).to(dev)).cpu().numpy()
    assert np.all(c[: 9 * N] == 0.0)
    assert np.array_equal(c[9 * N:], X[:, 0])
    prob.close()


@pytest.mark.parametrize("N", [synth.QUAD_PAPER, synth.QUAD_LARGE])
def test_large_full_arrays(ocp, N):
    """Every array in full at the paper's largest grid and at the benchmark's
    size, with the initial-state rows, in the launch configuration the
    benchmark times (paired Jacobian stores, N even); the assembly bit-exact."""
    _say(f"[quad] large N={N}")
    dev = torch.device("cuda", 0)
    q = synth.make_quadrotor(N, seed=0, bnd=1)
    prob, got = _evaluate(ocp, q)
    _check_values(q, got)
    rowptr, _, perm_j, perm_h = ocp.quad_kkt_pattern(N, 1, colind=False)
    kkt = prob.assemble_kkt(*(torch.from_numpy(a).to(dev)
                              for a in (perm_j, perm_h, rowptr, got["jac"], got["hess"])))
    want = oracle.assemble(rowptr, perm_j, got["jac"], perm_h, got["hess"], None)
    assert np.array_equal(kkt.cpu().numpy().view(np.uint64), want.view(np.uint64))
    prob.close()
    del kkt, got
    torch.cuda.empty_cache()


def test_coefficient_entry_points_reject_quadrotor(ocp):
    """The model has no coefficient arrays: the coefficient gradient and the
    coefficient update reject its handle."""
    dev = torch.device("cuda", 0)
    q = synth.make_quadrotor(10, seed=25, bnd=0)
    prob = ocp.QuadrotorProblem.from_instance(q, dev)
    z = torch.from_numpy(q.z).to(dev)
    y = torch.from_numpy(q.y).to(dev)
    with pytest.raises(ocp.OcpError) as e:
        prob.coef_grad(z, y)
    assert e.value.code == ocp.OCP_ERR_ARG
    A = torch.zeros((9, 9), dtype=torch.float64, device=dev)
    B = torch.zeros((9, 4), dtype=torch.float64, device=dev)
    g = torch.zeros(9, dtype=torch.float64, device=dev)
    with pytest.raises(ocp.OcpError) as e:
        prob.set_coefficients(A, B, g)
    assert e.value.code == ocp.OCP_ERR_ARG
    prob.close()


def _check_quad_derivatives(ocp, q, sigma, tag):
    dev = torch.device("cuda", 0)
    prob = ocp.QuadrotorProblem.from_instance(q, dev)
    z, y = torch.from_numpy(q.z).to(dev), torch.from_numpy(q.y).to(dev)
    v = np.random.default_rng(11).normal(size=len(q.z))
    vt = torch.from_numpy(v).to(dev)
    L = prob.lagrangian(z, y, sigma).cpu().numpy()
    Lo, Lm = oracle.quad_lagrangian(q, sigma=sigma)
    check_close(L, np.array([Lo]), np.array([Lm]), what=f"L {tag}")
    want, mu = oracle.quad_lag_grad(q, sigma=sigma)
    check_close(prob.lag_grad(z, y, sigma).cpu().numpy(), want, mu, what=f"grad_z L {tag}")
    want, mu = oracle.quad_hvp(q, v, sigma=sigma)
    check_close(prob.hvp(z, y, vt, sigma).cpu().numpy(), want, mu, what=f"H v {tag}")
    want, mu = oracle.quad_jvp(q, v)
    check_close(prob.jvp(z, vt).cpu().numpy(), want, mu, what=f"J v {tag}")
    prob.close()


@pytest.mark.parametrize("N,bnd", [(1, 0), (1, 2), (2, 1), (3, 0), (255, 1), (256, 2), (1000, 1), (4097, 0)])
def test_quadrotor_derivatives_match_oracle(ocp, N, bnd):
    """L, grad_z L, H v and J v of the quadrotor model against the oracle
    (values within 1e-12 mu)."""
    _say(f"[quad diff] N={N} bnd={bnd}")
    _check_quad_derivatives(ocp, synth.make_quadrotor(N, seed=26, bnd=bnd), 0.9, f"N={N} bnd={bnd}")


def test_quadrotor_derivatives_paper_grid(ocp):
    """The same at the paper's largest grid, N = 2e5, full arrays."""
    N = synth.QUAD_PAPER
    _say(f"[quad diff] N={N}")
    _check_quad_derivatives(ocp, synth.make_quadrotor(N, seed=0, bnd=1), 1.0, "N=2e5")

@pytest.mark.parametrize("N,bnd", [(3, 1), (2, 2)])
def test_quadrotor_autograd(ocp, N, bnd):
    """The autograd wrapper over the quadrotor model (no coefficient
    tensors): L.backward() against the oracle, and torch's gradcheck and
    gradgradcheck (which exercise grad_z L, H v and J v)."""
    from paper_2510_03932_amd.autograd import constraints, lagrangian, lagrangian_grad
    dev = torch.device("cuda", 0)
    q = synth.make_quadrotor(N, seed=27, bnd=bnd)
    prob = ocp.QuadrotorProblem.from_instance(q, dev)
    z = torch.from_numpy(q.z.copy()).to(dev).requires_grad_(True)
    y = torch.from_numpy(q.y.copy()).to(dev).requires_grad_(True)
    L = lagrangian(prob, z, y, sigma=0.9)
    L.backward()
    want, mu = oracle.quad_lag_grad(q, sigma=0.9)
    check_close(z.grad.cpu().numpy(), want, mu, what="z.grad")
    want, mu = oracle.quad_cons(q)
    check_close(y.grad.cpu().numpy(), want, mu, what="y.grad")
    z, y = z.detach().requires_grad_(True), y.detach().requires_grad_(True)
    f = lambda z, y: lagrangian(prob, z, y, sigma=1.2)
    assert torch.autograd.gradcheck(f, (z, y), eps=1e-6, atol=1e-6, rtol=1e-5)
    assert torch.autograd.gradgradcheck(f, (z, y), eps=1e-6, atol=1e-6, rtol=1e-5)
    fg = lambda z, y: lagrangian_grad(prob, z, y, sigma=1.2)
    assert torch.autograd.gradcheck(fg, (z, y), eps=1e-6, atol=1e-6, rtol=1e-5)
    fc = lambda z: constraints(prob, z)
    assert torch.autograd.gradcheck(fc, (z,), eps=1e-6, atol=1e-6, rtol=1e-5)
    prob.close()
