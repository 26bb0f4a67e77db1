"""GPU parity of the Lagrangian derivatives (L, grad_z L, H v, J v, dL/dtheta,
its mixed derivative along v and its adjoint) against the CPU oracle, and of the autograd wrapper against finite differences
(torch.autograd.gradcheck / gradgradcheck, and central differences at step
1e-6 on the 2e5-interval differentiation workload)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import check_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(1000, 4, 2), (777, 5, 3), (1, 1, 0), (1, 1, 1), (2, 2, 1), (3, 3, 0), (255, 2, 0),
          (257, 16, 8), (513, 32, 32), (300, 9, 4)]


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


def _dev_inputs(inst, seed=0):
    dev = torch.device("cuda", 0)
    v = np.random.default_rng(seed).normal(size=len(inst.z))
    return (dev, torch.from_numpy(inst.z).to(dev), torch.from_numpy(inst.y).to(dev),
            v, torch.from_numpy(v).to(dev))


def _check_all(ocp, inst, sigma, tag):
    dev, z, y, v, vt = _dev_inputs(inst)
    prob = ocp.Problem.from_instance(inst, dev)
    L = prob.lagrangian(z, y, sigma).cpu().numpy()
    g = prob.lag_grad(z, y, sigma).cpu().numpy()
    hv = prob.hvp(z, y, vt, sigma).cpu().numpy()
    jv = prob.jvp(z, vt).cpu().numpy()
    gA, gB, gg = (t.cpu().numpy() for t in prob.coef_grad(z, y))
    Lo, Lm = oracle.lagrangian(inst, sigma=sigma)
    check_close(L, np.array([Lo]), np.array([Lm]), what=f"L {tag}")
    want, mu = oracle.lag_grad(inst, sigma=sigma)
    check_close(g, want, mu, what=f"grad_z L {tag}")
    want, mu = oracle.hvp(inst, v, sigma=sigma)
    check_close(hv, want, mu, what=f"H v {tag}")
    want, mu = oracle.jvp(inst, v)
    check_close(jv, want, mu, what=f"J v {tag}")
    (oA, oB, og), (mA, mB, mg) = oracle.coef_grad(inst)
    check_close(gA, oA, mA, what=f"dL/dA {tag}")
    check_close(gB, oB, mB, what=f"dL/dB {tag}")
    check_close(gg, og, mg, what=f"dL/dgamma {tag}")
    prob.close()


@pytest.mark.parametrize("N,n,m", SHAPES)
def test_derivatives_match_oracle(ocp, N, n, m):
    _say(f"[diff] N={N} n={n} m={m}")
    _check_all(ocp, synth.make_instance(N, n, m, seed=2), 1.3, f"{N},{n},{m}")


def _check_all_ex(ocp, inst, sigma, tag):
    """Every derivative under the instance's scheme and boundary option,
    against the oracle's definitions over its _ex arrays."""
    scheme, bnd = inst.scheme, inst.bnd
    dev, z, y, v, vt = _dev_inputs(inst)
    prob = ocp.Problem.from_instance(inst, dev)
    L = prob.lagrangian(z, y, sigma).cpu().numpy()
    g = prob.lag_grad(z, y, sigma).cpu().numpy()
    hv = prob.hvp(z, y, vt, sigma).cpu().numpy()
    jv = prob.jvp(z, vt).cpu().numpy()
    gA, gB, gg = (t.cpu().numpy() for t in prob.coef_grad(z, y))
    Lo, Lm = oracle.lagrangian_ex(inst, scheme, bnd, sigma=sigma)
    check_close(L, np.array([Lo]), np.array([Lm]), what=f"L {tag}")
    want, mu = oracle.lag_grad_ex(inst, scheme, bnd, sigma=sigma)
    check_close(g, want, mu, what=f"grad_z L {tag}")
    want, mu = oracle.hvp_ex(inst, v, scheme, bnd, sigma=sigma)
    check_close(hv, want, mu, what=f"H v {tag}")
    want, mu = oracle.jvp_ex(inst, v, scheme, bnd)
    check_close(jv, want, mu, what=f"J v {tag}")
    (oA, oB, og), (mA, mB, mg) = oracle.coef_grad_ex(inst, scheme, bnd)
    check_close(gA.ravel(), oA.ravel(), mA.ravel(), what=f"dL/dA {tag}")
    check_close(gB.ravel(), oB.ravel(), mB.ravel(), what=f"dL/dB {tag}")
    check_close(gg, og, mg, what=f"dL/dgamma {tag}")
    prob.close()


EX_SHAPES = [(1000, 4, 2), (777, 5, 3), (1, 1, 0), (1, 1, 1), (2, 2, 1), (3, 3, 0), (257, 16, 8),
             (513, 32, 32), (300, 9, 4), (50, 2, 9)]


@pytest.mark.parametrize("scheme,bnd", [(0, 1), (0, 2), (1, 0), (1, 1), (1, 2)])
@pytest.mark.parametrize("N,n,m", EX_SHAPES)
def test_derivatives_other_schemes_match_oracle(ocp, N, n, m, scheme, bnd):
    """Forward Euler and boundary rows: every derivative entry point against
    the oracle (values within 1e-12 mu)."""
    _say(f"[diff ex] N={N} n={n} m={m} scheme={scheme} bnd={bnd}")
    inst = synth.make_instance(N, n, m, seed=7, scheme=scheme, bnd=bnd)
    _check_all_ex(ocp, inst, 1.3, f"{N},{n},{m},{scheme},{bnd}")


def test_derivatives_other_schemes_workload(ocp):
    """The differentiation workload's size (N = 2e5, n = 8, m = 4) under
    forward Euler with initial and final state rows, full arrays."""
    N, n, m = synth.DIFF
    _say(f"[diff ex] workload N={N} n={n} m={m} Euler bnd=2")
    _check_all_ex(ocp, synth.make_instance(N, n, m, seed=0, scheme=1, bnd=2), 1.0, "Euler 2e5")


# (n, m) for each (row blocks, column blocks) tiling of the coefficient
# gradient: ceil(n/16) x ceil((n+m)/16) = 1x1, 1x2, 1x3, 2x2, 2x3, 2x4
COEF_TILINGS = [(7, 5), (16, 1), (12, 30), (17, 15), (24, 16), (32, 31)]


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("n,m", COEF_TILINGS)
def test_coef_grad_every_tiling(ocp, n, m, scheme):
    """Every tiling of the coefficient-gradient kernel, at N = 389 (390
    nodes: several chunks and a ragged last one)."""
    N = 389
    _say(f"[coef grad] N={N} n={n} m={m} scheme={scheme}")
    inst = synth.make_instance(N, n, m, seed=13, scheme=scheme)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y = torch.from_numpy(inst.z).to(dev), torch.from_numpy(inst.y).to(dev)
    gA, gB, gg = (t.cpu().numpy() for t in prob.coef_grad(z, y))
    (oA, oB, og), (mA, mB, mg) = oracle.coef_grad_ex(inst, scheme, 0)
    tag = f"{N},{n},{m},{scheme}"
    check_close(gA.ravel(), oA.ravel(), mA.ravel(), what=f"dL/dA {tag}")
    check_close(gB.ravel(), oB.ravel(), mB.ravel(), what=f"dL/dB {tag}")
    check_close(gg, og, mg, what=f"dL/dgamma {tag}")
    prob.close()


@pytest.mark.parametrize("N,n,m,scheme", [(600_000, 5, 2, 0), (600_001, 3, 0, 1), (270_000, 17, 9, 0)])
def test_coef_grad_many_chunks_per_workgroup(ocp, N, n, m, scheme):
    """Sizes where each workgroup of the coefficient-gradient sum takes more
    than one chunk of nodes (the grid holds at most 1024 of them), with a
    ragged last chunk and, at n = 17, m = 9, two row and two column blocks.
    A second call must give the same bits (fixed summation order)."""
    _say(f"[coef grad] N={N} n={n} m={m} scheme={scheme}")
    inst = synth.make_instance(N, n, m, seed=11, scheme=scheme)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y = torch.from_numpy(inst.z).to(dev), torch.from_numpy(inst.y).to(dev)
    gA, gB, gg = (t.cpu().numpy() for t in prob.coef_grad(z, y))
    again = [t.cpu().numpy() for t in prob.coef_grad(z, y)]
    for first, second in zip((gA, gB, gg), again):
        assert np.array_equal(first.view(np.int64), second.view(np.int64))
    (oA, oB, og), (mA, mB, mg) = oracle.coef_grad_ex(inst, scheme, 0)
    tag = f"{N},{n},{m},{scheme}"
    check_close(gA.ravel(), oA.ravel(), mA.ravel(), what=f"dL/dA {tag}")
    check_close(gB.ravel(), oB.ravel(), mB.ravel(), what=f"dL/dB {tag}")
    check_close(gg, og, mg, what=f"dL/dgamma {tag}")
    prob.close()


def test_differentiation_workload_full_arrays(ocp):
    N, n, m = synth.DIFF
    _say(f"[diff] workload N={N} n={n} m={m}")
    _check_all(ocp, synth.make_instance(N, n, m, seed=0), 1.0, "2e5")


def test_deterministic(ocp):
    inst = synth.make_instance(50_000, 8, 4, seed=3)
    dev, z, y, v, vt = _dev_inputs(inst)
    prob = ocp.Problem.from_instance(inst, dev)
    for fn in (lambda: prob.lagrangian(z, y, 1.0), lambda: prob.lag_grad(z, y, 1.0),
               lambda: prob.hvp(z, y, vt, 1.0), lambda: prob.jvp(z, vt),
               lambda: torch.cat([t.ravel() for t in prob.coef_grad(z, y)])):
        a, b = fn(), fn()
        assert torch.equal(a.view(torch.int64), b.view(torch.int64))
    prob.close()


def _strided(a, dev):
    """The values of a as a non-contiguous device tensor."""
    if a.ndim == 2:
        return torch.from_numpy(np.ascontiguousarray(a.T)).to(dev).t()
    return torch.from_numpy(np.repeat(a, 2)).to(dev)[::2]


@pytest.mark.parametrize("layout", ["contiguous", "strided"])
@pytest.mark.parametrize("N,n,m", [(400, 5, 2), (300, 16, 8), (200, 3, 0), (100, 20, 32)])
def test_set_coefficients(ocp, N, n, m, layout):
    """Coefficients pushed from device tensors (contiguous, or strided views
    that the binding copies first) replace the ones given at creation,
    including the handle's padded column copies: every evaluation afterwards
    is bitwise equal to that of a handle created with the new coefficients,
    and the defects and grad_z L match the oracle."""
    _say(f"[set_coefficients] N={N} n={n} m={m} {layout}")
    inst = synth.make_instance(N, n, m, seed=4)
    other = synth.make_instance(N, n, m, seed=5)
    dev, z, y, v, vt = _dev_inputs(inst)
    prob = ocp.Problem.from_instance(other, dev)
    if layout == "strided":
        coefs = [_strided(a, dev) for a in (inst.A, inst.B, inst.gamma)]
        assert not any(t.is_contiguous() for t in coefs if t.numel() > 1)
    else:
        coefs = [torch.from_numpy(a).to(dev) for a in (inst.A, inst.B, inst.gamma)]
    prob.set_coefficients(*coefs)
    got = prob.lag_grad(z, y, 1.0).cpu().numpy()
    want, mu = oracle.lag_grad(inst)
    check_close(got, want, mu, what="after set_coefficients")
    c = prob.cons(z).cpu().numpy()
    want, mu = oracle.cons(inst)
    check_close(c, want, mu, what="cons after set_coefficients")
    fresh = ocp.Problem.from_instance(inst, dev)
    for name, fn in (("cons", lambda P: P.cons(z)), ("jac", lambda P: P.jac(z)),
                     ("hess", lambda P: P.hess(z, y, 0.9)), ("lag_grad", lambda P: P.lag_grad(z, y, 0.9)),
                     ("hvp", lambda P: P.hvp(z, y, vt, 0.9)), ("jvp", lambda P: P.jvp(z, vt)),
                     ("eval_kkt", lambda P: P.eval_kkt(z, y, 0.9))):
        a, b = fn(prob), fn(fresh)
        assert torch.equal(a.view(torch.int64), b.view(torch.int64)), name
    fresh.close()
    prob.close()


def _leaf_inputs(inst, dev, coef_grad=True):
    t = lambda a, rg=True: torch.from_numpy(np.array(a)).to(dev).requires_grad_(rg)
    return (t(inst.z), t(inst.y), t(inst.A, coef_grad), t(inst.B, coef_grad), t(inst.gamma, coef_grad))


@pytest.mark.parametrize("model,scheme,bnd", [("synthetic", 0, 0), ("synthetic", 1, 2), ("synthetic", 0, 1),
                                              ("quadrotor", 0, 1)])
def test_lagrangian_backward_equals_separate_calls(ocp, model, scheme, bnd):
    """ocp_eval_lagrangian_backward: every output is bit for bit the
    separate call's value times the incoming gradient, for every subset of
    outputs; and the calls it rejects."""
    _say(f"[lagrangian backward] {model} scheme={scheme} bnd={bnd}")
    dev = torch.device("cuda", 0)
    coef = model == "synthetic"
    if coef:
        inst = synth.make_instance(3000, 6, 3, seed=51, scheme=scheme, bnd=bnd)
        prob = ocp.Problem.from_instance(inst, dev)
    else:
        inst = synth.make_quadrotor(2000, seed=51, bnd=bnd)
        prob = ocp.QuadrotorProblem.from_instance(inst, dev)
    z, y = torch.from_numpy(inst.z).to(dev), torch.from_numpy(inst.y).to(dev)
    gL = torch.tensor(0.37, dtype=torch.float64, device=dev)
    parts = {"z": prob.lag_grad(z, y, 0.8) * gL, "y": prob.cons(z) * gL}
    if coef:
        parts["coef"] = tuple(t * gL for t in prob.coef_grad(z, y))
    same = lambda a, b: torch.equal(a.reshape(-1).view(torch.int64), b.reshape(-1).view(torch.int64))
    for want in ((True, True, coef), (True, False, False), (False, True, False), (False, False, coef)):
        if not any(want):
            continue
        gz, gy, gc = prob.lagrangian_backward(z, y, 0.8, gL, *want)
        assert (gz is not None, gy is not None, gc is not None) == want
        if want[0]:
            assert same(gz, parts["z"])
        if want[1]:
            assert same(gy, parts["y"])
        if want[2]:
            assert all(same(a, b) for a, b in zip(gc, parts["coef"]))
    L = ocp.lib()
    p = lambda t: t.data_ptr()
    out = torch.empty(len(inst.z), dtype=torch.float64, device=dev)
    assert L.ocp_eval_lagrangian_backward(prob._h, p(z), p(y), 0.8, p(gL), None, None, None, None, None,
                                          None) == ocp.OCP_ERR_ARG  # no output
    assert L.ocp_eval_lagrangian_backward(prob._h, p(z), p(y), 0.8, None, p(out), None, None, None, None,
                                          None) == ocp.OCP_ERR_ARG  # no incoming gradient
    assert L.ocp_eval_lagrangian_backward(prob._h, p(z), p(y), 0.8, p(gL), None, None, p(out), None, None,
                                          None) == ocp.OCP_ERR_ARG  # incomplete (or, quadrotor, any) coefficients
    with pytest.raises(ValueError):
        prob.lagrangian_backward(z, y, 0.8, gL, False, False, False)
    prob.close()


def test_backward_uses_its_own_forwards_coefficients(ocp):
    """The backward skips the coefficient upload only while its forward's
    upload is the handle's last one.  Two graphs on one handle with different
    coefficients, and an explicit upload between a forward and its backward:
    every gradient equals, bit for bit, that of a forward + backward run on
    its own (first and second order)."""
    from paper_2510_03932_amd.autograd import lagrangian, lagrangian_grad
    _say("[autograd] interleaved graphs on one handle")
    inst = synth.make_instance(700, 5, 2, seed=41, scheme=0, bnd=1)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    first, second = _leaf_inputs(inst, dev), _leaf_inputs(inst, dev)
    with torch.no_grad():
        second[2].mul_(1.5)
        second[3].add_(0.5)
        second[4].mul_(-2.0)
    grads = lambda L, x: torch.autograd.grad(L, x)
    want = [grads(lagrangian(prob, *x, 0.8), x) for x in (first, second)]
    L1 = lagrangian(prob, *first, 0.8)
    L2 = lagrangian(prob, *second, 0.8)  # the handle now holds the second coefficients
    got = [grads(L1, first), grads(L2, second)]
    L1 = lagrangian(prob, *first, 0.8)
    prob.set_coefficients(*(t.detach() for t in second[2:]))
    got.append(grads(L1, first))
    for g, w in zip(got, [want[0], want[1], want[0]]):
        for a, b in zip(g, w):
            assert torch.equal(a.view(torch.int64), b.view(torch.int64))
    # second order: H v through grad_z L after another graph's forward
    v = torch.from_numpy(np.random.default_rng(3).normal(size=len(inst.z))).to(dev)
    hv_want = torch.autograd.grad(lagrangian_grad(prob, *first, 0.8), first[0], v)[0]
    gz = lagrangian_grad(prob, *first, 0.8)
    lagrangian(prob, *second, 0.8)
    hv_got = torch.autograd.grad(gz, first[0], v)[0]
    assert torch.equal(hv_got.view(torch.int64), hv_want.view(torch.int64))
    prob.close()


def test_autograd_backward_matches_oracle(ocp):
    from paper_2510_03932_amd.autograd import lagrangian
    inst = synth.make_instance(2000, 6, 3, seed=6)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y, A, B, g = _leaf_inputs(inst, dev)
    L = lagrangian(prob, z, y, A, B, g, 0.9)
    L.backward()
    want, mu = oracle.lag_grad(inst, sigma=0.9)
    check_close(z.grad.cpu().numpy(), want, mu, what="z.grad")
    want, mu = oracle.cons(inst)
    check_close(y.grad.cpu().numpy(), want, mu, what="y.grad")
    (oA, oB, og), (mA, mB, mg) = oracle.coef_grad(inst)
    check_close(A.grad.cpu().numpy(), oA, mA, what="A.grad")
    check_close(B.grad.cpu().numpy(), oB, mB, what="B.grad")
    check_close(g.grad.cpu().numpy(), og, mg, what="gamma.grad")
    Lo, Lm = oracle.lagrangian(inst, sigma=0.9)
    assert abs(L.item() - Lo) <= 1e-12 * Lm
    prob.close()


@pytest.mark.parametrize("N,n,m,scheme,bnd", [(4, 3, 2, 0, 0), (3, 1, 1, 0, 0), (5, 2, 0, 0, 0),
                                              (4, 3, 2, 1, 2), (3, 1, 1, 1, 1), (5, 2, 0, 0, 2),
                                              (4, 2, 1, 1, 0)])
def test_autograd_gradcheck(ocp, N, n, m, scheme, bnd):
    from paper_2510_03932_amd.autograd import constraints, lagrangian, lagrangian_grad
    inst = synth.make_instance(N, n, m, seed=7, scheme=scheme, bnd=bnd)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y, A, B, g = _leaf_inputs(inst, dev)
    if m == 0:  # an empty B takes no part in a gradient check
        B = B.detach()
        f = lambda z, y, A, g: lagrangian(prob, z, y, A, B, g, 1.2)
        assert torch.autograd.gradcheck(f, (z, y, A, g), eps=1e-6, atol=1e-6, rtol=1e-5)
    else:
        f = lambda z, y, A, B, g: lagrangian(prob, z, y, A, B, g, 1.2)
        assert torch.autograd.gradcheck(f, (z, y, A, B, g), eps=1e-6, atol=1e-6, rtol=1e-5)
    z, y, A, B, g = _leaf_inputs(inst, dev, coef_grad=False)
    f2 = lambda z, y: lagrangian(prob, z, y, A, B, g, 1.2)
    assert torch.autograd.gradgradcheck(f2, (z, y), eps=1e-6, atol=1e-6, rtol=1e-5)
    # second order in every input: the mixed terms through grad_z L and the
    # derivatives of dL/dtheta in z and y
    z, y, A, B, g = _leaf_inputs(inst, dev)
    if m == 0:
        f3 = lambda z, y, A, g: lagrangian(prob, z, y, A, B.detach(), g, 1.2)
        assert torch.autograd.gradgradcheck(f3, (z, y, A, g), eps=1e-6, atol=1e-6, rtol=1e-5)
    else:
        f3 = lambda z, y, A, B, g: lagrangian(prob, z, y, A, B, g, 1.2)
        assert torch.autograd.gradgradcheck(f3, (z, y, A, B, g), eps=1e-6, atol=1e-6, rtol=1e-5)
    fg = lambda z, y: lagrangian_grad(prob, z, y, A, B, g, 1.2)
    assert torch.autograd.gradcheck(fg, (z, y), eps=1e-6, atol=1e-6, rtol=1e-5)
    z, y, A, B, g = _leaf_inputs(inst, dev)
    # grad_z L in every input, the coefficients included (the mixed terms)
    if m == 0:
        fgc = lambda z, y, A, g: lagrangian_grad(prob, z, y, A, B.detach(), g, 1.2)
        assert torch.autograd.gradcheck(fgc, (z, y, A, g), eps=1e-6, atol=1e-6, rtol=1e-5)
    else:
        fgc = lambda z, y, A, B, g: lagrangian_grad(prob, z, y, A, B, g, 1.2)
        assert torch.autograd.gradcheck(fgc, (z, y, A, B, g), eps=1e-6, atol=1e-6, rtol=1e-5)
    if m == 0:
        B = B.detach()
        fc = lambda z, A, g: constraints(prob, z, A, B, g)
        assert torch.autograd.gradcheck(fc, (z, A, g), eps=1e-6, atol=1e-6, rtol=1e-5)
    else:
        fc = lambda z, A, B, g: constraints(prob, z, A, B, g)
        assert torch.autograd.gradcheck(fc, (z, A, B, g), eps=1e-6, atol=1e-6, rtol=1e-5)
    prob.close()


def test_hvp_with_detached_coefficients(ocp):
    """The documented way to a Hessian-vector product while the coefficients
    require grad elsewhere: build grad_z L with them detached."""
    from paper_2510_03932_amd.autograd import lagrangian_grad
    inst = synth.make_instance(3000, 5, 2, seed=9, scheme=1, bnd=1)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y, A, B, g = _leaf_inputs(inst, dev)
    v = np.random.default_rng(3).normal(size=len(inst.z))
    gz = lagrangian_grad(prob, z, y, A.detach(), B.detach(), g.detach(), 0.8)
    (hv,) = torch.autograd.grad(gz, z, torch.from_numpy(v).to(dev))
    want, mu = oracle.hvp_ex(inst, v, 1, 1, sigma=0.8)
    check_close(hv.detach().cpu().numpy(), want, mu, what="H v through autograd, detached coefficients")
    assert A.grad is None and B.grad is None and g.grad is None
    prob.close()


def test_second_order_through_grad_z_with_coefficients(ocp):
    """grad_z L built from L with the coefficients requiring grad: a backward
    with v gives H v, J v and the mixed terms d/dtheta (v^T grad_z L), each
    against the oracle."""
    from paper_2510_03932_amd.autograd import lagrangian
    inst = synth.make_instance(700, 5, 3, seed=8, scheme=1, bnd=2)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y, A, B, g = _leaf_inputs(inst, dev)
    v = np.random.default_rng(12).normal(size=len(inst.z))
    L = lagrangian(prob, z, y, A, B, g, 0.7)
    (gz,) = torch.autograd.grad(L, z, create_graph=True)
    hv, jv, hA, hB, hg = torch.autograd.grad(gz, (z, y, A, B, g), torch.from_numpy(v).to(dev))
    want, mu = oracle.hvp_ex(inst, v, 1, 2, sigma=0.7)
    check_close(hv.cpu().numpy(), want, mu, what="H v")
    want, mu = oracle.jvp_ex(inst, v, 1, 2)
    check_close(jv.cpu().numpy(), want, mu, what="J v")
    (oA, oB, og), (mA, mB, mg) = oracle.coef_mixed_ex(inst, v, 1, 2)
    check_close(hA.cpu().numpy().ravel(), oA.ravel(), mA.ravel(), what="mixed A")
    check_close(hB.cpu().numpy().ravel(), oB.ravel(), mB.ravel(), what="mixed B")
    check_close(hg.cpu().numpy(), og, mg, what="mixed gamma")
    prob.close()


def test_coefficient_gradient_differentiated_again(ocp):
    """dL/dtheta as a function of (z, y): for cotangents tb, the gradient of
    tb . dL/dtheta is the coefficient part of grad_z L and of c under the
    coefficients tb, against the oracle's grad_z L and c evaluated with
    coefficients tb and with zero coefficients (sigma = 0) and against the
    oracle's adjoint; the handle's coefficients are the original ones
    afterwards; a third derivative raises."""
    import dataclasses
    from paper_2510_03932_amd.autograd import lagrangian
    inst = synth.make_instance(600, 4, 2, seed=23, scheme=0, bnd=1)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y, A, B, g = _leaf_inputs(inst, dev)
    rng = np.random.default_rng(17)
    tA, tB, tg = rng.normal(size=(4, 4)), rng.normal(size=(4, 2)), rng.normal(size=4)
    L = lagrangian(prob, z, y, A, B, g, 0.9)
    dA, dB, dg = torch.autograd.grad(L, (A, B, g), create_graph=True)
    gz, gy = torch.autograd.grad((dA, dB, dg), (z, y), tuple(torch.from_numpy(t).to(dev) for t in (tA, tB, tg)))
    with_tb = dataclasses.replace(inst, A=tA, B=tB, gamma=tg)
    zero = dataclasses.replace(inst, A=0 * tA, B=0 * tB, gamma=0 * tg)
    (g1, m1), (g0, m0) = (oracle.lag_grad_ex(i, 0, 1, sigma=0.0) for i in (with_tb, zero))
    check_close(gz.cpu().numpy(), g1 - g0, m1 + m0, what="d/dz of tb . dL/dtheta")
    (c1, n1), (c0, n0) = (oracle.cons_ex(i, 0, 1) for i in (with_tb, zero))
    check_close(gy.cpu().numpy(), c1 - c0, n1 + n0, what="d/dy of tb . dL/dtheta")
    (oz, oy), (mz, my) = oracle.coef_adjoint_ex(inst, tA, tB, tg, 0, 1)
    check_close(gz.cpu().numpy(), oz, mz, what="d/dz against the oracle's adjoint")
    check_close(gy.cpu().numpy(), oy, my, what="d/dy against the oracle's adjoint")
    # the handle holds the original coefficients again
    Lo, Lm = oracle.lagrangian_ex(inst, 0, 1, sigma=0.9)
    assert abs(prob.lagrangian(z.detach(), y.detach(), 0.9).item() - Lo) <= 1e-12 * Lm
    L = lagrangian(prob, z, y, A, B, g)
    (dA,) = torch.autograd.grad(L, A, create_graph=True)
    with pytest.raises(NotImplementedError):  # a graph for third derivatives
        torch.autograd.grad(dA.sum(), z, create_graph=True)
    prob.close()


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("n,m", COEF_TILINGS)
def test_coef_mixed_every_tiling(ocp, n, m, scheme):
    """The mixed derivative for every tiling of the coefficient kernel, at
    N = 389 (several chunks, a ragged last one), with boundary rows."""
    N = 389
    _say(f"[coef mixed] N={N} n={n} m={m} scheme={scheme}")
    bnd = 1 + scheme
    inst = synth.make_instance(N, n, m, seed=17, scheme=scheme, bnd=bnd)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    v = np.random.default_rng(n + m).normal(size=len(inst.z))
    z, y, vt = (torch.from_numpy(a).to(dev) for a in (inst.z, inst.y, v))
    gA, gB, gg = (t.cpu().numpy() for t in prob.coef_mixed(z, y, vt))
    (oA, oB, og), (mA, mB, mg) = oracle.coef_mixed_ex(inst, v, scheme, bnd)
    tag = f"{N},{n},{m},{scheme}"
    check_close(gA.ravel(), oA.ravel(), mA.ravel(), what=f"mixed A {tag}")
    check_close(gB.ravel(), oB.ravel(), mB.ravel(), what=f"mixed B {tag}")
    check_close(gg, og, mg, what=f"mixed gamma {tag}")
    prob.close()


@pytest.mark.parametrize("N,n,m,scheme", [(600_001, 3, 0, 1), (270_000, 17, 9, 0)])
def test_coef_mixed_many_chunks_per_workgroup(ocp, N, n, m, scheme):
    """Several chunks per workgroup and a ragged last chunk; a second call
    gives the same bits."""
    _say(f"[coef mixed] N={N} n={n} m={m} scheme={scheme}")
    inst = synth.make_instance(N, n, m, seed=19, scheme=scheme)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    v = np.random.default_rng(4).normal(size=len(inst.z))
    z, y, vt = (torch.from_numpy(a).to(dev) for a in (inst.z, inst.y, v))
    got = [t.cpu().numpy() for t in prob.coef_mixed(z, y, vt)]
    again = [t.cpu().numpy() for t in prob.coef_mixed(z, y, vt)]
    for first, second in zip(got, again):
        assert np.array_equal(first.view(np.int64), second.view(np.int64))
    (oA, oB, og), (mA, mB, mg) = oracle.coef_mixed_ex(inst, v, scheme, 0)
    tag = f"{N},{n},{m},{scheme}"
    check_close(got[0].ravel(), oA.ravel(), mA.ravel(), what=f"mixed A {tag}")
    check_close(got[1].ravel(), oB.ravel(), mB.ravel(), what=f"mixed B {tag}")
    check_close(got[2], og, mg, what=f"mixed gamma {tag}")
    prob.close()


@pytest.mark.parametrize("N,n,m,scheme,bnd", [(1, 1, 0, 0, 0), (5, 1, 0, 1, 2), (3, 2, 1, 0, 1), (2, 1, 3, 1, 0)])
def test_coef_mixed_degenerate_shapes(ocp, N, n, m, scheme, bnd):
    """One or two intervals, one state (gamma's partner is the state itself:
    the product X_i X_p(i) is X_i^2), no controls."""
    _say(f"[coef mixed] N={N} n={n} m={m} scheme={scheme} bnd={bnd}")
    inst = synth.make_instance(N, n, m, seed=29, scheme=scheme, bnd=bnd)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    v = np.random.default_rng(N + 10 * n).normal(size=len(inst.z))
    z, y, vt = (torch.from_numpy(a).to(dev) for a in (inst.z, inst.y, v))
    for got, (want, mu) in ((prob.coef_mixed(z, y, vt), oracle.coef_mixed_ex(inst, v, scheme, bnd)),
                            (prob.coef_grad(z, y), oracle.coef_grad_ex(inst, scheme, bnd))):
        for g, w, u, what in zip(got, want, mu, ("A", "B", "gamma")):
            check_close(g.cpu().numpy().ravel(), w.ravel(), u.ravel(), what=f"{what} {N},{n},{m}")
    prob.close()


def test_coef_mixed_rejects_quadrotor_and_null(ocp):
    q = synth.make_quadrotor(8, seed=0, bnd=1)
    dev = torch.device("cuda", 0)
    qp = ocp.QuadrotorProblem.from_instance(q, dev)
    z, y = torch.from_numpy(q.z).to(dev), torch.from_numpy(q.y).to(dev)
    with pytest.raises(ocp.OcpError):
        qp.coef_mixed(z, y, z.clone())
    qp.close()
    inst = synth.make_instance(10, 2, 1, seed=1)
    prob = ocp.Problem.from_instance(inst, dev)
    out = torch.empty(8, dtype=torch.float64, device=dev)
    rc = ocp.lib().ocp_eval_coef_mixed(prob._h, None, None, None, out.data_ptr(), out.data_ptr(),
                                       out.data_ptr(), None)
    assert rc == ocp.OCP_ERR_ARG
    prob.close()


def _cotangents(n, m, seed, dev):
    rng = np.random.default_rng(seed)
    t = rng.normal(size=(n, n)), rng.normal(size=(n, m)), rng.normal(size=n)
    return t, tuple(torch.from_numpy(a).to(dev) for a in t)


def _check_adjoint(ocp, inst, scheme, bnd, seed, tag):
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    (tA, tB, tg), dt = _cotangents(inst.n, inst.m, seed, dev)
    z, y = torch.from_numpy(inst.z).to(dev), torch.from_numpy(inst.y).to(dev)
    gz, gy = prob.coef_adjoint(z, y, *dt)
    (oz, oy), (mz, my) = oracle.coef_adjoint_ex(inst, tA, tB, tg, scheme, bnd)
    gz, gy = gz.cpu().numpy(), gy.cpu().numpy()
    check_close(gz, oz, mz, what=f"adjoint in z {tag}")
    check_close(gy, oy, my, what=f"adjoint in y {tag}")
    return prob, z, y, dt, gz, gy


ADJ_SHAPES = [(1000, 4, 2), (777, 5, 3), (1, 1, 0), (1, 1, 1), (2, 2, 1), (3, 3, 0), (255, 2, 0),
              (510, 8, 4), (257, 16, 8), (513, 32, 32), (300, 9, 4), (389, 17, 15)]


@pytest.mark.parametrize("scheme,bnd", [(0, 0), (0, 2), (1, 1), (1, 2)])
@pytest.mark.parametrize("N,n,m", ADJ_SHAPES)
def test_coef_adjoint_matches_oracle(ocp, N, n, m, scheme, bnd):
    """Every register tiling (n up to 4, 8, 16, 32), one or several chunks
    of 256 nodes with a ragged last one (N = 255 and 510 end exactly at a
    chunk's last node), one state (X_i X_p(i) = X_i^2), no controls, either
    scheme and boundary rows."""
    tag = f"N={N} n={n} m={m} scheme={scheme} bnd={bnd}"
    _say(f"[coef adjoint] {tag}")
    inst = synth.make_instance(N, n, m, seed=31 + n, scheme=scheme, bnd=bnd)
    prob, *_ = _check_adjoint(ocp, inst, scheme, bnd, 7 + N, tag)
    prob.close()


def test_coef_adjoint_differentiation_workload(ocp):
    """At the 2e5-interval differentiation workload, every entry; a second
    call gives the same bits; each output alone equals the joint call's."""
    N, n, m = synth.DIFF
    _say(f"[coef adjoint] N={N} n={n} m={m}")
    inst = synth.make_instance(N, n, m, seed=0)
    prob, z, y, dt, gz, gy = _check_adjoint(ocp, inst, 0, 0, 3, f"N={N}")
    gz2, gy2 = (t.cpu().numpy() for t in prob.coef_adjoint(z, y, *dt))
    assert np.array_equal(gz.view(np.int64), gz2.view(np.int64))
    assert np.array_equal(gy.view(np.int64), gy2.view(np.int64))
    only_z, none_y = prob.coef_adjoint(z, y, *dt, want_y=False)
    none_z, only_y = prob.coef_adjoint(z, y, *dt, want_z=False)
    assert none_y is None and none_z is None
    assert np.array_equal(only_z.cpu().numpy().view(np.int64), gz.view(np.int64))
    assert np.array_equal(only_y.cpu().numpy().view(np.int64), gy.view(np.int64))
    prob.close()


def test_coef_adjoint_leaves_the_handle_alone(ocp):
    """The adjoint reads the cotangents from the caller's arrays: the
    handle's own coefficients (hence every other evaluation) are the same
    bits before and after, and a different cotangent gives a different
    result (nothing is cached)."""
    _say("[coef adjoint] handle untouched")
    inst = synth.make_instance(300, 5, 2, seed=8, scheme=0, bnd=1)
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y = torch.from_numpy(inst.z).to(dev), torch.from_numpy(inst.y).to(dev)
    before = prob.lag_grad(z, y, 0.7).cpu().numpy()
    _, dt = _cotangents(5, 2, 1, dev)
    g1 = prob.coef_adjoint(z, y, *dt)[0].cpu().numpy()
    g2 = prob.coef_adjoint(z, y, *(2.0 * t for t in dt))[0].cpu().numpy()
    after = prob.lag_grad(z, y, 0.7).cpu().numpy()
    assert np.array_equal(before.view(np.int64), after.view(np.int64))
    check_close(g2, 2.0 * g1, 2.0 * np.abs(g1) + 1e-300, rel=1e-15, what="linear in t")
    prob.close()


def test_coef_adjoint_overlaps_coefficient_uploads(ocp):
    """The adjoint reads no coefficient of the handle, so it may overlap any
    other call on it: adjoints issued on one stream while another stream
    keeps uploading different coefficients into the same handle equal, bit
    for bit, the adjoint computed alone."""
    _say("[coef adjoint] overlapping uploads on another stream")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(20_000, 6, 3, seed=12)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y = torch.from_numpy(inst.z).to(dev), torch.from_numpy(inst.y).to(dev)
    _, dt = _cotangents(6, 3, 9, dev)
    want = prob.coef_adjoint(z, y, *dt)
    coefs = [tuple(torch.from_numpy(np.array(a) * s).to(dev) for a in (inst.A, inst.B, inst.gamma))
             for s in (1.0, -3.0)]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(dev), torch.cuda.Stream(dev)  # default priority
    got = []
    for r in range(20):
        with torch.cuda.stream(s2):
            prob.set_coefficients(*coefs[r % 2])
        with torch.cuda.stream(s1):
            got.append(prob.coef_adjoint(z, y, *dt))
    torch.cuda.synchronize()
    for gz, gy in got:
        assert torch.equal(gz.view(torch.int64), want[0].view(torch.int64))
        assert torch.equal(gy.view(torch.int64), want[1].view(torch.int64))
    prob.close()


def test_coef_adjoint_rejects_quadrotor_null_and_no_output(ocp):
    q = synth.make_quadrotor(8, seed=0, bnd=1)
    dev = torch.device("cuda", 0)
    qp = ocp.QuadrotorProblem.from_instance(q, dev)
    z, y = torch.from_numpy(q.z).to(dev), torch.from_numpy(q.y).to(dev)
    t = torch.zeros(81, dtype=torch.float64, device=dev)
    rc = ocp.lib().ocp_eval_coef_adjoint(qp._h, z.data_ptr(), y.data_ptr(), t.data_ptr(), t.data_ptr(),
                                         t.data_ptr(), t.data_ptr(), None, None)
    assert rc == ocp.OCP_ERR_ARG
    qp.close()
    inst = synth.make_instance(10, 2, 1, seed=1)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y = torch.from_numpy(inst.z).to(dev), torch.from_numpy(inst.y).to(dev)
    out = torch.empty(len(inst.z), dtype=torch.float64, device=dev)
    L = ocp.lib()
    assert L.ocp_eval_coef_adjoint(prob._h, z.data_ptr(), y.data_ptr(), None, t.data_ptr(), t.data_ptr(),
                                   out.data_ptr(), None, None) == ocp.OCP_ERR_ARG
    assert L.ocp_eval_coef_adjoint(prob._h, z.data_ptr(), y.data_ptr(), t.data_ptr(), None, t.data_ptr(),
                                   out.data_ptr(), None, None) == ocp.OCP_ERR_ARG
    assert L.ocp_eval_coef_adjoint(prob._h, z.data_ptr(), y.data_ptr(), t.data_ptr(), t.data_ptr(),
                                   t.data_ptr(), None, None, None) == ocp.OCP_ERR_ARG
    with pytest.raises(ValueError):
        prob.coef_adjoint(z, y, t[:4].view(2, 2), t[:2].view(2, 1), t[:2], want_z=False, want_y=False)
    prob.close()


def test_differentiation_workload_central_differences(ocp):
    """On the 2e5-interval workload, with the GPU's own Lagrangian:
    - central differences at step 1e-6 along sampled entries of z against
      grad_z L (a local perturbation: the unchanged terms round identically
      in both evaluations, so the difference resolves the derivative);
    - central differences of grad_z L along v (step 1e-6) against H v;
    - the coefficients: L is affine in (A, B, gamma), so a central difference
      is exact at any step up to the rounding of L, which is eps * mu_L with
      mu_L the sum of |terms| (2e6 here against |L| = 8.6).  Every coefficient
      perturbs every term, so the step is 1.0 to keep that rounding far below
      the derivative."""
    N, n, m = synth.DIFF
    inst = synth.make_instance(N, n, m, seed=0)
    dev, z, y, v, vt = _dev_inputs(inst, seed=9)
    prob = ocp.Problem.from_instance(inst, dev)
    _, muL = oracle.lagrangian(inst)
    eps = np.finfo(float).eps
    step = 1e-6
    g = prob.lag_grad(z, y, 1.0)
    L0 = abs(prob.lagrangian(z, y, 1.0).item())
    for e in np.random.default_rng(10).choice(len(inst.z), 24, replace=False).tolist() + [0, N, len(inst.z) - 1]:
        zp, zm = z.clone(), z.clone()
        zp[e] += step
        zm[e] -= step
        fd = (prob.lagrangian(zp, y, 1.0).item() - prob.lagrangian(zm, y, 1.0).item()) / (2 * step)
        assert abs(fd - g[e].item()) <= 64 * eps * L0 / step + 1e-6 * abs(g[e].item()), e
    hv = prob.hvp(z, y, vt, 1.0)
    fd = (prob.lag_grad(z + step * vt, y, 1.0) - prob.lag_grad(z - step * vt, y, 1.0)) / (2 * step)
    # the entries of grad_z L are O(1) while H v is O(h): the difference's
    # rounding, eps * mu(grad_z L) / step per entry, bounds the comparison
    _, mug = oracle.lag_grad(inst)
    bound = 16 * eps * torch.from_numpy(mug).to(dev) / step + 1e-6 * hv.abs().max()
    assert bool(((fd - hv).abs() <= bound).all())
    gA, gB, gg = (t.cpu().numpy() for t in prob.coef_grad(z, y))
    A0, B0, g0 = (torch.from_numpy(a).to(dev) for a in (inst.A, inst.B, inst.gamma))
    cstep = 1.0
    bound = 64 * eps * muL / cstep
    for name, base, grad in (("A", A0, gA), ("B", B0, gB), ("gamma", g0, gg)):
        flat = base.reshape(-1)
        for idx in range(flat.numel()):
            vals = []
            for sgn in (1, -1):
                pert = flat.clone()
                pert[idx] += sgn * cstep
                args = {"A": A0, "B": B0, "gamma": g0}
                args[name] = pert.reshape(base.shape)
                prob.set_coefficients(args["A"], args["B"], args["gamma"])
                vals.append(prob.lagrangian(z, y, 1.0).item())
            fd = (vals[0] - vals[1]) / (2 * cstep)
            assert abs(fd - grad.reshape(-1)[idx]) <= bound, (name, idx, fd, grad.reshape(-1)[idx])
    prob.set_coefficients(A0, B0, g0)
    prob.close()
