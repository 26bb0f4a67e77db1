"""Pins of the oracle's Lagrangian derivatives (the differentiation workload):
L = sigma f + y^T c, grad_z L, (Hessian of L) v, J v and dL/d(A, B, gamma),
each against a high-precision evaluation, complex-step or finite differences
of the independent definition module."""
from __future__ import annotations

import cmath

import numpy as np
import pytest

from oracle import defn
from tests.helpers import EPS, check_close, instance, mixed_hessian

SHAPES = [(1, 1, 0), (2, 1, 1), (3, 2, 1), (4, 3, 1), (5, 4, 2), (3, 5, 0), (6, 3, 3)]


def _L(inst, z, y, sigma, A=None, B=None, gamma=None, sin=cmath.sin):
    A0, B0, g0, q, r = defn.as_lists(inst)
    return defn.lagrangian(z, y, sigma, inst.N, inst.n, inst.m, A if A is not None else A0,
                           B if B is not None else B0, gamma if gamma is not None else g0, q, r,
                           sin=sin)


@pytest.mark.parametrize("N,n,m", [(7, 3, 2), (40, 4, 2), (1, 2, 1)])
def test_lagrangian_value_high_precision(orc, N, n, m):
    import mpmath
    mpmath.mp.dps = 50
    inst = instance(N, n, m, seed=50 + N)
    Lo, mu = orc.lagrangian(inst, sigma=1.3)
    mp = mpmath.mpf
    A, B, g, q, r = defn.as_lists(inst)
    cv = lambda x: [mp(v) for v in x]
    want = defn.lagrangian(cv(inst.z), cv(inst.y), mp(1.3), N, n, m, [cv(a) for a in A],
                           [cv(b) for b in B], cv(g), cv(q), cv(r), sin=mpmath.sin, dt=mp(1.0 / N))
    assert abs(Lo - float(want)) <= 1e-13 * mu


@pytest.mark.parametrize("N,n,m", SHAPES)
def test_lag_grad_complex_step(orc, N, n, m):
    inst = instance(N, n, m, seed=60 + N + n)
    sigma = 0.8
    g, mu = orc.lag_grad(inst, sigma=sigma)
    tau = 1e-30
    y = list(map(float, inst.y))
    cs = []
    for col in range(len(inst.z)):
        z = [complex(v) for v in inst.z]
        z[col] += 1j * tau
        cs.append(_L(inst, z, y, sigma).imag / tau)
    check_close(g, np.array(cs), mu, rel=1e-13, what="grad_z L")


def test_lag_grad_sampled_at_parity_size(orc):
    inst = instance(1000, 4, 2, seed=61)
    g, mu = orc.lag_grad(inst)
    tau = 1e-30
    y = list(map(float, inst.y))
    for col in (0, 1, 500, 1000, 1001, 2002, 4004, 5005, len(inst.z) - 1):
        z = [complex(v) for v in inst.z]
        z[col] += 1j * tau
        want = _L(inst, z, y, inst.sigma).imag / tau
        assert abs(g[col] - want) <= 1e-13 * mu[col], col


@pytest.mark.parametrize("N,n,m", [(1, 1, 1), (3, 1, 0), (3, 2, 1), (2, 3, 1), (2, 4, 2)])
def test_hvp_mixed_difference(orc, N, n, m):
    inst = instance(N, n, m, seed=70 + N + n)
    v = np.random.default_rng(1).normal(size=len(inst.z))
    hv, mu = orc.hvp(inst, v, sigma=1.1)
    H = mixed_hessian(inst, inst.y, 1.1)
    want = H @ v
    scale = np.abs(H).max() * np.abs(v).max()
    assert np.abs(hv - want).max() <= 1e-8 * scale


def test_hvp_node_ranges(orc):
    inst = instance(300, 5, 2, seed=71)
    v = np.random.default_rng(2).normal(size=len(inst.z))
    full = orc.hvp(inst, v)[0].reshape(7, 301)
    part = orc.hvp(inst, v, 100, 200)[0].reshape(7, 100)
    assert np.array_equal(full[:, 100:200], part)


@pytest.mark.parametrize("N,n,m", SHAPES + [(1000, 4, 2)])
def test_jvp_complex_step(orc, N, n, m):
    """J v is the directional derivative of c: Im c(z + i tau v) / tau."""
    inst = instance(N, n, m, seed=80 + N)
    v = np.random.default_rng(3).normal(size=len(inst.z))
    jv, mu = orc.jvp(inst, v)
    A, B, g, q, r = defn.as_lists(inst)
    tau = 1e-30
    z = [complex(a, tau * b) for a, b in zip(inst.z, v)]
    c = defn.constraints(z, N, n, m, A, B, g, sin=cmath.sin)
    check_close(jv, np.array([x.imag / tau for x in c]), mu, rel=1e-13, what="J v")


@pytest.mark.parametrize("N,n,m", [(5, 3, 2), (6, 1, 1), (4, 2, 0), (300, 4, 2)])
def test_coef_grad_complex_step_and_central_difference(orc, N, n, m):
    """L is affine in (A, B, gamma): complex step is exact to rounding, and so
    is a central difference at step 1e-6 up to its cancellation error."""
    inst = instance(N, n, m, seed=90 + N)
    (gA, gB, gg), (mA, mB, mg) = orc.coef_grad(inst)
    A, B, g, q, r = defn.as_lists(inst)
    y = list(map(float, inst.y))
    z = list(map(float, inst.z))
    tau, step = 1e-30, 1e-6
    L0 = abs(_L(inst, z, y, inst.sigma, sin=np.sin))
    for i in range(n):
        for j in range(n):
            Ac = [[complex(v) for v in row] for row in A]
            Ac[i][j] += 1j * tau
            want = _L(inst, z, y, inst.sigma, A=Ac).imag / tau
            assert abs(gA[i, j] - want) <= 1e-13 * mA[i, j] + 1e-300
            Ap = [row[:] for row in A]
            Am = [row[:] for row in A]
            Ap[i][j] += step
            Am[i][j] -= step
            fd = (_L(inst, z, y, inst.sigma, A=Ap, sin=np.sin)
                  - _L(inst, z, y, inst.sigma, A=Am, sin=np.sin)) / (2 * step)
            assert abs(gA[i, j] - fd) <= 64 * EPS * L0 / step
        for l in range(m):
            Bc = [[complex(v) for v in row] for row in B]
            Bc[i][l] += 1j * tau
            want = _L(inst, z, y, inst.sigma, B=Bc).imag / tau
            assert abs(gB[i, l] - want) <= 1e-13 * mB[i, l] + 1e-300
        gc = [complex(v) for v in g]
        gc[i] += 1j * tau
        want = _L(inst, z, y, inst.sigma, gamma=gc).imag / tau
        assert abs(gg[i] - want) <= 1e-13 * mg[i] + 1e-300


def test_coef_grad_thread_independent(orc):
    inst = instance(20_000, 4, 2, seed=91)
    t0 = orc.get_threads()
    try:
        orc.set_threads(1)
        a = orc.coef_grad(inst)[0]
        orc.set_threads(8)
        b = orc.coef_grad(inst)[0]
    finally:
        orc.set_threads(t0)
    for u, w in zip(a, b):
        assert np.array_equal(u, w)


def test_lag_grad_equals_sigma_grad_plus_jt_y(orc):
    """Consistency with the separately pinned gradient and Jacobian: grad_z L =
    sigma grad f + J^T y (J^T y accumulated from the COO pattern)."""
    inst = instance(500, 5, 3, seed=92)
    sigma = 0.6
    g, mu = orc.lag_grad(inst, sigma=sigma)
    gf, _ = orc.grad(inst)
    jv, jm = orc.jac(inst)
    jrow, jcol, _, _ = orc.pattern(inst.N, inst.n, inst.m)
    jty = np.zeros(len(inst.z))
    np.add.at(jty, jcol, jv * inst.y[jrow])
    check_close(g, sigma * gf + jty, mu, rel=1e-13, what="grad_z L vs sigma grad + J^T y")
