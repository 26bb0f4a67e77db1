"""Pins of the oracle's Lagrangian derivatives under every scheme and boundary
option (trapezoidal or forward Euler; no boundary rows, initial-state rows,
or initial- and final-state rows): L = sigma f + y^T c, grad_z L, (Hessian
of L) v, J v and dL/d(A, B, gamma), against a 50-digit evaluation,
complex-step and mixed differences of the independent definition module, and
against the C oracle's own trapezoidal functions; and the same derivatives
(no coefficients there) of the quadrotor model."""
from __future__ import annotations

import cmath
import math
import types

import numpy as np
import pytest

import synth
from oracle import defn
from tests.helpers import check_close

CASES = [(scheme, bnd) for scheme in (0, 1) for bnd in (0, 1, 2)]
SHAPES = [(1, 1, 0), (2, 1, 1), (3, 2, 1), (4, 3, 1), (3, 5, 0), (5, 3, 2)]


def _inst(N, n, m, seed, scheme, bnd):
    return synth.make_instance(N, n, m, seed=seed, scheme=scheme, bnd=bnd)


def _L(inst, z, y, sigma, A=None, B=None, gamma=None, sin=cmath.sin):
    A0, B0, g0, q, r = defn.as_lists(inst)
    return defn.lagrangian_ex(z, y, sigma, inst.N, inst.n, inst.m, A if A is not None else A0,
                              B if B is not None else B0, gamma if gamma is not None else g0, q, r,
                              inst.scheme, inst.bnd, sin=sin)


@pytest.mark.parametrize("scheme,bnd", CASES)
def test_lagrangian_ex_high_precision(orc, scheme, bnd):
    import mpmath
    mpmath.mp.dps = 50
    inst = _inst(9, 3, 2, 200 + 3 * scheme + bnd, scheme, bnd)
    Lo, mu = orc.lagrangian_ex(inst, scheme, bnd, sigma=1.3)
    mp = mpmath.mpf
    A, B, g, q, r = defn.as_lists(inst)
    cv = lambda x: [mp(v) for v in x]
    want = defn.lagrangian_ex(cv(inst.z), cv(inst.y), mp(1.3), inst.N, 3, 2, [cv(a) for a in A],
                              [cv(b) for b in B], cv(g), cv(q), cv(r), scheme, bnd, sin=mpmath.sin,
                              dt=mp(1) / inst.N)
    assert abs(Lo - float(want)) <= 1e-13 * mu


@pytest.mark.parametrize("scheme,bnd", CASES)
@pytest.mark.parametrize("N,n,m", SHAPES)
def test_lag_grad_ex_complex_step(orc, N, n, m, scheme, bnd):
    inst = _inst(N, n, m, 210 + N + n, scheme, bnd)
    sigma = 0.8
    g, mu = orc.lag_grad_ex(inst, scheme, bnd, sigma=sigma)
    tau = 1e-30
    y = list(map(float, inst.y))
    cs = []
    for col in range(len(inst.z)):
        z = [complex(v) for v in inst.z]
        z[col] += 1j * tau
        cs.append(_L(inst, z, y, sigma).imag / tau)
    check_close(g, np.array(cs), mu, rel=1e-13, what=f"grad_z L scheme={scheme} bnd={bnd}")


@pytest.mark.parametrize("scheme,bnd", CASES)
@pytest.mark.parametrize("N,n,m", SHAPES)
def test_jvp_ex_complex_step(orc, N, n, m, scheme, bnd):
    """J v is the directional derivative of c: Im c(z + i tau v) / tau."""
    inst = _inst(N, n, m, 220 + N + n, scheme, bnd)
    v = np.random.default_rng(4).normal(size=len(inst.z))
    jv, mu = orc.jvp_ex(inst, v, scheme, bnd)
    A, B, g, q, r = defn.as_lists(inst)
    tau = 1e-30
    z = [complex(a, tau * b) for a, b in zip(inst.z, v)]
    c = defn.constraints_ex(z, N, n, m, A, B, g, scheme, bnd, sin=cmath.sin)
    check_close(jv, np.array([x.imag / tau for x in c]), mu, rel=1e-13, what="J v")


@pytest.mark.parametrize("scheme,bnd", CASES)
@pytest.mark.parametrize("N,n,m", [(1, 1, 1), (3, 1, 0), (3, 2, 1), (2, 3, 1), (2, 4, 2)])
def test_hvp_ex_mixed_difference(orc, N, n, m, scheme, bnd):
    """(H v)_a = d/dz_a of the directional derivative of L along v: complex
    step in z_a, central difference (step 1e-5) along v."""
    inst = _inst(N, n, m, 230 + N + n, scheme, bnd)
    sigma = 1.1
    v = np.random.default_rng(5).normal(size=len(inst.z))
    hv, mu = orc.hvp_ex(inst, v, scheme, bnd, sigma=sigma)
    tau, delta = 1e-30, 1e-5
    y = list(map(float, inst.y))
    want = np.empty(len(inst.z))
    for a in range(len(inst.z)):
        vals = []
        for s in (+1, -1):
            z = [complex(x + s * delta * d) for x, d in zip(inst.z, v)]
            z[a] += 1j * tau
            vals.append(_L(inst, z, y, sigma).imag)
        want[a] = (vals[0] - vals[1]) / (2 * tau * delta)
    scale = max(float(np.max(mu)), 1.0)
    assert np.max(np.abs(hv - want)) <= 1e-7 * scale


@pytest.mark.parametrize("scheme,bnd", CASES)
@pytest.mark.parametrize("N,n,m", [(5, 3, 2), (6, 1, 1), (4, 2, 0), (40, 4, 2)])
def test_coef_grad_ex_complex_step(orc, N, n, m, scheme, bnd):
    """L is affine in (A, B, gamma): the complex step is exact to rounding."""
    inst = _inst(N, n, m, 240 + N, scheme, bnd)
    (gA, gB, gg), (mA, mB, mg) = orc.coef_grad_ex(inst, scheme, bnd)
    A, B, g, q, r = defn.as_lists(inst)
    y = list(map(float, inst.y))
    z = list(map(float, inst.z))
    tau = 1e-30
    for i in range(n):
        for j in range(n):
            Ac = [[complex(v) for v in row] for row in A]
            Ac[i][j] += 1j * tau
            want = _L(inst, z, y, inst.sigma, A=Ac).imag / tau
            assert abs(gA[i, j] - want) <= 1e-13 * mA[i, j] + 1e-300, ("A", i, j)
        for l in range(m):
            Bc = [[complex(v) for v in row] for row in B]
            Bc[i][l] += 1j * tau
            want = _L(inst, z, y, inst.sigma, B=Bc).imag / tau
            assert abs(gB[i, l] - want) <= 1e-13 * mB[i, l] + 1e-300, ("B", i, l)
        gc = [complex(v) for v in g]
        gc[i] += 1j * tau
        want = _L(inst, z, y, inst.sigma, gamma=gc).imag / tau
        assert abs(gg[i] - want) <= 1e-13 * mg[i] + 1e-300, ("gamma", i)


@pytest.mark.parametrize("scheme,bnd", CASES)
@pytest.mark.parametrize("N,n,m", [(4, 3, 2), (3, 1, 1), (3, 2, 0)])
def test_coef_mixed_ex_high_precision_differences(orc, N, n, m, scheme, bnd):
    """d/dtheta_p (v . grad_z L) from 50-digit evaluations of the definition
    module: L is affine in theta, so L(theta + e_p) - L(theta) is the
    coefficient's derivative g_p exactly, and the central difference of g_p
    along v at step 1e-20 is exact to far below double rounding."""
    import mpmath
    mpmath.mp.dps = 50
    inst = _inst(N, n, m, 260 + 7 * N + n, scheme, bnd)
    v = np.random.default_rng(31 + N).normal(size=len(inst.z))
    (gA, gB, gg), (mA, mB, mg) = orc.coef_mixed_ex(inst, v, scheme, bnd)
    mp = mpmath.mpf
    A, B, g, q, r = defn.as_lists(inst)
    cv = lambda x: [mp(float(t)) for t in x]
    eps = mp("1e-20")
    zp = [mp(float(a)) + eps * mp(float(b)) for a, b in zip(inst.z, v)]
    zm = [mp(float(a)) - eps * mp(float(b)) for a, b in zip(inst.z, v)]
    yy, qq, rr = cv(inst.y), cv(q), cv(r)
    A0, B0, g0 = [cv(a) for a in A], [cv(b) for b in B], cv(g)

    def L(z, A_, B_, g_):
        return defn.lagrangian_ex(z, yy, mp(float(inst.sigma)), N, n, m, A_, B_, g_, qq, rr, scheme, bnd,
                                  sin=mpmath.sin, dt=mp(1) / N)

    base = L(zp, A0, B0, g0) - L(zm, A0, B0, g0)

    def want(A_, B_, g_):
        return float((L(zp, A_, B_, g_) - L(zm, A_, B_, g_) - base) / (2 * eps))

    for i in range(n):
        for j in range(n):
            A1 = [row[:] for row in A0]
            A1[i][j] += 1
            assert abs(gA[i, j] - want(A1, B0, g0)) <= 1e-13 * mA[i, j] + 1e-300, ("A", i, j)
        for l in range(m):
            B1 = [row[:] for row in B0]
            B1[i][l] += 1
            assert abs(gB[i, l] - want(A0, B1, g0)) <= 1e-13 * mB[i, l] + 1e-300, ("B", i, l)
        g1 = g0[:]
        g1[i] += 1
        assert abs(gg[i] - want(A0, B0, g1)) <= 1e-13 * mg[i] + 1e-300, ("gamma", i)


def test_coef_mixed_ex_linear_in_v_and_zero_without_state_direction(orc):
    """The mixed derivative is linear in v; a direction that moves only the
    controls leaves the A and gamma parts zero (they depend on the states
    alone) and gives B's part as the coefficient gradient of a problem whose
    controls are v's control part (dL/dB is linear in U)."""
    inst = _inst(30, 4, 2, 271, 0, 1)
    rng = np.random.default_rng(8)
    v1, v2 = rng.normal(size=len(inst.z)), rng.normal(size=len(inst.z))
    (a1, b1, g1), (ma1, mb1, mg1) = orc.coef_mixed_ex(inst, v1, 0, 1)
    (a2, b2, g2), (ma2, mb2, mg2) = orc.coef_mixed_ex(inst, v2, 0, 1)
    (a3, b3, g3), _ = orc.coef_mixed_ex(inst, 2.0 * v1 - 3.0 * v2, 0, 1)
    check_close(a3.ravel(), (2 * a1 - 3 * a2).ravel(), (2 * ma1 + 3 * ma2).ravel(), rel=1e-13, what="A linear")
    check_close(b3.ravel(), (2 * b1 - 3 * b2).ravel(), (2 * mb1 + 3 * mb2).ravel(), rel=1e-13, what="B linear")
    check_close(g3, 2 * g1 - 3 * g2, 2 * mg1 + 3 * mg2, rel=1e-13, what="gamma linear")
    nx = inst.n * (inst.N + 1)
    vu = np.zeros(len(inst.z))
    vu[nx:] = v1[nx:]
    (a, b, g), _ = orc.coef_mixed_ex(inst, vu, 0, 1)
    assert np.all(a == 0.0) and np.all(g == 0.0)
    swapped = types.SimpleNamespace(**{k: getattr(inst, k) for k in ("N", "n", "m", "y", "A", "B", "gamma")})
    swapped.z = np.concatenate([np.asarray(inst.z[:nx], dtype=float), vu[nx:]])
    (_, bw, _), (_, mbw, _) = orc.coef_grad_ex(swapped, 0, 1)
    check_close(b.ravel(), bw.ravel(), mbw.ravel(), rel=1e-13, what="B part = dL/dB with U := V_U")


def _cotangents(n, m, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, n)), rng.normal(size=(n, m)), rng.normal(size=n)


@pytest.mark.parametrize("scheme,bnd", CASES)
@pytest.mark.parametrize("N,n,m", [(3, 3, 2), (3, 1, 1), (2, 2, 0), (2, 4, 1)])
def test_coef_adjoint_ex_high_precision(orc, N, n, m, scheme, bnd):
    """L is affine in theta, so t . dL/dtheta = L(theta + t) - L(theta)
    exactly.  From 50-digit evaluations of the definition module, its
    derivative in y_r is c_r(theta + t) - c_r(theta) and its derivative in
    z_a is a central difference at step 1e-20 (exact far below double
    rounding)."""
    import mpmath
    mpmath.mp.dps = 50
    inst = _inst(N, n, m, 280 + 5 * N + n, scheme, bnd)
    tA, tB, tg = _cotangents(n, m, 41 + N + n)
    (gz, gy), (mz, my) = orc.coef_adjoint_ex(inst, tA, tB, tg, scheme, bnd)
    mp = mpmath.mpf
    A, B, g, q, r = defn.as_lists(inst)
    cv = lambda x: [mp(float(t)) for t in x]
    A0, B0, g0 = [cv(a) for a in A], [cv(b) for b in B], cv(g)
    A1 = [[a + mp(float(t)) for a, t in zip(ra, rt)] for ra, rt in zip(A0, tA)]
    B1 = [[b + mp(float(t)) for b, t in zip(rb, rt)] for rb, rt in zip(B0, tB)]
    g1 = [a + mp(float(t)) for a, t in zip(g0, tg)]
    z0, yy, qq, rr = cv(inst.z), cv(inst.y), cv(q), cv(r)
    dt = mp(1) / N

    def tdot(z):
        L = lambda A_, B_, g_: defn.lagrangian_ex(z, yy, mp(float(inst.sigma)), N, n, m, A_, B_, g_, qq, rr,
                                                  scheme, bnd, sin=mpmath.sin, dt=dt)
        return L(A1, B1, g1) - L(A0, B0, g0)

    eps = mp("1e-20")
    want_z = []
    for a in range(len(z0)):
        zp, zm = z0[:], z0[:]
        zp[a] += eps
        zm[a] -= eps
        want_z.append(float((tdot(zp) - tdot(zm)) / (2 * eps)))
    c = lambda A_, B_, g_: defn.constraints_ex(z0, N, n, m, A_, B_, g_, scheme, bnd, sin=mpmath.sin, dt=dt)
    want_y = [float(a - b) for a, b in zip(c(A1, B1, g1), c(A0, B0, g0))]
    # the differences resolve 1e-50 / 1e-20: entries that are exactly zero
    # (Euler's last node carries no multiplier) come out near 1e-30, so the
    # bound gets an absolute floor of 1e-29 (1e-16 in units of mu)
    check_close(gz, np.array(want_z), mz + 1e-16, rel=1e-13, what=f"adjoint in z scheme={scheme} bnd={bnd}")
    check_close(gy, np.array(want_y), my, rel=1e-13, what=f"adjoint in y scheme={scheme} bnd={bnd}")


@pytest.mark.parametrize("scheme,bnd", CASES)
def test_coef_adjoint_ex_is_the_transpose_of_coef_grad_and_mixed(orc, scheme, bnd):
    """<gy, w> = t . dL/dtheta at multipliers w (dL/dtheta is linear in y),
    and <gz, v> = t . (the coefficient gradient's derivative along v): the
    adjoint is the transpose of the two node contractions, evaluated by the
    oracle's own coefficient gradient and mixed derivative."""
    inst = _inst(50, 5, 3, 290 + 3 * scheme + bnd, scheme, bnd)
    tA, tB, tg = _cotangents(5, 3, 43)
    (gz, gy), (mz, my) = orc.coef_adjoint_ex(inst, tA, tB, tg, scheme, bnd)
    rng = np.random.default_rng(44)
    w, v = rng.normal(size=len(inst.y)), rng.normal(size=len(inst.z))
    tdot = lambda parts: float(np.sum(tA * parts[0]) + np.sum(tB * parts[1]) + np.dot(tg, parts[2]))
    mdot = lambda parts: float(np.sum(np.abs(tA) * parts[0]) + np.sum(np.abs(tB) * parts[1])
                               + np.dot(np.abs(tg), parts[2]))
    cg, cgm = orc.coef_grad_ex(inst, scheme, bnd, y=w)
    assert abs(np.dot(gy, w) - tdot(cg)) <= 1e-12 * (np.dot(my, np.abs(w)) + mdot(cgm))
    cm, cmm = orc.coef_mixed_ex(inst, v, scheme, bnd)
    assert abs(np.dot(gz, v) - tdot(cm)) <= 1e-12 * (np.dot(mz, np.abs(v)) + mdot(cmm))


@pytest.mark.parametrize("N,n,m", [(40, 3, 2), (1, 1, 0), (17, 5, 1)])
def test_coef_adjoint_ex_affine_identity_through_c_oracle(orc, N, n, m):
    """With sigma = 0, grad_z L = J^T y, and J depends affinely on theta: the
    adjoint in z is J(t)^T y - J(0)^T y and the adjoint in y is
    c(t) - c(0), both from the C oracle's trapezoidal functions with the
    coefficients replaced by the cotangents and by zeros."""
    inst = _inst(N, n, m, 300 + N, 0, 0)
    tA, tB, tg = _cotangents(n, m, 45 + N)
    (gz, gy), (mz, my) = orc.coef_adjoint_ex(inst, tA, tB, tg, 0, 0)
    with_t = types.SimpleNamespace(**{k: getattr(inst, k) for k in ("N", "n", "m", "z", "y", "q", "r")})
    with_0 = types.SimpleNamespace(**vars(with_t))
    with_t.A, with_t.B, with_t.gamma = tA, tB, tg
    with_0.A, with_0.B, with_0.gamma = np.zeros_like(tA), np.zeros_like(tB), np.zeros_like(tg)
    (g1, m1), (g0, m0) = orc.lag_grad(with_t, sigma=0.0), orc.lag_grad(with_0, sigma=0.0)
    check_close(gz, g1 - g0, mz + 4 * np.finfo(float).eps * (m1 + m0), rel=1e-12, what="J(t)^T y - J(0)^T y")
    (c1, n1), (c0, n0) = orc.cons(with_t), orc.cons(with_0)
    check_close(gy, c1 - c0, my + 4 * np.finfo(float).eps * (n1 + n0), rel=1e-12, what="c(t) - c(0)")


@pytest.mark.parametrize("N,n,m", [(300, 4, 2), (1, 1, 0), (64, 6, 3)])
def test_trapezoidal_composites_equal_c_oracle(orc, N, n, m):
    """Without boundary rows the trapezoidal composites and the C oracle's
    node-by-node derivative functions (a different evaluation of the same
    definitions) agree within 1e-13 mu."""
    inst = _inst(N, n, m, 250 + N, 0, 0)
    v = np.random.default_rng(6).normal(size=len(inst.z))
    g1, m1 = orc.lag_grad_ex(inst, 0, 0, sigma=0.9)
    g2, _ = orc.lag_grad(inst, sigma=0.9)
    check_close(g1, g2, m1, rel=1e-13, what="grad_z L")
    h1, hm = orc.hvp_ex(inst, v, 0, 0, sigma=0.9)
    h2, _ = orc.hvp(inst, v, sigma=0.9)
    check_close(h1, h2, hm, rel=1e-13, what="H v")
    j1, jm = orc.jvp_ex(inst, v, 0, 0)
    j2, _ = orc.jvp(inst, v)
    check_close(j1, j2, jm, rel=1e-13, what="J v")
    L1, Lm = orc.lagrangian_ex(inst, 0, 0, sigma=0.9)
    L2, _ = orc.lagrangian(inst, sigma=0.9)
    assert abs(L1 - L2) <= 1e-13 * Lm
    (a1, b1, c1), (ma, mb, mc) = orc.coef_grad_ex(inst, 0, 0)
    (a2, b2, c2), _ = orc.coef_grad(inst)
    check_close(a1.ravel(), a2.ravel(), ma.ravel(), rel=1e-13, what="dL/dA")
    check_close(b1.ravel(), b2.ravel(), mb.ravel(), rel=1e-13, what="dL/dB")
    check_close(c1, c2, mc, rel=1e-13, what="dL/dgamma")


def test_boundary_rows_enter_linearly(orc):
    """A boundary row's multiplier adds exactly y_b to grad_z L at its state
    and nothing elsewhere; it leaves H v and dL/dtheta unchanged."""
    for scheme in (0, 1):
        inst = _inst(30, 3, 2, 260 + scheme, scheme, 2)
        N, n = inst.N, inst.n
        y0 = inst.y.copy()
        y0[n * N:] = 0.0
        g0, _ = orc.lag_grad_ex(inst, scheme, 2, y=y0)
        g1, _ = orc.lag_grad_ex(inst, scheme, 2)
        d = g1 - g0
        want = np.zeros_like(d)
        for i in range(n):
            want[i * (N + 1)] += inst.y[n * N + i]
            want[i * (N + 1) + N] += inst.y[n * N + n + i]
        check_close(d, want, np.abs(g1) + np.abs(g0) + 1e-300, rel=1e-15, what="boundary rows")
        v = np.random.default_rng(7).normal(size=len(inst.z))
        assert np.array_equal(orc.hvp_ex(inst, v, scheme, 2, y=y0)[0], orc.hvp_ex(inst, v, scheme, 2)[0])
        ca, _ = orc.coef_grad_ex(inst, scheme, 2, y=y0)
        cb, _ = orc.coef_grad_ex(inst, scheme, 2)
        for x, w in zip(ca, cb):
            assert np.array_equal(x, w)


# ---- the quadrotor model (paper Appendix A) ---------------------------------

QCFN = types.SimpleNamespace(sin=cmath.sin, cos=cmath.cos, tan=cmath.tan, pi=math.pi)


def _qL(q, z, y, sigma, fn=QCFN):
    return defn.quad_lagrangian(z, y, sigma, q.N, q.g, q.r, q.bnd, fn=fn)


@pytest.mark.parametrize("N,bnd", [(1, 0), (2, 1), (3, 2), (4, 1)])
def test_quad_lagrangian_high_precision(orc, N, bnd):
    import mpmath
    mpmath.mp.dps = 50
    q = synth.make_quadrotor(N, seed=300 + N, bnd=bnd)
    Lo, mu = orc.quad_lagrangian(q, sigma=0.9)
    mp = mpmath.mpf
    fn = types.SimpleNamespace(sin=mpmath.sin, cos=mpmath.cos, tan=mpmath.tan, pi=mpmath.pi)
    want = defn.quad_lagrangian([mp(v) for v in q.z], [mp(v) for v in q.y], mp("0.9"), N, mp(q.g),
                                mp(q.r), bnd, fn=fn, dt=mp(1) / N)
    assert abs(Lo - float(want)) <= 1e-13 * mu


@pytest.mark.parametrize("N,bnd", [(1, 0), (2, 1), (3, 2), (5, 1)])
def test_quad_lag_grad_complex_step(orc, N, bnd):
    q = synth.make_quadrotor(N, seed=310 + N, bnd=bnd)
    g, mu = orc.quad_lag_grad(q, sigma=0.8)
    tau = 1e-30
    y = list(map(float, q.y))
    cs = []
    for col in range(len(q.z)):
        z = [complex(v) for v in q.z]
        z[col] += 1j * tau
        cs.append(_qL(q, z, y, 0.8).imag / tau)
    check_close(g, np.array(cs), mu, rel=1e-13, what="quadrotor grad_z L")


@pytest.mark.parametrize("N,bnd", [(1, 0), (2, 1), (3, 2), (5, 1)])
def test_quad_jvp_complex_step(orc, N, bnd):
    q = synth.make_quadrotor(N, seed=320 + N, bnd=bnd)
    v = np.random.default_rng(8).normal(size=len(q.z))
    jv, mu = orc.quad_jvp(q, v)
    tau = 1e-30
    z = [complex(a, tau * b) for a, b in zip(q.z, v)]
    c = defn.quad_constraints(z, N, q.g, bnd, fn=QCFN)
    check_close(jv, np.array([x.imag / tau for x in c]), mu, rel=1e-13, what="quadrotor J v")


@pytest.mark.parametrize("N,bnd", [(1, 0), (2, 1), (3, 2)])
def test_quad_hvp_mixed_difference(orc, N, bnd):
    q = synth.make_quadrotor(N, seed=330 + N, bnd=bnd)
    v = np.random.default_rng(9).normal(size=len(q.z))
    hv, mu = orc.quad_hvp(q, v, sigma=1.1)
    tau, delta = 1e-30, 1e-5
    y = list(map(float, q.y))
    want = np.empty(len(q.z))
    for a in range(len(q.z)):
        vals = []
        for s in (+1, -1):
            z = [complex(x + s * delta * d) for x, d in zip(q.z, v)]
            z[a] += 1j * tau
            vals.append(_qL(q, z, y, 1.1).imag)
        want[a] = (vals[0] - vals[1]) / (2 * tau * delta)
    scale = max(float(np.max(mu)), 1.0)
    assert np.max(np.abs(hv - want)) <= 1e-7 * scale
