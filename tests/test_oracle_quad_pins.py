"""Pins of the oracle's quadrotor model (paper Appendix A, trapezoidal
transcription of Sec. 5).

The paper prints the model but no evaluated number, so the pins are
mathematical:
- the thrust terms of the dynamics are thrust times the third column of the
  yaw-pitch-roll rotation matrix, built here as a product of elementary
  rotations; the angle-rate terms rotate (u2, u3) by the roll angle, and the
  yaw rate exceeds u4 by the roll rate times sin(pitch);
- hover (level attitude, thrust g, no rates, no velocity) has zero defects,
  exactly;
- the defects along an accurate ODE solution shrink 8x per halving of h;
- the cost of the zero point is the trapezoidal rule applied to the squared
  references, which has a closed form, and exact tracking leaves only the
  control term; the value matches an mpmath evaluation at 50 digits;
- complex-step Jacobian and gradient, a mixed complex-step / central
  difference Hessian, and sympy's exact derivatives, each dense and zero
  outside the patterns;
- scipy's coo -> csr of tril(K) for the KKT structure.
"""
from __future__ import annotations

import cmath
import math
import types

import numpy as np
import pytest

import synth
from oracle import defn
from tests.helpers import EPS, dense_from_coo, sym_from_lower

G, R = synth.QUAD_G, synth.QUAD_R
CFN = types.SimpleNamespace(sin=cmath.sin, cos=cmath.cos, tan=cmath.tan, pi=math.pi)


def quad(N, seed=0, bnd=1, **over):
    q = synth.make_quadrotor(N, seed=seed, bnd=bnd)
    for k, v in over.items():
        setattr(q, k, v)
    return q


def _rot(axis, a):
    c, s = math.cos(a), math.sin(a)
    if axis == "x":
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if axis == "y":
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def rhs_from_rotations(x, u, g):
    """The quadrotor right-hand side assembled from rotation matrices, not from
    the model's printed trig products: translational acceleration is thrust
    along the body z axis (third column of Rz(x9) Ry(x8) Rx(x7)) minus
    gravity; the angle rates follow from the rotated body rates."""
    Rm = _rot("z", x[8]) @ _rot("y", x[7]) @ _rot("x", x[6])
    acc = u[0] * Rm[:, 2] - np.array([0.0, 0.0, g])
    w = _rot("z", -x[6])[:2, :2] @ np.array([u[1], u[2]])  # rotate (u2, u3) by -x7
    roll_rate = w[0] / math.cos(x[7])
    pitch_rate = w[1]
    yaw_rate = roll_rate * math.sin(x[7]) + u[3]
    return np.array([x[1], acc[0], x[3], acc[1], x[5], acc[2], roll_rate, pitch_rate, yaw_rate])


def test_rhs_matches_rotation_construction():
    rng = np.random.default_rng(1)
    for _ in range(50):
        x = rng.normal(size=9)
        x[6:] = rng.uniform(-1.2, 1.2, 3)
        u = rng.normal(size=4) * 3
        got = np.array(defn.quad_rhs(list(x), list(u), G))
        want = rhs_from_rotations(x, u, G)
        assert np.allclose(got, want, rtol=1e-13, atol=1e-13 * (1 + np.abs(u).max()))


def test_sizes_and_pattern(orc):
    for N, bnd in [(1, 0), (3, 1), (7, 2), (50, 1)]:
        s = orc.quad_sizes(N, bnd)
        assert s["nvar"] == 13 * (N + 1)
        assert s["ncon"] == 9 * N + 9 * bnd
        assert s["nnzj"] == 68 * N + 9 * bnd
        assert s["nnzh"] == 23 * (N + 1)
        jr, jc, hr, hc = orc.quad_pattern(N, bnd)
        assert len(set(zip(jr.tolist(), jc.tolist()))) == len(jr)
        assert len(set(zip(hr.tolist(), hc.tolist()))) == len(hr)
        assert np.all(hr >= hc)
        assert set(hr[hr == hc].tolist()) == set(range(s["nvar"]))
        # within a row, COO order (slot order) is ascending column order
        order = np.argsort(jr, kind="stable")
        same = jr[order][1:] == jr[order][:-1]
        assert np.all(jc[order][1:][same] > jc[order][:-1][same])


def test_hover_has_zero_defects_exactly(orc):
    N = 12
    q = quad(N, seed=2, bnd=2)
    X = np.zeros((9, N + 1))
    X[0], X[2], X[4] = 0.3, -1.7, 2.5   # any fixed position
    U = np.zeros((4, N + 1))
    U[0] = G
    q.z = np.concatenate([X.ravel(), U.ravel()])
    c, mu = orc.quad_cons(q)
    assert np.all(c[: 9 * N] == 0.0)
    assert np.array_equal(c[9 * N:], np.concatenate([X[:, 0], X[:, N]]))


def test_defects_of_exact_trajectory_are_third_order(orc):
    from scipy.integrate import solve_ivp
    rng = np.random.default_rng(3)
    a = rng.normal(size=4) * 0.3
    b = rng.normal(size=4) * 0.3

    def u_of(t):
        return np.array([G + a[0] + b[0] * t, a[1] + b[1] * np.sin(t), a[2] + b[2] * t, a[3] + b[3] * t * t])

    def f(t, x):
        return rhs_from_rotations(x, u_of(t), G)

    x0 = rng.normal(size=9) * 0.3
    sol = solve_ivp(f, (0.0, 1.0), x0, method="DOP853", rtol=1e-13, atol=1e-14, dense_output=True)
    maxc = []
    for N in (40, 80, 160):
        t = np.arange(N + 1) / N
        X = sol.sol(t)
        U = np.stack([u_of(tk) for tk in t], axis=1)
        q = quad(N, bnd=0, z=np.concatenate([X.ravel(), U.ravel()]))
        c, _ = orc.quad_cons(q)
        maxc.append(np.abs(c).max())
    for k in range(2):
        assert 7.0 < maxc[k] / maxc[k + 1] < 9.0, maxc


@pytest.mark.parametrize("N", [5, 7, 64, 1000])
def test_objective_closed_form_at_zero(orc, N):
    """X = 0, U = 0: f = 1/2 T_N[sin^2(2 pi t) + 4 sin^2(4 pi t) + 4 t^2]; the
    trapezoidal rule integrates the periodic terms exactly for N not dividing
    4, and 4 t^2 to 4/3 + 2 h^2 / 3, so f = 23/12 + h^2 / 3."""
    q = quad(N, z=np.zeros(13 * (N + 1)))
    f, mu = orc.quad_obj(q)
    h = 1.0 / N
    assert abs(f - (23.0 / 12.0 + h * h / 3.0)) <= 64 * EPS * mu


def test_objective_exact_tracking(orc):
    """States on the references, level attitude, constant controls: only the
    control term remains, 1/2 r |u|^2 times the sum of the weights (1)."""
    N = 333
    t = np.arange(N + 1) * (1.0 / N)
    X = np.zeros((9, N + 1))
    X[0] = [math.sin(2 * math.pi * tk) for tk in t]
    X[2] = [2 * math.sin(4 * math.pi * tk) for tk in t]
    X[4] = [2 * tk for tk in t]
    X[1], X[3], X[5] = 5.0, -2.0, 1.0   # velocities carry no cost
    U = np.tile(np.array([[9.0], [0.5], [-0.25], [2.0]]), (1, N + 1))
    q = quad(N, z=np.concatenate([X.ravel(), U.ravel()]))
    f, mu = orc.quad_obj(q)
    want = 0.5 * R * (81.0 + 0.25 + 0.0625 + 4.0)
    assert abs(f - want) <= 64 * EPS * mu
    g, _ = orc.quad_grad(q)
    Gm = g.reshape(13, N + 1)
    assert np.all(Gm[:9] == 0.0)


def test_objective_high_precision(orc):
    import mpmath
    mpmath.mp.dps = 50
    N = 40
    q = quad(N, seed=4)
    f, mu = orc.quad_obj(q)
    z = [mpmath.mpf(float(v)) for v in q.z]
    fm = defn.quad_objective(z, N, mpmath.mpf(R), fn=mpmath, dt=mpmath.mpf(1) / N)
    assert abs(f - float(fm)) <= 8 * EPS * mu


def test_constraints_match_definition(orc):
    N = 30
    q = quad(N, seed=5, bnd=2)
    c, mu = orc.quad_cons(q)
    want = defn.quad_constraints(list(q.z), N, G, 2)
    assert np.all(np.abs(c - np.array(want)) <= 8 * EPS * mu)


def _cs_jac(q, tau=1e-30):
    cols = []
    for col in range(len(q.z)):
        z = [complex(v) for v in q.z]
        z[col] += 1j * tau
        c = defn.quad_constraints(z, q.N, G, q.bnd, fn=CFN)
        cols.append([v.imag / tau for v in c])
    return np.array(cols).T


@pytest.mark.parametrize("N,bnd", [(1, 1), (3, 2), (4, 0)])
def test_jacobian_complex_step_and_pattern(orc, N, bnd):
    q = quad(N, seed=10 + N, bnd=bnd)
    s = orc.quad_sizes(N, bnd)
    J = _cs_jac(q)
    jr, jc, _, _ = orc.quad_pattern(N, bnd)
    jv, _ = orc.quad_jac(q)
    Jo = dense_from_coo(jr, jc, jv, (s["ncon"], s["nvar"]))
    assert np.abs(Jo - J).max() <= 1e-13 * max(1.0, np.abs(J).max())
    # the pattern is exactly the nonzero set at a random point
    nz = set(zip(*np.nonzero(J)))
    assert nz == set(zip(jr.tolist(), jc.tolist()))


def test_gradient_complex_step(orc):
    N = 6
    q = quad(N, seed=20)
    g, _ = orc.quad_grad(q)
    tau = 1e-30
    for col in range(len(q.z)):
        z = [complex(v) for v in q.z]
        z[col] += 1j * tau
        d = defn.quad_objective(z, N, R, fn=CFN).imag / tau
        assert abs(d - g[col]) <= 1e-14 * max(1.0, abs(d)), col


@pytest.mark.parametrize("N,bnd,sigma", [(1, 1, 1.3), (2, 2, 0.7)])
def test_hessian_mixed_difference(orc, N, bnd, sigma):
    q = quad(N, seed=30 + N, bnd=bnd)
    s = orc.quad_sizes(N, bnd)
    nv = s["nvar"]
    y = list(map(float, q.y))
    tau, delta = 1e-30, 1e-5
    H = np.zeros((nv, nv))
    for a in range(nv):
        for b in range(a + 1):
            vals = []
            for sg in (1, -1):
                z = [complex(v) for v in q.z]
                z[a] += 1j * tau
                z[b] += sg * delta
                vals.append(defn.quad_lagrangian(z, y, sigma, N, G, R, bnd, fn=CFN).imag)
            H[a, b] = H[b, a] = (vals[0] - vals[1]) / (2 * tau * delta)
    _, _, hr, hc = orc.quad_pattern(N, bnd)
    hv, _ = orc.quad_hess(q, sigma=sigma)
    Hs = sym_from_lower(hr, hc, hv, nv)
    scale = max(np.abs(H).max(), 1e-300)
    assert np.abs(Hs - H).max() <= 1e-8 * scale
    P = np.zeros_like(H, dtype=bool)
    P[hr, hc] = P[hc, hr] = True
    assert np.abs(H[~P]).max(initial=0.0) <= 1e-9 * scale


@pytest.mark.slow
def test_symbolic_derivatives(orc):
    """sympy differentiates the definition exactly; evaluated at the oracle's
    point every Jacobian and Hessian entry agrees to rounding, and every
    structural zero outside the patterns is identically zero."""
    import sympy as S
    N, bnd = 1, 1
    q = quad(N, seed=40, bnd=bnd)
    s = orc.quad_sizes(N, bnd)
    zs = S.symbols(f"z0:{s['nvar']}")
    ys = S.symbols(f"y0:{s['ncon']}")
    sig = S.Symbol("sigma")
    fn = types.SimpleNamespace(sin=S.sin, cos=S.cos, tan=S.tan, pi=S.pi)
    c = defn.quad_constraints(list(zs), N, S.Rational(G), bnd, fn=fn, dt=S.Rational(1, N))
    L = defn.quad_lagrangian(list(zs), list(ys), sig, N, S.Rational(G), S.Rational(R), bnd, fn=fn,
                             dt=S.Rational(1, N))
    sub = {zs[i]: S.Float(float(q.z[i]), 30) for i in range(len(zs))}
    sub.update({ys[i]: S.Float(float(q.y[i]), 30) for i in range(len(ys))})
    sub[sig] = S.Float(1.0, 30)
    jr, jc, hr, hc = orc.quad_pattern(N, bnd)
    jv, _ = orc.quad_jac(q)
    jpat = set(zip(jr.tolist(), jc.tolist()))
    for r_, ci in enumerate(c):
        for col in range(len(zs)):
            d = S.diff(ci, zs[col])
            if (r_, col) not in jpat:
                assert S.simplify(d) == 0, (r_, col)
    for e in range(len(jv)):
        d = S.diff(c[jr[e]], zs[jc[e]])
        assert abs(float(d.evalf(30, subs=sub)) - jv[e]) <= 1e-13 * max(1.0, abs(jv[e]))
    hv, _ = orc.quad_hess(q, sigma=1.0)
    hpat = set(zip(hr.tolist(), hc.tolist()))
    grad = [S.diff(L, v) for v in zs]
    for a in range(len(zs)):
        for b in range(a + 1):
            d = S.diff(grad[a], zs[b])
            if (a, b) not in hpat:
                assert S.simplify(d) == 0, (a, b)
    for e in range(len(hv)):
        d = S.diff(grad[hr[e]], zs[hc[e]])
        assert abs(float(d.evalf(30, subs=sub)) - hv[e]) <= 1e-13 * max(1.0, abs(hv[e]))


@pytest.mark.parametrize("N,bnd", [(3, 1), (20, 0), (9, 2)])
def test_kkt_matches_scipy(orc, N, bnd):
    import scipy.sparse as sp
    s = orc.quad_sizes(N, bnd)
    jr, jc, hr, hc = orc.quad_pattern(N, bnd)
    rowptr, colind, pj, ph = orc.quad_kkt(N, bnd)
    nv, dim = s["nvar"], s["dim"]
    rows = np.concatenate([hr, nv + jr, np.arange(dim)])
    cols = np.concatenate([hc, jc, np.arange(dim)])
    M = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(dim, dim)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    assert np.array_equal(M.indptr, rowptr) and np.array_equal(M.indices, colind)
    assert len(colind) == s["nnzh"] + s["nnzj"] + s["ncon"]
    slot_row = np.repeat(np.arange(dim), np.diff(rowptr))
    assert np.array_equal(colind[pj], jc) and np.array_equal(slot_row[pj], nv + jr)
    assert np.array_equal(colind[ph], hc) and np.array_equal(slot_row[ph], hr)
