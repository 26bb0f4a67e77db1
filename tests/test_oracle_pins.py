"""Pins of the CPU oracle against facts fixed outside it.

Nothing here compares the oracle with a re-typed copy of its own formulas:
each test checks it against the paper's printed generated code (golden
fixture), a closed form, an exact-arithmetic evaluation, a textbook or
library routine (complex-step and finite differences of the independent
definition module, an ODE integrator, scipy's sparse conversion, sympy's
symbolic differentiation) or a structural invariant.
"""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import defn
from tests.helpers import (EPS, REL, check_close, cs_gradient, cs_jacobian, dense_from_coo,
                           instance, mixed_hessian, sym_from_lower)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

SMALL = [(1, 1, 0), (1, 1, 1), (2, 2, 1), (3, 3, 1), (4, 4, 2), (5, 2, 0), (3, 1, 2), (6, 5, 3),
         (7, 3, 0), (8, 4, 2)]


def closed_sizes(N, n, m):
    npair = n if n >= 3 else (1 if n == 2 else 0)
    return dict(nvar=(n + m) * (N + 1), ncon=n * N, nnzj=2 * n * N * (n + m),
                nnzh=(N + 1) * (n + npair + m), npair=npair)


# ---- P1: the paper's generated trapezoidal code (golden worked example) ----

def test_golden_generated_code(orc):
    g = json.load(open(os.path.join(GOLDEN, "trapezoid_generated_code.json")))
    N = g["N"]
    assert g["dt"] == 1.0 / N
    inst = instance(N, 1, 1, A=np.zeros((1, 1)), B=np.ones((1, 1)), gamma=np.zeros(1),
                    q=np.array(g["q"]), r=np.array(g["r"]),
                    z=np.array(g["x"] + g["u"], dtype=np.float64), y=np.ones(N))
    c, _ = orc.cons(inst)
    assert c.tolist() == g["defects"]
    f, _ = orc.obj(inst)
    assert f == g["objective"]
    jv, _ = orc.jac(inst)
    row = g["jacobian_row"]
    # slots of row (0, k): x_k, x_{k+1}, u_k, u_{k+1}; position (0*T + t)*N + k
    for k in range(N):
        assert jv[0 * N + k] == row["d_x_j"]
        assert jv[1 * N + k] == row["d_x_j1"]
        assert jv[2 * N + k] == row["d_u_j"]
        assert jv[3 * N + k] == row["d_u_j1"]
    hv, _ = orc.hess(inst, sigma=1.0)
    # n = 1, m = 1: slots x diagonal (s = 0), u diagonal (s = 1); A = gamma = 0
    assert hv[N + 1:].tolist() == g["hessian_u_diag"]
    assert np.all(hv[: N + 1] == 0.0)


# ---- P8: sizes, patterns ----------------------------------------------------

@pytest.mark.parametrize("N,n,m", SMALL + [(1000, 4, 2), (37, 16, 8)])
def test_sizes_closed_form(orc, N, n, m):
    s = orc.sizes(N, n, m)
    for k, v in closed_sizes(N, n, m).items():
        assert s[k] == v, k
    assert s["dim"] == s["nvar"] + s["ncon"]


@pytest.mark.parametrize("N,n,m", SMALL + [(1000, 4, 2)])
def test_pattern_unique_lower(orc, N, n, m):
    s = orc.sizes(N, n, m)
    jrow, jcol, hrow, hcol = orc.pattern(N, n, m)
    assert jrow.min() >= 0 and jrow.max() < s["ncon"]
    assert jcol.min() >= 0 and jcol.max() < s["nvar"]
    assert len(set(zip(jrow.tolist(), jcol.tolist()))) == s["nnzj"]
    assert len(set(zip(hrow.tolist(), hcol.tolist()))) == s["nnzh"]
    assert np.all(hrow >= hcol)
    diag = set(hrow[hrow == hcol].tolist())
    assert diag == set(range(s["nvar"]))           # every variable diagonal present
    # within a row, the slots are in ascending column order
    T = 2 * n + 2 * m
    cols = jcol.reshape(n, T, N)
    assert np.all(np.diff(cols, axis=1) > 0)


@pytest.mark.parametrize("N,n,m", [(3, 1, 1), (4, 2, 1), (3, 3, 1), (2, 4, 2), (3, 3, 0)])
def test_jacobian_pattern_is_nonzero_set(orc, N, n, m):
    """With random coefficients the structural pattern equals the set of
    nonzero complex-step derivatives (and nothing outside it is nonzero)."""
    inst = instance(N, n, m, seed=3)
    s = orc.sizes(N, n, m)
    Jcs = cs_jacobian(inst, range(s["nvar"]))
    jrow, jcol, _, _ = orc.pattern(N, n, m)
    P = np.zeros_like(Jcs, dtype=bool)
    P[jrow, jcol] = True
    assert np.array_equal(Jcs != 0, P)


# ---- P9: KKT indices against scipy; symmetric SpMV ------------------------

@pytest.mark.parametrize("N,n,m", SMALL + [(1000, 4, 2), (100, 16, 8)])
def test_kkt_matches_scipy(orc, N, n, m):
    import scipy.sparse as sp
    s = orc.sizes(N, n, m)
    jrow, jcol, hrow, hcol = orc.pattern(N, n, m)
    rowptr, colind, perm_j, perm_h = orc.kkt(N, n, m)
    nv, dim = s["nvar"], s["dim"]
    rows = np.concatenate([hrow, nv + jrow, np.arange(dim)])
    cols = np.concatenate([hcol, jcol, np.arange(dim)])
    M = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(dim, dim)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    assert np.array_equal(M.indptr, rowptr)
    assert np.array_equal(M.indices, colind)
    assert len(colind) == s["nnzh"] + s["nnzj"] + s["ncon"]
    # perm sends each COO entry to the slot holding its (row, col)
    slot_row = np.repeat(np.arange(dim), np.diff(rowptr))
    assert np.array_equal(colind[perm_h], hcol) and np.array_equal(slot_row[perm_h], hrow)
    assert np.array_equal(colind[perm_j], jcol) and np.array_equal(slot_row[perm_j], nv + jrow)
    # injective, and the diagonal is the last entry of every row
    used = np.concatenate([perm_h, perm_j])
    assert len(np.unique(used)) == len(used)
    assert np.array_equal(colind[rowptr[1:] - 1], np.arange(dim))


@pytest.mark.parametrize("N,n,m", [(3, 3, 1), (4, 2, 1), (2, 4, 2), (3, 1, 0)])
def test_kkt_spmv_equals_dense(orc, N, n, m):
    """Symmetric SpMV with the assembled lower CSR equals the dense K v built
    from complex-step J and the mixed complex-step Hessian."""
    inst = instance(N, n, m, seed=5)
    s = orc.sizes(N, n, m)
    nv, dim = s["nvar"], s["dim"]
    rowptr, colind, perm_j, perm_h = orc.kkt(N, n, m)
    jv, _ = orc.jac(inst)
    hv, _ = orc.hess(inst)
    reg = np.random.default_rng(9).normal(size=dim)
    kv = orc.assemble(rowptr, perm_j, jv, perm_h, hv, reg)
    v = np.random.default_rng(10).normal(size=dim)
    out = np.zeros(dim)
    for d in range(dim):
        for x in range(rowptr[d], rowptr[d + 1]):
            c = colind[x]
            out[d] += kv[x] * v[c]
            if c != d:
                out[c] += kv[x] * v[d]
    J = cs_jacobian(inst, range(nv))
    H = mixed_hessian(inst, inst.y, inst.sigma)
    K = np.zeros((dim, dim))
    K[:nv, :nv] = H
    K[nv:, :nv] = J
    K[:nv, nv:] = J.T
    K += np.diag(reg)
    ref = K @ v
    scale = np.abs(K) @ np.abs(v)
    assert np.all(np.abs(out - ref) <= 1e-7 * scale + 1e-12)


# ---- P2, P12: objective -----------------------------------------------------

@pytest.mark.parametrize("N", [1, 2, 7, 64, 1000, 4096, 100_000])
def test_objective_constant_state(orc, N):
    """X = c, U = 0 gives f = n c^2 sum(w) = n c^2 (sum of weights = N h = 1)."""
    n, m, c = 3, 2, 0.75
    inst = instance(N, n, m)
    inst.z = np.concatenate([np.full(n * (N + 1), c), np.zeros(m * (N + 1))])
    f, mu = orc.obj(inst)
    assert abs(f - n * c * c) <= 4 * EPS * mu
    if N & (N - 1) == 0:           # h exact: the weights sum to 1 exactly
        assert f == n * c * c


@pytest.mark.parametrize("N", [1, 3, 10, 1000])
def test_objective_trapezoid_exactness(orc, N):
    """Trapezoid rule on u(t) = t: r sum_k w_k t_k^2 = r (1/3 + h^2/6) exactly in
    reals; checked against the exact rational value of the same quadrature."""
    inst = instance(N, 1, 1, q=np.zeros(1), r=np.ones(1))
    t = np.arange(N + 1) / N
    inst.z = np.concatenate([np.zeros(N + 1), t])
    f, mu = orc.obj(inst)
    h = Fraction(1, N)
    exact = Fraction(1, 3) + h * h / 6
    # the nodes t_k = k/N are rounded to double, so compare within a few ulp
    assert abs(f - float(exact)) <= 8 * EPS * mu


@pytest.mark.parametrize("N,n,m", [(1000, 4, 2), (5000, 3, 1), (1, 2, 2)])
def test_objective_vs_exact_rational(orc, N, n, m):
    """f against the exact rational value of the definition module's sum with
    the same double inputs and double weights (P12: oracle within 2 ulp)."""
    inst = instance(N, n, m, seed=7)
    f, mu = orc.obj(inst)
    dt = Fraction(1.0 / N)
    zf = [Fraction(float(v)) for v in inst.z]
    exact = defn.objective(zf, N, n, m, [Fraction(float(v)) for v in inst.q],
                           [Fraction(float(v)) for v in inst.r], dt=dt)
    # weights in the oracle: h and 0.5 h, both exact multiples of dt as a double
    assert abs(f - float(exact)) <= 2 * math.ulp(float(exact)) + 2 * EPS * EPS * mu


def test_objective_thread_independent(orc):
    inst = instance(50_000, 4, 2, seed=11)
    t0 = orc.get_threads()
    try:
        orc.set_threads(1)
        a = orc.obj(inst)
        orc.set_threads(max(2, os.cpu_count() or 2))
        b = orc.obj(inst)
    finally:
        orc.set_threads(t0)
    assert a == b


# ---- P3: linear-quadratic case in closed form -------------------------------

@pytest.mark.parametrize("N,n,m", [(20, 3, 2), (9, 1, 1), (16, 2, 3), (33, 4, 0)])
def test_linear_quadratic_case(orc, N, n, m):
    """A = 0, gamma = 0: F = B U.  For x(t) = x0 + B (a t + b t^2 / 2), the
    exact solution under the affine control u(t) = a + b t, the trapezoidal
    defects vanish; the Jacobian is the constant template and the Hessian is
    sigma * 2 w_k diag(q, r) at any point and any multipliers."""
    rng = np.random.default_rng(N + 10 * n + 100 * m)
    inst = instance(N, n, m, seed=1, A=np.zeros((n, n)), gamma=np.zeros(n))
    x0 = rng.normal(size=n)
    a = rng.normal(size=m)
    b = rng.normal(size=m)
    t = np.arange(N + 1) / N
    U = a[:, None] + b[:, None] * t[None, :]
    X = x0[:, None] + inst.B @ (a[:, None] * t[None, :] + b[:, None] * t[None, :] ** 2 / 2)
    inst.z = np.concatenate([X.ravel(), U.ravel()])
    c, mu = orc.cons(inst)
    assert np.all(np.abs(c) <= 16 * EPS * mu)
    h = 1.0 / N
    hh = 0.5 * h
    T = 2 * n + 2 * m
    for trial in range(2):
        if trial:
            inst.z = np.random.default_rng(99).normal(size=inst.z.shape)
        jv, _ = orc.jac(inst)
        J = jv.reshape(n, T, N)
        for i in range(n):
            for j in range(n):
                d = 1.0 if i == j else 0.0
                assert np.all(J[i, 2 * j] == -d) and np.all(J[i, 2 * j + 1] == d)
            for l in range(m):
                assert np.all(J[i, 2 * n + 2 * l] == -hh * inst.B[i, l])
                assert np.all(J[i, 2 * n + 2 * l + 1] == -hh * inst.B[i, l])
        sigma = 1.7
        y = np.random.default_rng(trial).normal(size=n * N)
        hv, _ = orc.hess(inst, sigma=sigma, y=y)
        S = len(hv) // (N + 1)
        H = hv.reshape(S, N + 1)
        w = np.full(N + 1, h)
        w[0] = w[N] = hh
        npair = S - n - m
        for j in range(n):
            np.testing.assert_array_equal(H[j], 2.0 * sigma * w * inst.q[j])
        assert np.all(H[n:n + npair] == 0.0)
        for l in range(m):
            np.testing.assert_array_equal(H[n + npair + l], 2.0 * sigma * w * inst.r[l])


# ---- the nonlinear defects against an ODE integrator -------------------------

@pytest.mark.parametrize("n,m", [(4, 2), (3, 1), (2, 0), (1, 1)])
def test_defects_of_exact_trajectory_are_third_order(orc, n, m):
    """Along an accurate numerical solution of x' = f(x, u(t)) (scipy DOP853),
    the trapezoidal defects are the local truncation error -h^3 x'''/12: they
    shrink 8x when N doubles.  A wrong sign, index or dropped term in the
    dynamics leaves an O(h) defect instead, which shrinks only 2x."""
    from scipy.integrate import solve_ivp
    rng = np.random.default_rng(40 + n)
    base = instance(8, n, m, seed=40 + n)
    A, B, gam = base.A, base.B, base.gamma
    a = rng.normal(size=m) * 0.5
    b = rng.normal(size=m) * 0.5
    x0 = rng.normal(size=n) * 0.5

    def f(t, x):  # the workload family's right-hand side, from its definition
        u = a + b * t
        return A @ np.sin(x) + B @ u + gam * x * np.roll(x, -1)

    sol = solve_ivp(f, (0.0, 1.0), x0, method="DOP853", rtol=1e-13, atol=1e-14,
                    dense_output=True)
    maxc = []
    for N in (40, 80, 160):
        t = np.arange(N + 1) / N
        X = sol.sol(t)
        U = a[:, None] + b[:, None] * t[None, :]
        inst = instance(N, n, m, A=A, B=B, gamma=gam,
                        z=np.concatenate([X.ravel(), U.ravel()]))
        c, _ = orc.cons(inst)
        maxc.append(np.abs(c).max())
    for k in range(2):
        assert 6.5 < maxc[k] / maxc[k + 1] < 9.5, maxc
    assert maxc[-1] < 1e-5


# ---- P4, P6: Jacobian and gradient by complex step / finite differences ----

@pytest.mark.parametrize("N,n,m", [(1, 1, 0), (2, 1, 1), (3, 2, 1), (4, 3, 1), (5, 4, 2),
                                   (3, 5, 0), (8, 4, 2)])
def test_jacobian_dense_complex_step(orc, N, n, m):
    inst = instance(N, n, m, seed=N + n + m)
    s = orc.sizes(N, n, m)
    Jcs = cs_jacobian(inst, range(s["nvar"]))
    jrow, jcol, _, _ = orc.pattern(N, n, m)
    jv, mu = orc.jac(inst)
    check_close(jv, Jcs[jrow, jcol], mu, rel=1e-13, what="jac vs complex step")
    # nothing outside the pattern
    Jd = dense_from_coo(jrow, jcol, jv, Jcs.shape)
    mask = Jd == 0
    mask[jrow, jcol] = False
    assert np.all(Jcs[mask] == 0)


def test_jacobian_sampled_complex_step_parity_size(orc):
    N, n, m = 1000, 4, 2
    inst = instance(N, n, m)
    s = orc.sizes(N, n, m)
    rng = np.random.default_rng(2)
    cols = sorted(set(rng.integers(0, s["nvar"], 12).tolist()) | {0, N, N + 1, s["nvar"] - 1})
    Jcs = cs_jacobian(inst, cols)
    jrow, jcol, _, _ = orc.pattern(N, n, m)
    jv, mu = orc.jac(inst)
    for a, col in enumerate(cols):
        sel = jcol == col
        check_close(jv[sel], Jcs[jrow[sel], a], mu[sel], rel=1e-13, what=f"col {col}")
        other = np.ones(s["ncon"], bool)
        other[jrow[sel]] = False
        assert np.all(Jcs[other, a] == 0)


@pytest.mark.parametrize("N,n,m", [(5, 3, 2), (1000, 4, 2)])
def test_gradient_complex_step_and_central_difference(orc, N, n, m):
    inst = instance(N, n, m, seed=4)
    s = orc.sizes(N, n, m)
    g, mu = orc.grad(inst)
    cols = list(range(s["nvar"])) if s["nvar"] < 100 else [0, 1, N, N + 1, 3 * (N + 1) + 17,
                                                           s["nvar"] - 1, s["nvar"] - N - 1]
    gcs = cs_gradient(inst, cols)
    check_close(g[cols], gcs, mu[cols], rel=4 * EPS, what="grad vs complex step")
    # f is quadratic: the central difference is exact up to rounding
    A, B, gm, q, r = defn.as_lists(inst)
    step = 1e-6
    fd = []
    for col in cols:
        zp = inst.z.copy()
        zm = inst.z.copy()
        zp[col] += step
        zm[col] -= step
        fd.append((defn.objective(list(zp), N, n, m, q, r)
                   - defn.objective(list(zm), N, n, m, q, r)) / (zp[col] - zm[col]))
    fscale = abs(defn.objective(list(inst.z), N, n, m, q, r))
    assert np.all(np.abs(np.array(fd) - g[cols]) <= 1e-9 * fscale / step + 1e-12)


def test_jacobian_central_difference(orc):
    """Central differences (step 1e-6) of the definition's constraints; the
    control columns are exact (c is affine in U)."""
    N, n, m = 6, 4, 2
    inst = instance(N, n, m, seed=8)
    A, B, gm, q, r = defn.as_lists(inst)
    s = orc.sizes(N, n, m)
    jrow, jcol, _, _ = orc.pattern(N, n, m)
    jv, mu = orc.jac(inst)
    J = dense_from_coo(jrow, jcol, jv, (s["ncon"], s["nvar"]))
    step = 1e-6
    for col in range(s["nvar"]):
        zp = inst.z.copy()
        zm = inst.z.copy()
        zp[col] += step
        zm[col] -= step
        d = (np.array(defn.constraints(list(zp), N, n, m, A, B, gm))
             - np.array(defn.constraints(list(zm), N, n, m, A, B, gm))) / (zp[col] - zm[col])
        tol = 1e-8 if col < n * (N + 1) else 1e-9
        assert np.all(np.abs(d - J[:, col]) <= tol), col


# ---- P5, P7: Hessian ----------------------------------------------------------

@pytest.mark.parametrize("N,n,m", [(1, 1, 1), (3, 1, 0), (3, 2, 1), (2, 3, 1), (2, 4, 2),
                                   (4, 3, 0)])
def test_hessian_dense_mixed_difference(orc, N, n, m):
    inst = instance(N, n, m, seed=20 + N + n)
    s = orc.sizes(N, n, m)
    Hfd = mixed_hessian(inst, inst.y, 1.3)
    _, _, hrow, hcol = orc.pattern(N, n, m)
    hv, mu = orc.hess(inst, sigma=1.3)
    H = sym_from_lower(hrow, hcol, hv, s["nvar"])
    scale = np.abs(Hfd).max()
    assert np.abs(H - Hfd).max() <= 1e-8 * scale
    # P7: symmetric to FD noise, zero across nodes and outside the pattern
    assert np.abs(Hfd - Hfd.T).max() <= 1e-8 * scale
    P = np.zeros_like(H, dtype=bool)
    P[hrow, hcol] = P[hcol, hrow] = True
    assert np.abs(Hfd[~P]).max(initial=0.0) <= 1e-9 * scale
    node = np.arange(s["nvar"]) % (N + 1)
    cross = node[:, None] != node[None, :]
    assert not np.any(P & cross)


# ---- P13: symbolic differentiation -------------------------------------------

@pytest.mark.slow
@pytest.mark.parametrize("N,n,m", [(2, 3, 1), (3, 2, 1), (2, 1, 1), (2, 4, 2), (1, 3, 0)])
def test_symbolic_derivatives(orc, N, n, m):
    """sympy differentiates the definition module's exact Lagrangian; every
    Jacobian and Hessian slot must match and everything outside the patterns
    must be identically zero."""
    import sympy as S
    inst = instance(N, n, m, seed=30 + N * n + m)
    s = orc.sizes(N, n, m)
    R = lambda v: S.Rational(float(v))  # exact binary value of each double
    A = [[R(v) for v in row] for row in inst.A]
    B = [[R(v) for v in row] for row in inst.B] if m else [[] for _ in range(n)]
    gam = [R(v) for v in inst.gamma]
    q = [R(v) for v in inst.q]
    r = [R(v) for v in inst.r]
    zs = S.symbols(f"z0:{s['nvar']}")
    ys = S.symbols(f"y0:{s['ncon']}")
    sig = S.Symbol("sigma")
    dt = S.Rational(1, N)
    c = defn.constraints(list(zs), N, n, m, A, B, gam, sin=S.sin, dt=dt)
    L = defn.lagrangian(list(zs), list(ys), sig, N, n, m, A, B, gam, q, r, sin=S.sin, dt=dt)
    sub = {zs[i]: R(inst.z[i]) for i in range(s["nvar"])}
    sub.update({ys[i]: R(inst.y[i]) for i in range(s["ncon"])})
    sub[sig] = R(inst.sigma)
    jrow, jcol, hrow, hcol = orc.pattern(N, n, m)
    jv, jmu = orc.jac(inst)
    hv, hmu = orc.hess(inst)
    inJ = set(zip(jrow.tolist(), jcol.tolist()))
    for a in range(s["ncon"]):
        for b in range(s["nvar"]):
            d = S.diff(c[a], zs[b])
            if (a, b) not in inJ:
                assert S.simplify(d) == 0
    for e in range(s["nnzj"]):
        want = float(S.N(S.diff(c[jrow[e]], zs[jcol[e]]).subs(sub), 40))
        assert abs(jv[e] - want) <= 1e-14 * jmu[e] + 1e-300
    inH = set(zip(hrow.tolist(), hcol.tolist()))
    for a in range(s["nvar"]):
        for b in range(a + 1):
            d = S.diff(L, zs[a], zs[b])
            if (a, b) not in inH:
                assert S.simplify(d) == 0, (a, b)
    for e in range(s["nnzh"]):
        want = float(S.N(S.diff(L, zs[hrow[e]], zs[hcol[e]]).subs(sub), 40))
        assert abs(hv[e] - want) <= 1e-14 * hmu[e] + 1e-300


# ---- consistency of the definition module with exact arithmetic --------------

def test_cons_matches_definition_in_exact_arithmetic_linear_part(orc):
    """With A = 0 the defects involve no transcendental function, so the
    definition module evaluated in exact rationals gives the true value; the
    oracle must agree within a few ulp of mu."""
    N, n, m = 50, 3, 2
    inst = instance(N, n, m, seed=12, A=np.zeros((3, 3)))
    c, mu = orc.cons(inst)
    Fr = lambda v: Fraction(float(v))
    B = [[Fr(v) for v in row] for row in inst.B]
    exact = defn.constraints([Fr(v) for v in inst.z], N, n, m, [[0] * n] * n, B,
                             [Fr(v) for v in inst.gamma], sin=lambda x: 0,
                             dt=Fraction(1.0 / N))
    check_close(c, np.array([float(v) for v in exact]), mu, rel=8 * EPS, what="cons exact")


# ---- node ranges reproduce the full-size arrays ------------------------------

def test_node_ranges_match_full(orc):
    N, n, m = 777, 5, 3
    inst = instance(N, n, m, seed=13)
    T, S = 2 * n + 2 * m, orc.sizes(N, n, m)["S"]
    full = {"jac": orc.jac(inst)[0].reshape(n * T, N),
            "cons": orc.cons(inst)[0].reshape(n, N),
            "hess": orc.hess(inst)[0].reshape(S, N + 1),
            "grad": orc.grad(inst)[0].reshape(n + m, N + 1)}
    for k0, k1 in [(0, 1), (5, 300), (700, 777)]:
        assert np.array_equal(orc.jac(inst, k0, k1)[0].reshape(n * T, -1), full["jac"][:, k0:k1])
        assert np.array_equal(orc.cons(inst, k0, k1)[0].reshape(n, -1), full["cons"][:, k0:k1])
    for k0, k1 in [(0, 1), (5, 300), (700, 778)]:
        assert np.array_equal(orc.hess(inst, k0, k1)[0].reshape(S, -1), full["hess"][:, k0:k1])
        assert np.array_equal(orc.grad(inst, k0, k1)[0].reshape(n + m, -1), full["grad"][:, k0:k1])


def test_bad_arguments_rejected(orc):
    with pytest.raises(ValueError):
        orc.sizes(0, 4, 2)
    with pytest.raises(ValueError):
        orc.sizes(10, 0, 2)
    with pytest.raises(ValueError):
        orc.sizes(10, 4, -1)
