"""Pins of the oracle's forward-Euler scheme and boundary rows (the _ex family):
the paper's Sec. 3 definitions worked by hand, an ODE integrator, complex
step, mixed differences, sympy and scipy -- and agreement of the _ex family's
trapezoidal branch with the separately pinned trapezoidal functions."""
from __future__ import annotations

import cmath
import json
import os

import numpy as np
import pytest

import synth
from oracle import defn
from tests.helpers import EPS, check_close, dense_from_coo, sym_from_lower

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CASES = [(s, b) for s in (0, 1) for b in (0, 1, 2)]


def inst_ex(N, n, m, scheme, bnd, seed=0, **over):
    inst = synth.make_instance(N, n, m, seed=seed, scheme=scheme, bnd=bnd)
    for k, v in over.items():
        setattr(inst, k, v)
    return inst


def test_golden_euler_and_boundary(orc):
    g = json.load(open(os.path.join(GOLDEN, "euler_and_boundary.json")))
    N = g["N"]
    assert g["dt"] == 1.0 / N
    inst = inst_ex(N, 1, 1, 1, 2, A=np.zeros((1, 1)), B=np.ones((1, 1)), gamma=np.zeros(1),
                   q=np.array(g["q"]), r=np.array(g["r"]),
                   z=np.array(g["x"] + g["u"], dtype=np.float64), y=np.ones(N + 2))
    c, _ = orc.cons_ex(inst, 1, 2)
    assert c.tolist() == g["rows"]
    f, _ = orc.obj_ex(inst, 1, 2)
    assert f == g["objective"]
    jv, _ = orc.jac_ex(inst, 1, 2)
    row = g["jacobian_row"]
    # Euler slots of row (0, k) in column order: x_k, x_{k+1}, u_k; then the boundary entries
    T = 3
    for k in range(N):
        assert jv[0 * N + k] == row["d_x_i"]
        assert jv[1 * N + k] == row["d_x_i1"]
        assert jv[2 * N + k] == row["d_u_i"]
    assert jv[T * N:].tolist() == [1.0, 1.0]
    hv, _ = orc.hess_ex(inst, 1, 2, sigma=1.0)
    assert hv[:N + 1].tolist() == g["hessian_x_diag"]
    assert hv[N + 1:].tolist() == g["hessian_u_diag"]


@pytest.mark.parametrize("N,n,m", [(1000, 4, 2), (7, 1, 0), (9, 2, 1), (33, 5, 3)])
def test_trapezoidal_branch_equals_pinned_functions(orc, N, n, m):
    inst = synth.make_instance(N, n, m, seed=3)
    assert orc.obj_ex(inst, 0, 0) == orc.obj(inst)
    for a, b in ((orc.grad_ex(inst, 0, 0), orc.grad(inst)), (orc.cons_ex(inst, 0, 0), orc.cons(inst)),
                 (orc.jac_ex(inst, 0, 0), orc.jac(inst)), (orc.hess_ex(inst, 0, 0), orc.hess(inst))):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for a, b in zip(orc.pattern_ex(N, n, m, 0, 0), orc.pattern(N, n, m)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n,m", [(4, 2), (2, 1), (1, 1)])
def test_euler_defects_of_exact_trajectory_are_second_order(orc, n, m):
    """Along an accurate solution of x' = f(x, u(t)), forward-Euler defects are
    the local error h^2 x''/2: they shrink 4x when N doubles (a wrong sign,
    index or dropped term leaves O(h))."""
    from scipy.integrate import solve_ivp
    rng = np.random.default_rng(140 + n)
    base = synth.make_instance(8, n, m, seed=140 + n)
    A, B, gam = base.A, base.B, base.gamma
    a, b = rng.normal(size=m) * 0.5, rng.normal(size=m) * 0.5
    x0 = rng.normal(size=n) * 0.5

    def f(t, x):
        return A @ np.sin(x) + B @ (a + b * t) + gam * x * np.roll(x, -1)

    sol = solve_ivp(f, (0.0, 1.0), x0, method="DOP853", rtol=1e-13, atol=1e-14, dense_output=True)
    maxc = []
    for N in (50, 100, 200):
        t = np.arange(N + 1) / N
        X = sol.sol(t)
        U = a[:, None] + b[:, None] * t[None, :N]
        inst = inst_ex(N, n, m, 1, 0, A=A, B=B, gamma=gam, z=np.concatenate([X.ravel(), U.ravel()]))
        c, _ = orc.cons_ex(inst, 1, 0)
        maxc.append(np.abs(c).max())
    for k in range(2):
        assert 3.5 < maxc[k] / maxc[k + 1] < 4.5, maxc


def _cs_jac_ex(inst, scheme, bnd, tau=1e-30):
    A, B, g, q, r = defn.as_lists(inst)
    cols = []
    for col in range(len(inst.z)):
        z = [complex(v) for v in inst.z]
        z[col] += 1j * tau
        c = defn.constraints_ex(z, inst.N, inst.n, inst.m, A, B, g, scheme, bnd, sin=cmath.sin)
        cols.append([v.imag / tau for v in c])
    return np.array(cols).T


@pytest.mark.parametrize("scheme,bnd", CASES)
@pytest.mark.parametrize("N,n,m", [(3, 3, 1), (4, 1, 1), (2, 2, 2), (3, 4, 0)])
def test_jacobian_complex_step_and_pattern(orc, N, n, m, scheme, bnd):
    inst = inst_ex(N, n, m, scheme, bnd, seed=20 + N + n)
    s = orc.sizes_ex(N, n, m, scheme, bnd)
    J = _cs_jac_ex(inst, scheme, bnd)
    assert J.shape == (s["ncon"], s["nvar"])
    jr, jc, _, _ = orc.pattern_ex(N, n, m, scheme, bnd)
    jv, mu = orc.jac_ex(inst, scheme, bnd)
    check_close(jv, J[jr, jc], mu, rel=1e-13, what="jac_ex")
    P = np.zeros_like(J, dtype=bool)
    P[jr, jc] = True
    assert np.all(J[~P] == 0)
    assert len(set(zip(jr.tolist(), jc.tolist()))) == s["nnzj"]
    # slots of every defect row in ascending column order
    cols = jc[: n * s["T"] * N].reshape(n, s["T"], N)
    assert np.all(np.diff(cols, axis=1) > 0)


@pytest.mark.parametrize("scheme,bnd", CASES)
def test_gradient_complex_step(orc, scheme, bnd):
    N, n, m = 6, 3, 2
    inst = inst_ex(N, n, m, scheme, bnd, seed=31)
    A, B, g, q, r = defn.as_lists(inst)
    gv, mu = orc.grad_ex(inst, scheme, bnd)
    cs = []
    for col in range(len(inst.z)):
        z = [complex(v) for v in inst.z]
        z[col] += 1e-30j
        cs.append(defn.objective_ex(z, N, n, m, q, r, scheme).imag / 1e-30)
    check_close(gv, np.array(cs), mu, rel=4 * EPS, what="grad_ex")


@pytest.mark.parametrize("scheme,bnd", CASES)
@pytest.mark.parametrize("N,n,m", [(3, 3, 1), (2, 1, 1), (3, 2, 0)])
def test_hessian_mixed_difference(orc, N, n, m, scheme, bnd):
    inst = inst_ex(N, n, m, scheme, bnd, seed=40 + N)
    s = orc.sizes_ex(N, n, m, scheme, bnd)
    A, B, g, q, r = defn.as_lists(inst)
    y = list(map(float, inst.y))
    nv = len(inst.z)
    H = np.zeros((nv, nv))
    tau, delta = 1e-30, 1e-5
    for a in range(nv):
        for b in range(nv):
            vals = []
            for sg in (1, -1):
                z = [complex(v) for v in inst.z]
                z[a] += 1j * tau
                z[b] += sg * delta
                vals.append(defn.lagrangian_ex(z, y, 1.4, N, n, m, A, B, g, q, r, scheme, bnd,
                                               sin=cmath.sin).imag)
            H[a, b] = (vals[0] - vals[1]) / (2 * tau * delta)
    _, _, hr, hc = orc.pattern_ex(N, n, m, scheme, bnd)
    hv, _ = orc.hess_ex(inst, scheme, bnd, sigma=1.4)
    Hs = sym_from_lower(hr, hc, hv, nv)
    scale = max(np.abs(H).max(), 1e-300)
    assert np.abs(Hs - H).max() <= 1e-8 * scale
    P = np.zeros_like(H, dtype=bool)
    P[hr, hc] = P[hc, hr] = True
    assert np.abs(H[~P]).max(initial=0.0) <= 1e-9 * scale
    assert set(hr[hr == hc].tolist()) == set(range(s["nvar"]))


@pytest.mark.parametrize("scheme,bnd", CASES)
@pytest.mark.parametrize("N,n,m", [(5, 3, 2), (40, 4, 1), (3, 1, 0), (6, 2, 3)])
def test_kkt_generic_matches_scipy(orc, N, n, m, scheme, bnd):
    import scipy.sparse as sp
    s = orc.sizes_ex(N, n, m, scheme, bnd)
    jr, jc, hr, hc = orc.pattern_ex(N, n, m, scheme, bnd)
    rowptr, colind, pj, ph = orc.kkt_ex(N, n, m, scheme, bnd)
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


@pytest.mark.parametrize("bnd", [0, 2])
def test_euler_linear_quadratic_case(orc, bnd):
    """A = 0, gamma = 0: c = X_{k+1} - X_k - h B U_k vanishes on the exact
    solution x(t) = x0 + B sum_{j<k} h u_j of the piecewise-constant control;
    the Jacobian is the constant template and the Hessian sigma 2 w diag(q, r)."""
    N, n, m = 16, 3, 2
    rng = np.random.default_rng(5)
    inst = inst_ex(N, n, m, 1, bnd, seed=6, A=np.zeros((n, n)), gamma=np.zeros(n))
    h = 1.0 / N
    U = rng.normal(size=(m, N))
    X = np.zeros((n, N + 1))
    X[:, 0] = rng.normal(size=n)
    for k in range(N):
        X[:, k + 1] = X[:, k] + h * (inst.B @ U[:, k])
    inst.z = np.concatenate([X.ravel(), U.ravel()])
    c, mu = orc.cons_ex(inst, 1, bnd)
    assert np.all(np.abs(c[: n * N]) <= 16 * EPS * mu[: n * N])
    jv, _ = orc.jac_ex(inst, 1, bnd)
    J = jv[: n * (n + 1 + m) * N].reshape(n, n + 1 + m, N)
    for i in range(n):
        for t in range(n + 1 + m):
            if t == i + 1:
                want = 1.0
            elif t <= n:
                j = t if t <= i else t - 1
                want = -1.0 if j == i else -0.0
            else:
                want = -h * inst.B[i, t - n - 1]
            assert np.all(J[i, t] == want)
    hv, _ = orc.hess_ex(inst, 1, bnd, sigma=2.0)
    w = np.full(N + 1, h)
    w[N] = 0.0
    for j in range(n):
        assert np.array_equal(hv[j * (N + 1):(j + 1) * (N + 1)], 2.0 * 2.0 * w * inst.q[j])
    base = (n + n) * (N + 1)
    for l in range(m):
        assert np.array_equal(hv[base + l * N: base + (l + 1) * N], 2.0 * 2.0 * h * inst.r[l] * np.ones(N))


@pytest.mark.slow
@pytest.mark.parametrize("N,n,m,bnd", [(2, 3, 1, 1), (3, 2, 1, 2), (2, 1, 1, 0)])
def test_euler_symbolic(orc, N, n, m, bnd):
    import sympy as S
    inst = inst_ex(N, n, m, 1, bnd, seed=70 + N)
    s = orc.sizes_ex(N, n, m, 1, bnd)
    R = lambda v: S.Rational(float(v))
    A = [[R(v) for v in row] for row in inst.A]
    B = [[R(v) for v in row] for row in inst.B] if m else [[] for _ in range(n)]
    gam = [R(v) for v in inst.gamma]
    q = [R(v) for v in inst.q]
    r = [R(v) for v in inst.r]
    zs = S.symbols(f"z0:{s['nvar']}")
    ys = S.symbols(f"y0:{s['ncon']}")
    dt = S.Rational(1, N)
    c = defn.constraints_ex(list(zs), N, n, m, A, B, gam, 1, bnd, sin=S.sin, dt=dt)
    L = defn.lagrangian_ex(list(zs), list(ys), 1, N, n, m, A, B, gam, q, r, 1, bnd, sin=S.sin, dt=dt)
    sub = {zs[i]: R(inst.z[i]) for i in range(s["nvar"])}
    sub.update({ys[i]: R(inst.y[i]) for i in range(s["ncon"])})
    jr, jc, hr, hc = orc.pattern_ex(N, n, m, 1, bnd)
    jv, jm = orc.jac_ex(inst, 1, bnd)
    hv, hm = orc.hess_ex(inst, 1, bnd, sigma=1.0)
    for e in range(s["nnzj"]):
        want = float(S.N(S.diff(c[jr[e]], zs[jc[e]]).subs(sub), 40))
        assert abs(jv[e] - want) <= 1e-14 * jm[e] + 1e-300
    inH = set(zip(hr.tolist(), hc.tolist()))
    for a in range(s["nvar"]):
        for b in range(a + 1):
            if (a, b) not in inH:
                assert S.simplify(S.diff(L, zs[a], zs[b])) == 0, (a, b)
    for e in range(s["nnzh"]):
        want = float(S.N(S.diff(L, zs[hr[e]], zs[hc[e]]).subs(sub), 40))
        assert abs(hv[e] - want) <= 1e-14 * hm[e] + 1e-300
