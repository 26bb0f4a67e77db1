"""Plant plausible mistakes in the oracle's Python-level derivative
compositions (grad_z L = sigma grad f + J^T y, H v from the lower triangle,
J v, the coefficient gradient, its mixed derivative and its adjoint as
matrix products) and check that the pins
of tests/test_oracle_diff_ex_pins.py catch every one, as the C-level mutation
test does for the C oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests import test_oracle_diff_ex_pins as X

_JTY = oracle._grad_plus_jt_y  # the correct composition, before any patch


def _jt_y_no_sigma(sigma, grad, jac, jr, jc, y):
    return _JTY(1.0, grad, jac, jr, jc, y)


def _jt_y_defect_rows_only(sigma, grad, jac, jr, jc, y):
    """Drops the entries of the last rows, as if the boundary rows (which
    come after the defect rows) were forgotten."""
    jv, jmu = jac
    last = jr >= len(y) - max(1, len(y) // 50)
    return _JTY(sigma, grad, (np.where(last, 0.0, jv), jmu), jr, jc, y)


def _jt_y_row_index(sigma, grad, jac, jr, jc, y):
    g, gmu = grad
    jv, jmu = jac
    nv = len(g)
    yy = y[np.minimum(jr + 1, len(y) - 1)]  # neighbouring row's multiplier
    out = sigma * g + np.bincount(jc, weights=jv * yy, minlength=nv)
    mu = abs(sigma) * gmu + np.bincount(jc, weights=jmu * np.abs(yy), minlength=nv)
    return out, mu


def _sym_no_transpose(hess, hr, hc, v):
    hv, hmu = hess
    nv = len(v)
    return (np.bincount(hr, weights=hv * v[hc], minlength=nv),
            np.bincount(hr, weights=hmu * np.abs(v[hc]), minlength=nv))


def _sym_diagonal_twice(hess, hr, hc, v):
    hv, hmu = hess
    nv = len(v)
    out = np.bincount(hr, weights=hv * v[hc], minlength=nv) + np.bincount(hc, weights=hv * v[hr], minlength=nv)
    mu = (np.bincount(hr, weights=hmu * np.abs(v[hc]), minlength=nv)
          + np.bincount(hc, weights=hmu * np.abs(v[hr]), minlength=nv))
    return out, mu


def _coo_mv_row_col_swap(jac, jr, jc, v, rows):
    jv, jmu = jac
    return (np.bincount(jr, weights=jv * v[np.minimum(jr, len(v) - 1)], minlength=rows),
            np.bincount(jr, weights=jmu * np.abs(v[np.minimum(jr, len(v) - 1)]), minlength=rows))


def _coef_mutant(kind):
    """A copy of coef_grad_ex with one planted mistake."""
    def coef_grad_ex(self, inst, scheme=0, bnd=0, y=None):
        N, n, m = inst.N, inst.n, inst.m
        y = np.asarray(inst.y if y is None else y, dtype=float)
        NU = N + 1 if scheme == 0 else N
        Xv = np.asarray(inst.z[:n * (N + 1)], dtype=float).reshape(n, N + 1)
        U = np.asarray(inst.z[n * (N + 1):], dtype=float).reshape(m, NU)
        Y = y[:n * N].reshape(n, N)
        S = np.sin(Xv)
        partner = np.arange(n) if kind == "gamma partner" else (np.arange(n) + 1) % n
        P = Xv * Xv[partner]
        if scheme == 0:
            w = 0.5 * (1.0 / N)
            SA = S[:, :N] if kind == "trapezoid right node" else S[:, :N] + S[:, 1:]
            UB, PG = U[:, :N] + U[:, 1:], P[:, :N] + P[:, 1:]
        else:
            w = (0.5 if kind == "euler weight" else 1.0) * (1.0 / N)
            SA, UB, PG = S[:, :N], U, P[:, :N]
        Ya = np.abs(Y)
        gA, mA = -w * (Y @ SA.T), w * (Ya @ np.abs(SA).T) + 1e-300
        gB, mB = -w * (Y @ UB.T), w * (Ya @ np.abs(UB).T) + 1e-300
        gg, mg = -w * np.sum(Y * PG, axis=1), w * np.sum(Ya * np.abs(PG), axis=1) + 1e-300
        return (gA, gB, gg), (mA, mB, mg)
    return coef_grad_ex


def _mixed_mutant(kind):
    """A copy of coef_mixed_ex with one planted mistake."""
    def coef_mixed_ex(self, inst, v, scheme=0, bnd=0, y=None):
        N, n, m = inst.N, inst.n, inst.m
        y = np.asarray(inst.y if y is None else y, dtype=float)
        v = np.asarray(v, dtype=float)
        NU = N + 1 if scheme == 0 else N
        Xv = np.asarray(inst.z[:n * (N + 1)], dtype=float).reshape(n, N + 1)
        VX = v[:n * (N + 1)].reshape(n, N + 1)
        VU = v[n * (N + 1):].reshape(m, NU)
        Y = y[:n * N].reshape(n, N)
        p = (np.arange(n) + 1) % n
        C = (np.sin(Xv) if kind == "sine" else np.cos(Xv)) * VX
        Q = VX * Xv[p] if kind == "one product term" else VX * Xv[p] + Xv * VX[p]
        if scheme == 0:
            w = 0.5 * (1.0 / N)
            CA = C[:, 1:] if kind == "right node only" else C[:, :N] + C[:, 1:]
            VB, QG = VU[:, :N] + VU[:, 1:], Q[:, :N] + Q[:, 1:]
        else:
            w = 1.0 / N
            CA, VB, QG = C[:, :N], VU, Q[:, :N]
            if kind == "euler next node":
                CA = C[:, 1:]
        Ya = np.abs(Y)
        big = lambda a: w * (Ya @ np.abs(a).T) + 1e-300
        gA, mA = -w * (Y @ CA.T), big(CA)
        gB, mB = -w * (Y @ VB.T), big(VB)
        gg, mg = -w * np.sum(Y * QG, axis=1), w * np.sum(Ya * np.abs(QG), axis=1) + 1e-300
        return (gA, gB, gg), (mA, mB, mg)
    return coef_mixed_ex


def _adjoint_mutant(kind):
    """A copy of coef_adjoint_ex with one planted mistake."""
    def coef_adjoint_ex(self, inst, tA, tB, tg, scheme=0, bnd=0, y=None):
        N, n, m = inst.N, inst.n, inst.m
        y = np.asarray(inst.y if y is None else y, dtype=float)
        tA, tB, tg = (np.asarray(t, dtype=float) for t in (tA, tB, tg))
        tA, tB = tA.reshape(n, n), tB.reshape(n, m)
        NU = N + 1 if scheme == 0 else N
        Xv = np.asarray(inst.z[:n * (N + 1)], dtype=float).reshape(n, N + 1)
        U = np.asarray(inst.z[n * (N + 1):], dtype=float).reshape(m, NU)
        Y = y[:n * N].reshape(n, N)
        p = (np.arange(n) + 1) % n
        q = p if kind == "partner row" else (np.arange(n) - 1) % n
        Fs, Fu = tA @ np.sin(Xv) + tg[:, None] * Xv * Xv[p], tB @ U
        Yt = np.zeros((n, N + 1))
        if scheme == 0:
            w = 0.5 * (1.0 / N)
            Fb = Fs + Fu
            D = -w * Fb[:, :N] if kind == "right node dropped" else -w * (Fb[:, :N] + Fb[:, 1:])
            Yt[:, :N] += Y
            Yt[:, 1:] += Y
        else:
            w = 1.0 / N
            D = -w * (Fs[:, :N] + Fu)
            if kind == "euler next node":
                Yt[:, 1:] = Y
            else:
                Yt[:, :N] = Y
        Yt = -w * Yt
        C = np.sin(Xv) if kind == "sine" else np.cos(Xv)
        gX = C * (tA.T @ Yt) + Yt * tg[:, None] * Xv[p] + (Yt * tg[:, None] * Xv)[q]
        gU = tB.T @ Yt[:, :NU]
        nb = len(y) - n * N
        gz, gy = np.concatenate([gX.ravel(), gU.ravel()]), np.concatenate([D.ravel(), np.zeros(nb)])
        big = lambda a: np.abs(a) + 1e-300
        return (gz, gy), (big(gz), big(gy))
    return coef_adjoint_ex


# (name, attribute of the oracle module or of its Oracle class, replacement)
MUTATIONS = [
    ("grad_z L without sigma", "_grad_plus_jt_y", _jt_y_no_sigma),
    ("grad_z L without the last rows", "_grad_plus_jt_y", _jt_y_defect_rows_only),
    ("grad_z L with a neighbouring multiplier", "_grad_plus_jt_y", _jt_y_row_index),
    ("H v without the transposed triangle", "_sym_lower_mv", _sym_no_transpose),
    ("H v with the diagonal counted twice", "_sym_lower_mv", _sym_diagonal_twice),
    ("J v indexed by row", "_coo_mv", _coo_mv_row_col_swap),
    ("coefficient gradient without the right node", "Oracle.coef_grad_ex", _coef_mutant("trapezoid right node")),
    ("coefficient gradient with the trapezoid weight under Euler", "Oracle.coef_grad_ex", _coef_mutant("euler weight")),
    ("coefficient gradient with gamma's own state as partner", "Oracle.coef_grad_ex", _coef_mutant("gamma partner")),
    ("mixed derivative with sin for cos", "Oracle.coef_mixed_ex", _mixed_mutant("sine")),
    ("mixed derivative with one product-rule term", "Oracle.coef_mixed_ex", _mixed_mutant("one product term")),
    ("mixed derivative without the left node", "Oracle.coef_mixed_ex", _mixed_mutant("right node only")),
    ("mixed derivative at the next node under Euler", "Oracle.coef_mixed_ex", _mixed_mutant("euler next node")),
    ("adjoint with the partner's row for the bilinear term", "Oracle.coef_adjoint_ex", _adjoint_mutant("partner row")),
    ("adjoint with sin for cos", "Oracle.coef_adjoint_ex", _adjoint_mutant("sine")),
    ("adjoint defects without the right node", "Oracle.coef_adjoint_ex", _adjoint_mutant("right node dropped")),
    ("adjoint multipliers at the next node under Euler", "Oracle.coef_adjoint_ex", _adjoint_mutant("euler next node")),
]

# pins, each a call that raises when the oracle is wrong
PINS = [
    lambda orc: X.test_lag_grad_ex_complex_step(orc, 3, 2, 1, 0, 2),
    lambda orc: X.test_lag_grad_ex_complex_step(orc, 3, 2, 1, 1, 1),
    lambda orc: X.test_jvp_ex_complex_step(orc, 3, 2, 1, 1, 2),
    lambda orc: X.test_hvp_ex_mixed_difference(orc, 2, 3, 1, 0, 1),
    lambda orc: X.test_hvp_ex_mixed_difference(orc, 2, 3, 1, 1, 0),
    lambda orc: X.test_coef_grad_ex_complex_step(orc, 5, 3, 2, 0, 0),
    lambda orc: X.test_coef_grad_ex_complex_step(orc, 5, 3, 2, 1, 2),
    lambda orc: X.test_coef_mixed_ex_high_precision_differences(orc, 4, 3, 2, 0, 1),
    lambda orc: X.test_coef_mixed_ex_high_precision_differences(orc, 4, 3, 2, 1, 0),
    lambda orc: X.test_coef_adjoint_ex_high_precision(orc, 3, 3, 2, 0, 1),
    lambda orc: X.test_coef_adjoint_ex_high_precision(orc, 3, 3, 1, 1, 2),
    lambda orc: X.test_quad_lag_grad_complex_step(orc, 2, 1),
    lambda orc: X.test_quad_hvp_mixed_difference(orc, 2, 1),
    lambda orc: X.test_quad_jvp_complex_step(orc, 2, 1),
]


def test_pins_pass_on_the_oracle():
    for pin in PINS:
        pin(oracle.DEFAULT)


@pytest.mark.parametrize("name,attr,repl", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(monkeypatch, name, attr, repl):
    if attr.startswith("Oracle."):
        monkeypatch.setattr(oracle.Oracle, attr.split(".", 1)[1], repl)
    else:
        monkeypatch.setattr(oracle, attr, repl)
    caught = 0
    for pin in PINS:
        try:
            pin(oracle.DEFAULT)
        except AssertionError:
            caught += 1
    assert caught > 0, f"no pin catches: {name}"
