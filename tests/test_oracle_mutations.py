"""Plant plausible mistakes in a copy of the oracle source (on the CPU) and check
that the pins catch every one of them: a pin set that passes a wrong oracle
would prove nothing."""
from __future__ import annotations

import os

import pytest

import oracle
from tests import test_oracle_diff_pins as D
from tests import test_oracle_ex_pins as E
from tests import test_oracle_perm_pins as R
from tests import test_oracle_pins as P
from tests import test_oracle_quad_pins as Q

# (name, text in ocp_oracle.c, replacement)
MUTATIONS = [
    ("defect sign", "(x1 - x0) - hh * (F0[i] + F1[i])", "(x1 - x0) + hh * (F0[i] + F1[i])"),
    ("defect pairing", "(x1 - x0) - hh * (F0[i] + F1[i])", "(x1 - x0) - hh * (F0[i] + F0[i])"),
    ("defect direction", "(x1 - x0) - hh * (F0[i] + F1[i])", "(x0 - x1) - hh * (F0[i] + F1[i])"),
    ("bilinear partner index", "int p = (i + 1) % n;\n        t = gam[i]", "int p = i;\n        t = gam[i]"),
    ("dropped control term", "t = B[i * m + l] * U", "t = 0.0 * U"),
    ("transposed A in dynamics", "t = A[i * n + j] * sin(", "t = A[j * n + i] * sin("),
    ("end weight at N", "(k == 0 || k == N) ? hh : h", "(k == 0) ? hh : h"),
    ("jac right node", "out[e1] = d - hh * g1;", "out[e1] = d - hh * g0;"),
    ("jac identity sign", "out[e0] = -d - hh * g0;", "out[e0] = d - hh * g0;"),
    ("jac cos->sin", "double a = A[i * n + j] * cos(", "double a = A[i * n + j] * sin("),
    ("jac bilinear partner", "if (j == p) { g += gam[i] * X[(int64_t)i", "if (j == p) { g += gam[i] * X[(int64_t)p"),
    ("jac control slot", "double v = -hh * B[i * m + l];", "double v = hh * B[i * m + l];"),
    ("pattern slot order", "col = j * (N + 1) + k + (t % 2);", "col = j * (N + 1) + k + 1 - (t % 2);"),
    ("hess pair sign", "out[e] = -hh * yt[i] * gam[i];", "out[e] = hh * yt[i] * gam[i];"),
    ("hess multiplier range", "if (k <= N - 1) { a += y", "if (k < N - 1) { a += y"),
    ("hess transposed A", "s += yt[i] * A[i * n + j];", "s += yt[i] * A[j * n + i];"),
    ("hess n=1 fold", "v += -h * yt[0] * gam[0];", "v += -hh * yt[0] * gam[0];"),
    ("hess sigma", "double v = 2.0 * sigma * w * q[j] + hh * sx * s;", "double v = 2.0 * w * q[j] + hh * sx * s;"),
    ("pattern pair triangle", "int hi = a > b ? a : b", "int hi = a"),
    ("grad factor", "double v = 2.0 * w * q[j] * X", "double v = w * q[j] * X"),
    ("grad control weight", "double v = 2.0 * w * r[l] * U", "double v = 2.0 * r[l] * U"),
    ("kkt column order", "if (x->col != y->col) return x->col < y->col ? -1 : 1;",
     "if (x->col != y->col) return x->col < y->col ? 1 : -1;"),
    ("kkt diagonal position", "kkt[rowptr[d + 1] - 1] += reg[d]", "kkt[rowptr[d]] += reg[d]"),
    ("obj control term", "double t = r[l] * u * u;", "double t = r[l] * u;"),
    ("lagrangian sigma", "out[0] = sigma * fo[0] + yc;", "out[0] = fo[0] + yc;"),
    ("J^T y node side", "*v = (right ? d : -d) - hh * g;", "*v = (right ? -d : d) - hh * g;"),
    ("J^T y multiplier index", "s += v * y[(int64_t)i * N + k - 1];", "s += v * y[(int64_t)i * N + k];"),
    ("J^T y control weight", "double v = -hh * B[i * m + l];\n                if (k >= 1)",
     "double v = -hh * B[l * n + i];\n                if (k >= 1)"),
    ("hvp pair symmetry", "Hb[p * nv + i] += -hh * yt[i] * gam[i];", "Hb[p * nv + i] += 0.0 * yt[i];"),
    ("hvp curvature sign", "double t = -hh * yt[i] * (-A[i * n + a] * sx);",
     "double t = -hh * yt[i] * (A[i * n + a] * sx);"),
    ("jvp control node", "double vv = VU[(int64_t)l * (N + 1) + k + right];",
     "double vv = VU[(int64_t)l * (N + 1) + k];"),
    ("coef grad A node", "d = -hh * (sin(X[(int64_t)idx * (N + 1) + k]) + sin(X[(int64_t)idx * (N + 1) + k + 1]));",
     "d = -hh * (sin(X[(int64_t)idx * (N + 1) + k]) + sin(X[(int64_t)idx * (N + 1) + k]));"),
    ("coef grad gamma partner", "d = -hh * (X[(int64_t)i * (N + 1) + k] * X[(int64_t)p * (N + 1) + k]",
     "d = -hh * (X[(int64_t)i * (N + 1) + k] * X[(int64_t)i * (N + 1) + k]"),
    ("euler defect factor", "c[r0] = (x1 - x0) - h * F0[i];", "c[r0] = (x1 - x0) - hh * F0[i];"),
    ("euler cost at last node", "return k < d->N ? h : 0.0;", "return k <= d->N ? h : 0.0;"),
    ("euler next-node entry", "v = 1.0; va = 1.0;", "v = -1.0; va = 1.0;"),
    ("euler column order", "if (t <= i) return (int64_t)t * (d->N + 1) + k;",
     "if (t < i) return (int64_t)t * (d->N + 1) + k;"),
    ("euler state slot", "int j = t <= i ? t : t - 1;", "int j = t < i ? t : t - 1;"),
    ("euler multiplier of node", "if (scheme == 0 && k >= 1) { a += y", "if (k >= 1) { a += y"),
    ("euler hessian factor", "double fac = scheme == 0 ? 0.5 * h : h;", "double fac = 0.5 * h;"),
    ("final boundary node", "int64_t node = b < n ? 0 : N;", "int64_t node = 0;"),
    ("final boundary column", "(b % n) * (N + 1) + (b < n ? 0 : N));", "(b % n) * (N + 1) + (b < n ? 0 : N - 1));"),
    ("quad F4 sign", "F[3] = a - b;", "F[3] = a + b;"),
    ("quad F7 roll term", "a = u[1] * t.c7 / t.c8; b = u[2] * t.s7 / t.c8;", "a = u[1] * t.c7 / t.c8; b = u[2] * t.s7 * t.c8;"),
    ("quad gravity sign", "F[5] = a - g;", "F[5] = a + g;"),
    ("quad yaw rate partner", "a = u[1] * t.c7 * t.t8; b = u[2] * t.s7 * t.t8; c = u[3];", "a = u[1] * t.c7 * t.t8; b = u[2] * t.s7 * t.t8; c = u[2];"),
    ("quad jac pitch partial", "SET1(1, 7, u[0] * t.c7 * t.c8 * t.c9);", "SET1(1, 7, u[0] * t.c7 * t.c8 * t.s9);"),
    ("quad jac sec^2", "SET2(8, 7, u[1] * t.c7 * sec2, u[2] * t.s7 * sec2);", "SET2(8, 7, u[1] * t.c7 / t.c8, u[2] * t.s7 * sec2);"),
    ("quad jac thrust column", "SET2(3, 9, t.c7 * t.s8 * t.s9, -t.s7 * t.c9);", "SET2(3, 9, t.c7 * t.s8 * t.s9, t.s7 * t.c9);"),
    ("quad support of F8", "{ 6, 7, 10, 11 },        /* F8", "{ 6, 7, 9, 11 },        /* F8"),
    ("quad jac identity side", "double id = v == i ? (s ? 1.0 : -1.0) : 0.0;", "double id = v == i ? (s ? -1.0 : 1.0) : 0.0;"),
    ("quad hess second of 1/cos", "double dsec2 = (1.0 + s8 * s8) / (c8 * c8 * c8);", "double dsec2 = (1.0 - s8 * s8) / (c8 * c8 * c8);"),
    ("quad hess cross term sign", "S1(5, 6, 7, u[0] * t.s7 * t.s8);", "S1(5, 6, 7, -u[0] * t.s7 * t.s8);"),
    ("quad hess node multiplier", "if (k >= 1) yt[i] += y[(int64_t)i * N + k - 1];", "if (k >= 1) yt[i] += y[(int64_t)i * N + k];"),
    ("quad hess pattern entry", "{ 10, 6 }, { 10, 7 }, { 10, 10 },", "{ 10, 6 }, { 10, 8 }, { 10, 10 },"),
    ("quad tracked states", "{ 1, 0, 1, 0, 1, 0, 1, 1, 1, 0, 0, 0, 0 }", "{ 1, 1, 0, 0, 1, 0, 1, 1, 1, 0, 0, 0, 0 }"),
    ("quad reference amplitude", "d[1] = 2.0 * sin(4.0 * Q_PI * t);", "d[1] = sin(4.0 * Q_PI * t);"),
    ("quad reference ramp", "d[2] = 2.0 * t;", "d[2] = t;"),
    ("quad cost half", "acc_add(&a, w * (0.5 * L));", "acc_add(&a, w * L);"),
    ("quad boundary node", "double v = z[(int64_t)(b % QN) * (N + 1) + (b < QN ? 0 : N)];", "double v = z[(int64_t)(b % QN) * (N + 1) + (b < QN ? 0 : N - 1)];"),
    ("permute column of an entry", "ent_t t = { col, q };", "ent_t t = { row, q };"),
    ("permute inverse ordering", "        pos[o] = i;\n", "        pos[i] = o;\n"),
    ("permute diagonal map", "diag2[d] = (int32_t)map[rowptr[d + 1] - 1];", "diag2[d] = (int32_t)map[rowptr[d]];"),
    ("mapped assembly reg add", "kkt[diag[d]] += reg[d];", "kkt[diag[d]] = reg[d];"),
]

# Pins run against each mutant: (test function, arguments after the oracle).
PINS = [
    (P.test_golden_generated_code, ()),
    (P.test_pattern_unique_lower, (5, 2, 0)),
    (P.test_jacobian_pattern_is_nonzero_set, (3, 3, 1)),
    (P.test_kkt_matches_scipy, (6, 5, 3)),
    (P.test_kkt_spmv_equals_dense, (3, 3, 1)),
    (P.test_kkt_spmv_equals_dense, (3, 1, 0)),
    (P.test_objective_constant_state, (7,)),
    (P.test_objective_vs_exact_rational, (1000, 4, 2)),
    (P.test_linear_quadratic_case, (20, 3, 2)),
    (P.test_defects_of_exact_trajectory_are_third_order, (4, 2)),
    (P.test_jacobian_dense_complex_step, (5, 4, 2)),
    (P.test_jacobian_dense_complex_step, (2, 1, 1)),
    (P.test_gradient_complex_step_and_central_difference, (5, 3, 2)),
    (P.test_hessian_dense_mixed_difference, (2, 4, 2)),
    (P.test_hessian_dense_mixed_difference, (3, 1, 0)),
    (D.test_lagrangian_value_high_precision, (7, 3, 2)),
    (D.test_lag_grad_complex_step, (4, 3, 1)),
    (D.test_lag_grad_complex_step, (6, 3, 3)),
    (D.test_hvp_mixed_difference, (2, 4, 2)),
    (D.test_hvp_mixed_difference, (3, 1, 0)),
    (D.test_jvp_complex_step, (5, 4, 2)),
    (D.test_coef_grad_complex_step_and_central_difference, (5, 3, 2)),
    (E.test_golden_euler_and_boundary, ()),
    (E.test_euler_defects_of_exact_trajectory_are_second_order, (4, 2)),
    (E.test_jacobian_complex_step_and_pattern, (3, 3, 1, 1, 2)),
    (E.test_jacobian_complex_step_and_pattern, (4, 1, 1, 1, 1)),
    (E.test_hessian_mixed_difference, (3, 3, 1, 1, 1)),
    (E.test_hessian_mixed_difference, (2, 1, 1, 1, 0)),
    (E.test_kkt_generic_matches_scipy, (5, 3, 2, 1, 2)),
    (E.test_euler_linear_quadratic_case, (2,)),
    (E.test_trapezoidal_branch_equals_pinned_functions, (9, 2, 1)),
    (Q.test_sizes_and_pattern, ()),
    (Q.test_hover_has_zero_defects_exactly, ()),
    (Q.test_defects_of_exact_trajectory_are_third_order, ()),
    (Q.test_objective_closed_form_at_zero, (7,)),
    (Q.test_objective_exact_tracking, ()),
    (Q.test_constraints_match_definition, ()),
    (Q.test_jacobian_complex_step_and_pattern, (3, 2)),
    (Q.test_gradient_complex_step, ()),
    (Q.test_hessian_mixed_difference, (1, 1, 1.3)),
    (Q.test_kkt_matches_scipy, (3, 1)),
    (R.test_permuted_structure_matches_scipy, (5, 3, 2, 0, 0)),
    (R.test_mapped_assembly_equals_dense_reordering, (6, 3, 2, 0, 0)),
]


def test_mutations_apply_to_current_source():
    src = open(oracle.SRC).read()
    for name, old, _new in MUTATIONS:
        assert src.count(old) >= 1, name


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(oracle.SRC).read()
    assert old in src
    mutant = oracle.build_variant(src.replace(old, new, 1), os.path.join(tmp_path, "mut.so"))
    caught = []
    for fn, args in PINS:
        try:
            fn(mutant, *args)
        except (AssertionError, ValueError) as e:  # noqa: PERF203
            caught.append(fn.__name__)
    assert caught, f"no pin catches the planted mistake '{name}'"
