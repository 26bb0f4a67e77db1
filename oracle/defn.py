"""Definition of the transcribed NLP's objective and constraints, in any number type.

Test infrastructure only.  Pure-Python loops over a flat unknown vector, so it
works with floats, complex numbers (complex-step differentiation), mpmath
numbers and sympy expressions alike; only for small N.

Written from the paper's statement of direct transcription (Sec. 3) and its
trapezoidal generated code (Sec. 5): one defect generator per state component,
    c_i(k) = (x_i[k+1] - x_i[k]) - dt * (f_i[k] + f_i[k+1]) / 2,
and the Lagrange cost as the sum of two generators, the end nodes k in {0, N}
weighted dt/2 and the interior nodes weighted dt.  The dynamics and cost are
those of the synthetic workload family:
    f_i(x, u) = sum_j A_ij sin(x_j) + sum_l B_il u_l + gamma_i x_i x_{(i+1) mod n}
    running cost  x^T diag(q) x + u^T diag(r) u.
"""
from __future__ import annotations

import math


def unpack(z, N, n, m):
    """Per-node state and control lists from the component-major unknowns."""
    xs = [[z[j * (N + 1) + k] for j in range(n)] for k in range(N + 1)]
    off = n * (N + 1)
    us = [[z[off + l * (N + 1) + k] for l in range(m)] for k in range(N + 1)]
    return xs, us


def rhs(x, u, A, B, gamma, sin=math.sin):
    """Right-hand side f(x, u) of the ODE at one node."""
    n, m = len(x), len(u)
    out = []
    for i in range(n):
        acc = 0
        for j in range(n):
            acc = acc + A[i][j] * sin(x[j])
        for l in range(m):
            acc = acc + B[i][l] * u[l]
        acc = acc + gamma[i] * x[i] * x[(i + 1) % n]
        out.append(acc)
    return out


def running_cost(x, u, q, r):
    acc = 0
    for j in range(len(x)):
        acc = acc + q[j] * x[j] * x[j]
    for l in range(len(u)):
        acc = acc + r[l] * u[l] * u[l]
    return acc


def objective(z, N, n, m, q, r, dt=None):
    """Trapezoidal Lagrange cost: end-node generator (weight dt/2) + interior one (dt)."""
    dt = 1.0 / N if dt is None else dt
    xs, us = unpack(z, N, n, m)
    ends = 0
    for k in (0, N):
        ends = ends + dt * running_cost(xs[k], us[k], q, r) / 2
    inner = 0
    for k in range(1, N):
        inner = inner + dt * running_cost(xs[k], us[k], q, r)
    return ends + inner


def constraints(z, N, n, m, A, B, gamma, sin=math.sin, dt=None):
    """Defects, one generator per state component: list indexed i*N + k."""
    dt = 1.0 / N if dt is None else dt
    xs, us = unpack(z, N, n, m)
    fs = [rhs(xs[k], us[k], A, B, gamma, sin) for k in range(N + 1)]
    c = []
    for i in range(n):
        for k in range(N):
            c.append((xs[k + 1][i] - xs[k][i]) - dt * (fs[k][i] + fs[k + 1][i]) / 2)
    return c


def lagrangian(z, y, sigma, N, n, m, A, B, gamma, q, r, sin=math.sin, dt=None):
    """L(z, y) = sigma f(z) + y^T c(z)."""
    f = objective(z, N, n, m, q, r, dt)
    c = constraints(z, N, n, m, A, B, gamma, sin, dt)
    acc = sigma * f
    for a, b in zip(y, c):
        acc = acc + a * b
    return acc


def as_lists(inst):
    """Coefficients of a synth.Instance as nested Python lists."""
    return ([list(map(float, row)) for row in inst.A], [list(map(float, row)) for row in inst.B],
            list(map(float, inst.gamma)), list(map(float, inst.q)), list(map(float, inst.r)))


# ---- forward Euler (paper Sec. 3) and boundary rows --------------------------

def unpack_ex(z, N, n, m, scheme):
    """Per-node states (N+1 nodes) and controls (N+1 nodes trapezoidal, N Euler)."""
    NU = N + 1 if scheme == 0 else N
    xs = [[z[j * (N + 1) + k] for j in range(n)] for k in range(N + 1)]
    off = n * (N + 1)
    us = [[z[off + l * NU + k] for l in range(m)] for k in range(NU)]
    return xs, us


def objective_ex(z, N, n, m, q, r, scheme, dt=None):
    """Trapezoidal cost (scheme 0) or the forward-Euler Bolza-type sum
    sum_{i<N} h f0(X_i, U_i) (scheme 1)."""
    if scheme == 0:
        return objective(z, N, n, m, q, r, dt)
    dt = 1.0 / N if dt is None else dt
    xs, us = unpack_ex(z, N, n, m, 1)
    acc = 0
    for k in range(N):
        acc = acc + dt * running_cost(xs[k], us[k], q, r)
    return acc


def constraints_ex(z, N, n, m, A, B, gamma, scheme, bnd, sin=math.sin, dt=None):
    """Defect rows (one generator per state component; trapezoidal, or forward
    Euler X_{i+1} - X_i - h f(X_i, U_i)), then the boundary rows: the initial
    state X_0 (bnd >= 1) and the final state X_N (bnd == 2), component by
    component, as the paper's x(0) == x0 generator with lcon = ucon."""
    dt_ = 1.0 / N if dt is None else dt
    if scheme == 0:
        c = constraints(z, N, n, m, A, B, gamma, sin, dt)
    else:
        xs, us = unpack_ex(z, N, n, m, 1)
        c = []
        for i in range(n):
            for k in range(N):
                f = rhs(xs[k], us[k], A, B, gamma, sin)
                c.append(xs[k + 1][i] - xs[k][i] - dt_ * f[i])
    xs, _ = unpack_ex(z, N, n, m, scheme)
    if bnd >= 1:
        c.extend(xs[0][i] for i in range(n))
    if bnd == 2:
        c.extend(xs[N][i] for i in range(n))
    return c


def lagrangian_ex(z, y, sigma, N, n, m, A, B, gamma, q, r, scheme, bnd, sin=math.sin, dt=None):
    f = objective_ex(z, N, n, m, q, r, scheme, dt)
    c = constraints_ex(z, N, n, m, A, B, gamma, scheme, bnd, sin, dt)
    acc = sigma * f
    for a, b in zip(y, c):
        acc = acc + a * b
    return acc


# ---- the quadrotor model (paper Appendix A) -----------------------------------
#
# States x1..x9 are indices 0..8 (positions x1, x3, x5; velocities x2, x4, x6;
# Euler angles x7, x8, x9), controls u1..u4 are indices 0..3.  Transcribed with
# the trapezoidal scheme of Sec. 5 on t in [0, 1]; the cost is one half of the
# integral of the tracking error of x1, x3, x5 against sin(2 pi t),
# 2 sin(4 pi t) and 2 t, plus the squared angles and r times the squared
# controls.  ``fn`` supplies sin, cos, tan and pi (math, cmath, mpmath or sympy).

def quad_unpack(z, N):
    xs = [[z[j * (N + 1) + k] for j in range(9)] for k in range(N + 1)]
    off = 9 * (N + 1)
    us = [[z[off + l * (N + 1) + k] for l in range(4)] for k in range(N + 1)]
    return xs, us


def quad_rhs(x, u, g, fn=math):
    """The nine right-hand sides of the quadrotor ODE, as the paper states them."""
    s7, c7 = fn.sin(x[6]), fn.cos(x[6])
    s8, c8, t8 = fn.sin(x[7]), fn.cos(x[7]), fn.tan(x[7])
    s9, c9 = fn.sin(x[8]), fn.cos(x[8])
    return [
        x[1],
        u[0] * c7 * s8 * c9 + u[0] * s7 * s9,
        x[3],
        u[0] * c7 * s8 * s9 - u[0] * s7 * c9,
        x[5],
        u[0] * c7 * c8 - g,
        u[1] * c7 / c8 + u[2] * s7 / c8,
        -u[1] * s7 + u[2] * c7,
        u[1] * c7 * t8 + u[2] * s7 * t8 + u[3],
    ]


def quad_running_cost(t, x, u, r, fn=math):
    """Integrand of the quadrotor cost, including its factor one half."""
    d1 = fn.sin(2 * fn.pi * t)
    d3 = 2 * fn.sin(4 * fn.pi * t)
    d5 = 2 * t
    acc = (x[0] - d1) ** 2 + (x[2] - d3) ** 2 + (x[4] - d5) ** 2
    acc = acc + x[6] ** 2 + x[7] ** 2 + x[8] ** 2
    acc = acc + r * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2 + u[3] ** 2)
    return acc / 2


def quad_objective(z, N, r, fn=math, dt=None):
    """Trapezoidal cost: end nodes weighted dt/2, interior nodes dt; t_k = k dt."""
    dt = 1.0 / N if dt is None else dt
    xs, us = quad_unpack(z, N)
    ends = 0
    for k in (0, N):
        ends = ends + dt * quad_running_cost(k * dt, xs[k], us[k], r, fn) / 2
    inner = 0
    for k in range(1, N):
        inner = inner + dt * quad_running_cost(k * dt, xs[k], us[k], r, fn)
    return ends + inner


def quad_constraints(z, N, g, bnd, fn=math, dt=None):
    """Trapezoidal defects (row i N + k), then the boundary rows X_i0 (bnd >= 1)
    and X_iN (bnd == 2)."""
    dt = 1.0 / N if dt is None else dt
    xs, us = quad_unpack(z, N)
    fs = [quad_rhs(xs[k], us[k], g, fn) for k in range(N + 1)]
    c = []
    for i in range(9):
        for k in range(N):
            c.append((xs[k + 1][i] - xs[k][i]) - dt * (fs[k][i] + fs[k + 1][i]) / 2)
    if bnd >= 1:
        c.extend(xs[0][i] for i in range(9))
    if bnd == 2:
        c.extend(xs[N][i] for i in range(9))
    return c


def quad_lagrangian(z, y, sigma, N, g, r, bnd, fn=math, dt=None):
    f = quad_objective(z, N, r, fn, dt)
    c = quad_constraints(z, N, g, bnd, fn, dt)
    acc = sigma * f
    for a, b in zip(y, c):
        acc = acc + a * b
    return acc
