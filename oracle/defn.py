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
