"""Seeded synthetic inputs for the trapezoidal optimal-control NLP workloads.

This module only draws random numbers and lays them out; it contains none of
the transcription arithmetic (no dynamics, no derivatives, no weights).  Both
the CPU oracle and the GPU library consume what it returns.

Workload family (one instance):
    dynamics   f_i(x, u) = sum_j A_ij sin(x_j) + sum_l B_il u_l + gamma_i x_i x_{(i+1) mod n}
    cost       integral of x^T Q x + u^T R u, Q = diag(q), R = diag(r)
    grid       uniform, t in [0, 1], N intervals, N + 1 nodes

Draw order for one instance, from ``numpy.random.default_rng(seed)`` (PCG64):
    A ~ N(0, 1/n)  (standard deviation n**-0.5), shape (n, n)
    B ~ N(0, 1), shape (n, m)
    gamma ~ U(-0.5, 0.5), shape (n,)
    X ~ N(0, 1), shape (n, N + 1)       state at every node
    U ~ U(-1, 1), shape (m, N + 1)      control at every node
    y ~ N(0, 1), shape (n, N)           one multiplier per defect row
and q = 1, r = 0.1, sigma = 1.  The unknown vector is z = [X.ravel(), U.ravel()]
(component-major: all nodes of state 0, then state 1, ..., then the controls).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Instance:
    N: int
    n: int
    m: int
    A: np.ndarray      # (n, n) row-major
    B: np.ndarray      # (n, m) row-major
    gamma: np.ndarray  # (n,)
    q: np.ndarray      # (n,)
    r: np.ndarray      # (m,)
    z: np.ndarray      # (nvar,) = [X (n, N+1) | U (m, N+1)], row-major blocks
    y: np.ndarray      # (ncon,) multipliers, row (i, k) at i*N + k, then boundary rows
    sigma: float
    scheme: int = 0    # 0 trapezoidal (controls on N+1 nodes), 1 forward Euler (N nodes)
    bnd: int = 0       # boundary rows: 0 none, 1 initial state, 2 initial and final state

    @property
    def NU(self) -> int:
        return self.N + 1 if self.scheme == 0 else self.N

    @property
    def X(self) -> np.ndarray:
        return self.z[: self.n * (self.N + 1)].reshape(self.n, self.N + 1)

    @property
    def U(self) -> np.ndarray:
        return self.z[self.n * (self.N + 1):].reshape(self.m, self.NU)


def coefficients(rng: np.random.Generator, n: int, m: int):
    """Draw (A, B, gamma) in the fixed order."""
    A = rng.normal(0.0, n ** -0.5, (n, n))
    B = rng.normal(0.0, 1.0, (n, m))
    gamma = rng.uniform(-0.5, 0.5, n)
    return A, B, gamma


def point(rng: np.random.Generator, N: int, n: int, m: int):
    """Draw an evaluation point (X, U) and multipliers y, in that order."""
    X = rng.normal(0.0, 1.0, (n, N + 1))
    U = rng.uniform(-1.0, 1.0, (m, N + 1))
    y = rng.normal(0.0, 1.0, (n, N))
    return X, U, y


def make_instance(N: int, n: int, m: int, seed=0, scheme: int = 0, bnd: int = 0) -> Instance:
    """One instance of the workload family; ``seed`` may be an int or a list.
    Under the forward-Euler scheme the controls live on N nodes; boundary rows
    add n (initial) or 2n (initial and final) multipliers, drawn after the
    defect multipliers."""
    rng = np.random.default_rng(seed)
    A, B, gamma = coefficients(rng, n, m)
    NU = N + 1 if scheme == 0 else N
    X = rng.normal(0.0, 1.0, (n, N + 1))
    U = rng.uniform(-1.0, 1.0, (m, NU))
    y = rng.normal(0.0, 1.0, n * N + bnd * n)
    z = np.concatenate([X.ravel(), U.ravel()])
    return Instance(N=N, n=n, m=m, A=np.ascontiguousarray(A), B=np.ascontiguousarray(B),
                    gamma=gamma, q=np.ones(n), r=np.full(m, 0.1),
                    z=np.ascontiguousarray(z), y=np.ascontiguousarray(y),
                    sigma=1.0, scheme=scheme, bnd=bnd)


# Named workloads: (N, n, m).
PARITY = (1000, 4, 2)           # one evaluation of everything, seed 0
IPM_LOOP = (100_000, 8, 4)      # repeated cons + jac + hess + assemble
LARGE = (1_000_000, 16, 8)      # dense 16x16 A; the roofline workload
DIFF = (200_000, 8, 4)          # Lagrangian differentiation workload


def batched_sizes(count: int = 512, lo: int = 200, hi: int = 20000, seed: int = 0) -> np.ndarray:
    """Per-instance interval counts N_b ~ U{lo..hi} for the batched workload."""
    return np.random.default_rng(seed).integers(lo, hi + 1, count)


def device_point(torch, device, N: int, n: int, m: int, seed: int):
    """A fresh evaluation point drawn on the GPU with torch's generator:
    z = [X ~ N(0,1) (n, N+1) | U ~ U(-1,1) (m, N+1)] and y ~ N(0,1) (n*N),
    drawn in that order from ``torch.Generator(device).manual_seed(seed)``."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = dict(dtype=torch.float64, device=device)
    X = torch.randn(n * (N + 1), generator=g, **f64)
    U = torch.rand(m * (N + 1), generator=g, **f64) * 2.0 - 1.0
    y = torch.randn(n * N, generator=g, **f64)
    return torch.cat([X, U]), y


def make_batch(count: int = 512, n: int = 6, m: int = 3, seed: int = 0, Ns=None, scheme: int = 0,
               bnd: int = 0):
    """Instances of the batched workload: N_b from ``batched_sizes`` (unless
    given), instance b drawn from ``default_rng([seed, b])`` in the
    single-instance order (A, B, gamma, X, U, y), with the given scheme and
    boundary option."""
    Ns = batched_sizes(count, seed=seed) if Ns is None else Ns
    return [make_instance(int(N), n, m, seed=[seed, b], scheme=scheme, bnd=bnd) for b, N in enumerate(Ns)]


def pack(insts):
    """Packed z and y of a list of instances (instance after instance)."""
    return (np.concatenate([i.z for i in insts]), np.concatenate([i.y for i in insts]))


# ---- quadrotor-shaped workload ------------------------------------------------
#
# The paper's quadrotor benchmark (Appendix A): 9 states (positions x1, x3, x5,
# velocities x2, x4, x6, Euler angles x7, x8, x9), 4 controls (thrust u1, body
# rates u2, u3, u4), on t in [0, 1] with g = 9.8 and control weight r = 0.1,
# and the initial state fixed.  Only the evaluation point is drawn here:
#     positions and velocities ~ N(0, 1), shape (6, N + 1)
#     angles ~ U(-0.5, 0.5) rad, shape (3, N + 1)   (|x8| < pi/2 keeps 1/cos finite)
#     thrust ~ U(5, 15), shape (1, N + 1)           (around hover, u1 = g)
#     rates ~ U(-1, 1), shape (3, N + 1)
#     y ~ N(0, 1), 9 N defect multipliers then 9 per boundary group
# drawn in that order from ``default_rng(seed)``; sigma = 1.

QUAD_N, QUAD_M = 9, 4
QUAD_G, QUAD_R = 9.8, 0.1


@dataclass
class QuadInstance:
    N: int
    z: np.ndarray    # [X (9, N+1) | U (4, N+1)], row-major blocks
    y: np.ndarray    # 9 N defect multipliers, then 9 per boundary group
    sigma: float
    g: float = QUAD_G
    r: float = QUAD_R
    bnd: int = 1     # boundary rows: 0 none, 1 initial state (the paper's model), 2 initial and final
    n: int = QUAD_N
    m: int = QUAD_M

    @property
    def X(self) -> np.ndarray:
        return self.z[: 9 * (self.N + 1)].reshape(9, self.N + 1)

    @property
    def U(self) -> np.ndarray:
        return self.z[9 * (self.N + 1):].reshape(4, self.N + 1)


def make_quadrotor(N: int, seed=0, bnd: int = 1) -> QuadInstance:
    """One evaluation point of the quadrotor-shaped workload (draw order above)."""
    rng = np.random.default_rng(seed)
    pv = rng.normal(0.0, 1.0, (6, N + 1))
    ang = rng.uniform(-0.5, 0.5, (3, N + 1))
    thrust = rng.uniform(5.0, 15.0, (1, N + 1))
    rates = rng.uniform(-1.0, 1.0, (3, N + 1))
    y = rng.normal(0.0, 1.0, 9 * N + 9 * bnd)
    z = np.concatenate([pv.ravel(), ang.ravel(), thrust.ravel(), rates.ravel()])
    return QuadInstance(N=N, z=np.ascontiguousarray(z), y=np.ascontiguousarray(y), sigma=1.0, bnd=bnd)


QUAD_LARGE = 1_000_000   # quadrotor roofline workload
QUAD_PAPER = 200_000     # the paper's largest quadrotor grid
