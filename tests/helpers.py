"""Shared test helpers: dense matrices from COO patterns, complex-step derivatives
of the definition module, and the element-wise magnitude-relative comparison."""
from __future__ import annotations

import cmath
import math

import numpy as np

import synth
from oracle import defn

EPS = np.finfo(np.float64).eps
# Values must agree within REL * mu, mu being the sum of |terms| of each entry.
REL = 1e-12


def instance(N, n, m, seed=0, **over):
    inst = synth.make_instance(N, n, m, seed)
    for k, v in over.items():
        setattr(inst, k, v)
    return inst


def dense_from_coo(rows, cols, vals, shape):
    M = np.zeros(shape)
    M[rows, cols] = vals
    return M


def sym_from_lower(rows, cols, vals, dim):
    H = np.zeros((dim, dim))
    H[rows, cols] = vals
    H[cols, rows] = vals
    return H


def cs_jacobian(inst, cols, tau=1e-30):
    """Complex-step columns of dc/dz from the definition module."""
    A, B, g, q, r = defn.as_lists(inst)
    z0 = [complex(v) for v in inst.z]
    out = np.zeros((inst.n * inst.N, len(cols)))
    for a, col in enumerate(cols):
        z = list(z0)
        z[col] = z[col] + 1j * tau
        c = defn.constraints(z, inst.N, inst.n, inst.m, A, B, g, sin=cmath.sin)
        out[:, a] = [v.imag / tau for v in c]
    return out


def cs_gradient(inst, cols, tau=1e-30):
    A, B, g, q, r = defn.as_lists(inst)
    z0 = [complex(v) for v in inst.z]
    out = np.zeros(len(cols))
    for a, col in enumerate(cols):
        z = list(z0)
        z[col] = z[col] + 1j * tau
        out[a] = defn.objective(z, inst.N, inst.n, inst.m, q, r).imag / tau
    return out


def mixed_hessian(inst, y, sigma, tau=1e-30, delta=1e-5):
    """Dense Hessian of L by complex step in one direction and central
    difference in the other:  H_ab = [Im L(z + i tau e_a + delta e_b)
    - Im L(z + i tau e_a - delta e_b)] / (2 tau delta)."""
    A, B, g, q, r = defn.as_lists(inst)
    nv = len(inst.z)
    yl = list(map(float, y))
    H = np.zeros((nv, nv))
    for a in range(nv):
        for b in range(nv):
            vals = []
            for s in (+1, -1):
                z = [complex(v) for v in inst.z]
                z[a] += 1j * tau
                z[b] += s * delta
                L = defn.lagrangian(z, yl, sigma, inst.N, inst.n, inst.m, A, B, g, q, r,
                                    sin=cmath.sin)
                vals.append(L.imag)
            H[a, b] = (vals[0] - vals[1]) / (2 * tau * delta)
    return H


def check_close(got, want, mu, rel=REL, what=""):
    """|got - want| <= rel * mu element-wise, with equality where mu == 0."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    mu = np.asarray(mu, np.float64)
    assert got.shape == want.shape == mu.shape, (what, got.shape, want.shape, mu.shape)
    err = np.abs(got - want)
    bad = err > rel * mu
    if bad.any():
        i = int(np.flatnonzero(bad)[0])
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} entries off; first at {i}: "
                             f"got {got.flat[i]!r} want {want.flat[i]!r} mu {mu.flat[i]!r}")
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(mu > 0, err / mu, 0.0)
    return float(r.max()) if r.size else 0.0


def ulp(x):
    return math.ulp(abs(x)) if x != 0 else math.ulp(0.0)
