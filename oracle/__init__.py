"""CPU oracle for the trapezoidal transcription NLP -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It shares no code with the GPU library: the C source in this
folder is compiled with gcc (never hipcc) into ``liboracle.so`` and loaded
here with ctypes.  ``defn.py`` holds an independent, dtype-generic definition
of the objective and constraints used to pin the C oracle.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ocp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc; returns the path of the shared library."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Oracle:
    """One loaded copy of the oracle library (the default one, or a variant
    compiled from an edited source in a mutation test)."""

    def __init__(self, path: str = LIB):
        self.path = path
        self._L = None

    @property
    def L(self):
        if self._L is None:
            if self.path == LIB and not os.path.exists(LIB):
                build(force=False)
            L = ctypes.CDLL(self.path)
            i64, i32, dbl, ptr = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
            L.orc_sizes.argtypes = [i64, i32, i32, ptr]
            L.orc_obj.argtypes = [i64, i32, i32, ptr, ptr, ptr, ptr]
            L.orc_grad.argtypes = [i64, i32, i32, ptr, ptr, ptr, i64, i64, ptr, ptr]
            L.orc_cons.argtypes = [i64, i32, i32, ptr, ptr, ptr, ptr, i64, i64, ptr, ptr]
            L.orc_jac.argtypes = [i64, i32, i32, ptr, ptr, ptr, ptr, i64, i64, ptr, ptr]
            L.orc_hess.argtypes = [i64, i32, i32, ptr, ptr, ptr, ptr, ptr, ptr, ptr, dbl,
                                   i64, i64, ptr, ptr]
            L.orc_pattern.argtypes = [i64, i32, i32, ptr, ptr, ptr, ptr]
            L.orc_kkt.argtypes = [i64, i32, i32, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr]
            L.orc_assemble.argtypes = [i64, i64, ptr, i64, ptr, ptr, i64, ptr, ptr, ptr, ptr]
            L.orc_lagrangian.argtypes = [i64, i32, i32, ptr, ptr, ptr, ptr, ptr, ptr, ptr, dbl, ptr]
            L.orc_lag_grad.argtypes = [i64, i32, i32, ptr, ptr, ptr, ptr, ptr, ptr, ptr, dbl,
                                       i64, i64, ptr, ptr]
            L.orc_hvp.argtypes = [i64, i32, i32, ptr, ptr, ptr, ptr, ptr, ptr, dbl, ptr,
                                  i64, i64, ptr, ptr]
            L.orc_jvp.argtypes = [i64, i32, i32, ptr, ptr, ptr, ptr, ptr, i64, i64, ptr, ptr]
            L.orc_coef_grad.argtypes = [i64, i32, i32, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr]
            L.orc_sizes_ex.argtypes = [i64, i32, i32, i32, i32, ptr]
            L.orc_obj_ex.argtypes = [i64, i32, i32, i32, i32, ptr, ptr, ptr, ptr]
            L.orc_grad_ex.argtypes = [i64, i32, i32, i32, i32, ptr, ptr, ptr, ptr, ptr]
            L.orc_cons_ex.argtypes = [i64, i32, i32, i32, i32, ptr, ptr, ptr, ptr, ptr, ptr]
            L.orc_pattern_ex.argtypes = [i64, i32, i32, i32, i32, ptr, ptr, ptr, ptr]
            L.orc_jac_ex.argtypes = [i64, i32, i32, i32, i32, ptr, ptr, ptr, ptr, ptr, ptr]
            L.orc_hess_ex.argtypes = [i64, i32, i32, i32, i32, ptr, ptr, ptr, ptr, ptr, ptr, dbl,
                                      ptr, ptr]
            L.orc_kkt_generic.argtypes = [i64, i64, i64, i64, ptr, ptr, ptr, ptr, ptr, ptr, ptr,
                                          ptr, ptr]
            L.orc_quad_sizes.argtypes = [i64, i32, ptr]
            L.orc_quad_pattern.argtypes = [i64, i32, ptr, ptr, ptr, ptr]
            L.orc_quad_obj.argtypes = [i64, dbl, ptr, ptr]
            L.orc_quad_grad.argtypes = [i64, dbl, ptr, ptr, ptr]
            L.orc_quad_cons.argtypes = [i64, i32, dbl, ptr, ptr, ptr]
            L.orc_quad_jac.argtypes = [i64, i32, ptr, ptr, ptr]
            L.orc_quad_hess.argtypes = [i64, dbl, ptr, ptr, dbl, ptr, ptr]
            L.orc_kkt_permute.argtypes = [i64, ptr, ptr, i64, ptr, i64, ptr, ptr, ptr, ptr, ptr, ptr,
                                           ptr]
            L.orc_assemble_mapped.argtypes = [i64, i64, ptr, i64, ptr, ptr, i64, ptr, ptr, ptr, ptr]
            L.orc_set_threads.argtypes = [i32]
            L.orc_set_threads.restype = None
            L.orc_get_threads.restype = i32
            self._L = L
        return self._L

    def set_threads(self, t: int) -> None:
        self.L.orc_set_threads(int(t))

    def get_threads(self) -> int:
        return int(self.L.orc_get_threads())

    def sizes(self, N, n, m) -> dict:
        out = np.zeros(8, np.int64)
        _check(self.L.orc_sizes(N, n, m, _p(out)), "sizes")
        keys = ["nvar", "ncon", "nnzj", "nnzh", "dim", "npair", "T", "S"]
        return {k: int(v) for k, v in zip(keys, out)}

    def obj(self, inst):
        """(f, mu_f)."""
        out = np.zeros(2)
        _check(self.L.orc_obj(inst.N, inst.n, inst.m, _p(_d(inst.q)), _p(_d(inst.r)),
                              _p(_d(inst.z)), _p(out)), "obj")
        return float(out[0]), float(out[1])

    def grad(self, inst, k0=0, k1=None):
        k1 = inst.N + 1 if k1 is None else k1
        K = k1 - k0
        g = np.empty((inst.n + inst.m) * K)
        mu = np.empty_like(g)
        _check(self.L.orc_grad(inst.N, inst.n, inst.m, _p(_d(inst.q)), _p(_d(inst.r)),
                               _p(_d(inst.z)), k0, k1, _p(g), _p(mu)), "grad")
        return g, mu

    def cons(self, inst, k0=0, k1=None):
        k1 = inst.N if k1 is None else k1
        K = k1 - k0
        c = np.empty(inst.n * K)
        mu = np.empty_like(c)
        _check(self.L.orc_cons(inst.N, inst.n, inst.m, _p(_d(inst.A)), _p(_d(inst.B)),
                               _p(_d(inst.gamma)), _p(_d(inst.z)), k0, k1, _p(c), _p(mu)), "cons")
        return c, mu

    def jac(self, inst, k0=0, k1=None):
        k1 = inst.N if k1 is None else k1
        K = k1 - k0
        T = 2 * inst.n + 2 * inst.m
        v = np.empty(inst.n * T * K)
        mu = np.empty_like(v)
        _check(self.L.orc_jac(inst.N, inst.n, inst.m, _p(_d(inst.A)), _p(_d(inst.B)),
                              _p(_d(inst.gamma)), _p(_d(inst.z)), k0, k1, _p(v), _p(mu)), "jac")
        return v, mu

    def hess(self, inst, k0=0, k1=None, sigma=None, y=None):
        k1 = inst.N + 1 if k1 is None else k1
        K = k1 - k0
        S = self.sizes(inst.N, inst.n, inst.m)["S"]
        v = np.empty(S * K)
        mu = np.empty_like(v)
        sigma = inst.sigma if sigma is None else sigma
        y = inst.y if y is None else y
        _check(self.L.orc_hess(inst.N, inst.n, inst.m, _p(_d(inst.A)), _p(_d(inst.B)),
                               _p(_d(inst.gamma)), _p(_d(inst.q)), _p(_d(inst.r)), _p(_d(inst.z)),
                               _p(_d(y)), float(sigma), k0, k1, _p(v), _p(mu)), "hess")
        return v, mu

    def pattern(self, N, n, m):
        """(jrow, jcol, hrow, hcol) int32 COO patterns."""
        s = self.sizes(N, n, m)
        jrow = np.empty(s["nnzj"], np.int32)
        jcol = np.empty(s["nnzj"], np.int32)
        hrow = np.empty(s["nnzh"], np.int32)
        hcol = np.empty(s["nnzh"], np.int32)
        _check(self.L.orc_pattern(N, n, m, _p(jrow), _p(jcol), _p(hrow), _p(hcol)), "pattern")
        return jrow, jcol, hrow, hcol

    def kkt(self, N, n, m, pat=None):
        """Generic sort-based KKT build: (rowptr, colind, perm_j, perm_h)."""
        s = self.sizes(N, n, m)
        jrow, jcol, hrow, hcol = self.pattern(N, n, m) if pat is None else pat
        rowptr = np.empty(s["dim"] + 1, np.int32)
        colind = np.empty(s["nnzh"] + s["nnzj"] + s["dim"], np.int32)
        perm_j = np.empty(s["nnzj"], np.int32)
        perm_h = np.empty(s["nnzh"], np.int32)
        nnzk = np.zeros(1, np.int64)
        _check(self.L.orc_kkt(N, n, m, _p(jrow), _p(jcol), _p(hrow), _p(hcol), _p(rowptr),
                              _p(colind), _p(perm_j), _p(perm_h), _p(nnzk)), "kkt")
        return rowptr, colind[: int(nnzk[0])].copy(), perm_j, perm_h

    def assemble(self, rowptr, perm_j, jvals, perm_h, hvals, reg=None):
        nnzk = int(rowptr[-1])
        dim = len(rowptr) - 1
        out = np.empty(nnzk)
        regp = None if reg is None else _d(reg)
        _check(self.L.orc_assemble(nnzk, dim, _p(np.ascontiguousarray(rowptr, np.int32)),
                                   len(perm_j), _p(np.ascontiguousarray(perm_j, np.int32)),
                                   _p(_d(jvals)), len(perm_h),
                                   _p(np.ascontiguousarray(perm_h, np.int32)), _p(_d(hvals)),
                                   _p(regp), _p(out)), "assemble")
        return out

    # ---- Lagrangian L = sigma f + y^T c and its derivatives ----------------
    def lagrangian(self, inst, sigma=None, y=None):
        """(L, mu_L)."""
        out = np.zeros(2)
        sigma = inst.sigma if sigma is None else sigma
        y = inst.y if y is None else y
        _check(self.L.orc_lagrangian(inst.N, inst.n, inst.m, _p(_d(inst.A)), _p(_d(inst.B)),
                                     _p(_d(inst.gamma)), _p(_d(inst.q)), _p(_d(inst.r)),
                                     _p(_d(inst.z)), _p(_d(y)), float(sigma), _p(out)), "lagrangian")
        return float(out[0]), float(out[1])

    def lag_grad(self, inst, k0=0, k1=None, sigma=None, y=None):
        """grad_z L at nodes [k0, k1) (layout of grad)."""
        k1 = inst.N + 1 if k1 is None else k1
        K = k1 - k0
        g = np.empty((inst.n + inst.m) * K)
        mu = np.empty_like(g)
        sigma = inst.sigma if sigma is None else sigma
        y = inst.y if y is None else y
        _check(self.L.orc_lag_grad(inst.N, inst.n, inst.m, _p(_d(inst.A)), _p(_d(inst.B)),
                                   _p(_d(inst.gamma)), _p(_d(inst.q)), _p(_d(inst.r)),
                                   _p(_d(inst.z)), _p(_d(y)), float(sigma), k0, k1, _p(g), _p(mu)),
               "lag_grad")
        return g, mu

    def hvp(self, inst, v, k0=0, k1=None, sigma=None, y=None):
        """(Hessian of L) v at nodes [k0, k1) (layout of grad); v has nvar entries."""
        k1 = inst.N + 1 if k1 is None else k1
        K = k1 - k0
        g = np.empty((inst.n + inst.m) * K)
        mu = np.empty_like(g)
        sigma = inst.sigma if sigma is None else sigma
        y = inst.y if y is None else y
        _check(self.L.orc_hvp(inst.N, inst.n, inst.m, _p(_d(inst.A)), _p(_d(inst.gamma)),
                              _p(_d(inst.q)), _p(_d(inst.r)), _p(_d(inst.z)), _p(_d(y)), float(sigma),
                              _p(_d(v)), k0, k1, _p(g), _p(mu)), "hvp")
        return g, mu

    def jvp(self, inst, v, k0=0, k1=None):
        """J v at intervals [k0, k1) (layout of cons); v has nvar entries."""
        k1 = inst.N if k1 is None else k1
        K = k1 - k0
        g = np.empty(inst.n * K)
        mu = np.empty_like(g)
        _check(self.L.orc_jvp(inst.N, inst.n, inst.m, _p(_d(inst.A)), _p(_d(inst.B)),
                              _p(_d(inst.gamma)), _p(_d(inst.z)), _p(_d(v)), k0, k1, _p(g), _p(mu)),
               "jvp")
        return g, mu

    def coef_grad(self, inst, y=None):
        """(dL/dA (n,n), dL/dB (n,m), dL/dgamma (n,)) and their mu arrays."""
        n, m = inst.n, inst.m
        y = inst.y if y is None else y
        gA, gB, gg = np.empty((n, n)), np.empty((n, m)), np.empty(n)
        mA, mB, mg = np.empty((n, n)), np.empty((n, m)), np.empty(n)
        _check(self.L.orc_coef_grad(inst.N, n, m, _p(_d(inst.z)), _p(_d(y)), _p(gA),
                                    _p(gB) if m else None, _p(gg), _p(mA), _p(mB) if m else None,
                                    _p(mg)), "coef_grad")
        return (gA, gB, gg), (mA, mB, mg)

    # ---- Lagrangian derivatives for every scheme and boundary option --------
    # The definitions written out over the oracle's own _ex arrays:
    # L = sigma f + y^T c, grad_z L = sigma grad f + J^T y, (Hessian of L) v
    # from the lower-triangle Hessian, J v, and dL/dtheta = y^T dc/dtheta for
    # theta = (A, B, gamma), where the defects are linear in theta.  The sparse
    # products are scatter-adds in COO order (numpy bincount); each mu is the
    # same sum over the entries' magnitudes (the _ex arrays' own mu) times |y|
    # or |v|.  The paper's Sec. 8 names differentiable programming as future
    # work; the scheme and boundary rows follow Sec. 3 and Sec. 4.
    def lagrangian_ex(self, inst, scheme=0, bnd=0, sigma=None, y=None):
        """(L, mu_L); y has ncon entries (defect rows, then boundary rows)."""
        sigma = inst.sigma if sigma is None else sigma
        y = _d(inst.y if y is None else y)
        f, fmu = self.obj_ex(inst, scheme, bnd)
        c, cmu = self.cons_ex(inst, scheme, bnd)
        yc = math.fsum(y * c)
        return sigma * f + yc, abs(sigma) * fmu + float(np.abs(y) @ cmu)

    def lag_grad_ex(self, inst, scheme=0, bnd=0, sigma=None, y=None):
        """grad_z L (nvar entries, the layout of z) and its mu."""
        sigma = inst.sigma if sigma is None else sigma
        jr, jc, _, _ = self.pattern_ex(inst.N, inst.n, inst.m, scheme, bnd)
        return _grad_plus_jt_y(sigma, self.grad_ex(inst, scheme, bnd), self.jac_ex(inst, scheme, bnd),
                               jr, jc, _d(inst.y if y is None else y))

    def hvp_ex(self, inst, v, scheme=0, bnd=0, sigma=None, y=None):
        """(Hessian of L) v and its mu; the Hessian is the symmetric matrix
        whose lower triangle hess_ex holds."""
        _, _, hr, hc = self.pattern_ex(inst.N, inst.n, inst.m, scheme, bnd)
        return _sym_lower_mv(self.hess_ex(inst, scheme, bnd, sigma, y), hr, hc, _d(v))

    def jvp_ex(self, inst, v, scheme=0, bnd=0):
        """J v (ncon entries, the layout of c) and its mu."""
        jr, jc, _, _ = self.pattern_ex(inst.N, inst.n, inst.m, scheme, bnd)
        nc = self.sizes_ex(inst.N, inst.n, inst.m, scheme, bnd)["ncon"]
        return _coo_mv(self.jac_ex(inst, scheme, bnd), jr, jc, _d(v), nc)

    def coef_grad_ex(self, inst, scheme=0, bnd=0, y=None):
        """(dL/dA, dL/dB, dL/dgamma) and their mu arrays.  With S = sin X and
        Y the defect multipliers as an n x N matrix (boundary rows do not
        depend on the coefficients):
          trapezoidal  dc_ik/dA_ij = -h/2 (S_jk + S_j,k+1), dc_ik/dB_il = -h/2 (U_lk + U_l,k+1),
                       dc_ik/dgamma_i = -h/2 (X_ik X_pk + X_i,k+1 X_p,k+1);
          Euler        dc_ik/dA_ij = -h S_jk, dc_ik/dB_il = -h U_lk, dc_ik/dgamma_i = -h X_ik X_pk,
        with p = (i+1) mod n; the sums over k are matrix products."""
        N, n, m = inst.N, inst.n, inst.m
        y = _d(inst.y if y is None else y)
        NU = N + 1 if scheme == 0 else N
        X = _d(inst.z[:n * (N + 1)]).reshape(n, N + 1)
        U = _d(inst.z[n * (N + 1):]).reshape(m, NU)
        Y = y[:n * N].reshape(n, N)
        S = np.sin(X)
        P = X * X[(np.arange(n) + 1) % n]
        if scheme == 0:
            w = 0.5 * (1.0 / N)
            SA, UB, PG = S[:, :N] + S[:, 1:], U[:, :N] + U[:, 1:], P[:, :N] + P[:, 1:]
            SAm = np.abs(S[:, :N]) + np.abs(S[:, 1:])
            UBm = np.abs(U[:, :N]) + np.abs(U[:, 1:])
            PGm = np.abs(P[:, :N]) + np.abs(P[:, 1:])
        else:
            w = 1.0 / N
            SA, UB, PG = S[:, :N], U, P[:, :N]
            SAm, UBm, PGm = np.abs(SA), np.abs(UB), np.abs(PG)
        Ya = np.abs(Y)
        gA, mA = -w * (Y @ SA.T), w * (Ya @ SAm.T)
        gB, mB = -w * (Y @ UB.T), w * (Ya @ UBm.T)
        gg, mg = -w * np.sum(Y * PG, axis=1), w * np.sum(Ya * PGm, axis=1)
        return (gA, gB, gg), (mA, mB, mg)

    def coef_mixed_ex(self, inst, v, scheme=0, bnd=0, y=None):
        """The derivative of (dL/dA, dL/dB, dL/dgamma) along the direction v
        of z -- the mixed second derivatives d2L/(dtheta dz) contracted with
        v -- and their mu arrays.  With V_X and V_U the state and control
        parts of v (laid out as in z), C = cos X * V_X and Q_i = V_X,i X_p +
        X_i V_X,p (p = (i+1) mod n), it is coef_grad_ex with sin X, U and
        X_i X_p replaced by their derivatives along v, C, V_U and Q:
          trapezoidal  -h/2 sum_k y_ik (C_jk + C_j,k+1), -h/2 sum_k y_ik (V_U,lk + V_U,l,k+1),
                       -h/2 sum_k y_ik (Q_ik + Q_i,k+1);
          Euler        -h sum_k y_ik C_jk, -h sum_k y_ik V_U,lk, -h sum_k y_ik Q_ik.
        Boundary rows do not depend on the coefficients (paper Sec. 8 names
        differentiable programming as future work; the defects follow Sec. 3)."""
        N, n, m = inst.N, inst.n, inst.m
        y = _d(inst.y if y is None else y)
        v = _d(v)
        NU = N + 1 if scheme == 0 else N
        X = _d(inst.z[:n * (N + 1)]).reshape(n, N + 1)
        VX = v[:n * (N + 1)].reshape(n, N + 1)
        VU = v[n * (N + 1):].reshape(m, NU)
        Y = y[:n * N].reshape(n, N)
        p = (np.arange(n) + 1) % n
        C = np.cos(X) * VX
        Q = VX * X[p] + X * VX[p]
        Cm = np.abs(np.cos(X) * VX)
        Qm = np.abs(VX * X[p]) + np.abs(X * VX[p])
        if scheme == 0:
            w = 0.5 * (1.0 / N)
            CA, VB, QG = C[:, :N] + C[:, 1:], VU[:, :N] + VU[:, 1:], Q[:, :N] + Q[:, 1:]
            CAm = Cm[:, :N] + Cm[:, 1:]
            VBm = np.abs(VU[:, :N]) + np.abs(VU[:, 1:])
            QGm = Qm[:, :N] + Qm[:, 1:]
        else:
            w = 1.0 / N
            CA, VB, QG = C[:, :N], VU, Q[:, :N]
            CAm, VBm, QGm = Cm[:, :N], np.abs(VU), Qm[:, :N]
        Ya = np.abs(Y)
        gA, mA = -w * (Y @ CA.T), w * (Ya @ CAm.T)
        gB, mB = -w * (Y @ VB.T), w * (Ya @ VBm.T)
        gg, mg = -w * np.sum(Y * QG, axis=1), w * np.sum(Ya * QGm, axis=1)
        return (gA, gB, gg), (mA, mB, mg)

    def coef_adjoint_ex(self, inst, tA, tB, tg, scheme=0, bnd=0, y=None):
        """The adjoint of the coefficient gradient: for cotangents tA (n, n),
        tB (n, m), tg (n,) of (dL/dA, dL/dB, dL/dgamma), the gradients in z
        and in y of  t . dL/dtheta = sum tA * dL/dA + sum tB * dL/dB + tg . dL/dgamma,
        as ((gz, gy), (mu_z, mu_y)).  The defects are linear in theta, so
        t . dL/dtheta = sum_ik y_ik D_ik, D being the defects' theta part with
        theta := t: with Fb = tA sin X + tB U + tg * (X_i X_p) at each node
        (p = (i+1) mod n),
          trapezoidal  D_ik = -h/2 (Fb_ik + Fb_i,k+1),   Euler  D_ik = -h Fb_ik.
        Hence gy = D on the defect rows and 0 on the boundary rows (which do
        not depend on theta); and with the node multipliers Yt (trapezoidal
        -h/2 (y_i,k-1 + y_ik), Euler -h y_ik, the missing neighbours zero)
          gz on X_jk = cos X_jk (tA^T Yt)_jk + Yt_jk tg_j X_p(j)k + Yt_qk tg_q X_qk,
          gz on U_lk = (tB^T Yt)_lk,
        q = (j-1) mod n being the row whose bilinear partner is j.  Paper
        Sec. 8 names differentiable programming as future work; the defects
        follow Sec. 3."""
        N, n, m = inst.N, inst.n, inst.m
        y = _d(inst.y if y is None else y)
        tA, tB, tg = _d(tA).reshape(n, n), _d(tB).reshape(n, m), _d(tg).reshape(n)
        NU = N + 1 if scheme == 0 else N
        X = _d(inst.z[:n * (N + 1)]).reshape(n, N + 1)
        U = _d(inst.z[n * (N + 1):]).reshape(m, NU)
        Y = y[:n * N].reshape(n, N)
        p = (np.arange(n) + 1) % n
        q = (np.arange(n) - 1) % n
        S, C, P = np.sin(X), np.cos(X), X * X[p]
        aA, aB, ag = np.abs(tA), np.abs(tB), np.abs(tg)
        Fs, Fsm = tA @ S + tg[:, None] * P, aA @ np.abs(S) + ag[:, None] * np.abs(P)
        Fu, Fum = tB @ U, aB @ np.abs(U)
        Yt, Ya = np.zeros((n, N + 1)), np.zeros((n, N + 1))
        if scheme == 0:
            w = 0.5 * (1.0 / N)
            Fb, Fbm = Fs + Fu, Fsm + Fum
            D, Dm = -w * (Fb[:, :N] + Fb[:, 1:]), w * (Fbm[:, :N] + Fbm[:, 1:])
            Yt[:, :N] += Y
            Yt[:, 1:] += Y
            Ya[:, :N] += np.abs(Y)
            Ya[:, 1:] += np.abs(Y)
        else:
            w = 1.0 / N
            D, Dm = -w * (Fs[:, :N] + Fu), w * (Fsm[:, :N] + Fum)
            Yt[:, :N] = Y
            Ya[:, :N] = np.abs(Y)
        Yt, Ya = -w * Yt, w * Ya
        B1, B1m = Yt * tg[:, None] * X, Ya * ag[:, None] * np.abs(X)
        gX = C * (tA.T @ Yt) + Yt * tg[:, None] * X[p] + B1[q]
        mX = np.abs(C) * (aA.T @ Ya) + Ya * ag[:, None] * np.abs(X[p]) + B1m[q]
        gU, mU = tB.T @ Yt[:, :NU], aB.T @ Ya[:, :NU]
        nb = len(y) - n * N
        gz, mz = np.concatenate([gX.ravel(), gU.ravel()]), np.concatenate([mX.ravel(), mU.ravel()])
        gy, my = np.concatenate([D.ravel(), np.zeros(nb)]), np.concatenate([Dm.ravel(), np.zeros(nb)])
        return (gz, gy), (mz, my)

    # ---- schemes (0 trapezoidal, 1 forward Euler) and boundary rows --------
    def sizes_ex(self, N, n, m, scheme=0, bnd=0) -> dict:
        out = np.zeros(10, np.int64)
        _check(self.L.orc_sizes_ex(N, n, m, scheme, bnd, _p(out)), "sizes_ex")
        keys = ["nvar", "ncon", "nnzj", "nnzh", "dim", "npair", "T", "S", "NU", "nb"]
        return {k: int(v) for k, v in zip(keys, out)}

    def obj_ex(self, inst, scheme=0, bnd=0):
        out = np.zeros(2)
        _check(self.L.orc_obj_ex(inst.N, inst.n, inst.m, scheme, bnd, _p(_d(inst.q)), _p(_d(inst.r)),
                                 _p(_d(inst.z)), _p(out)), "obj_ex")
        return float(out[0]), float(out[1])

    def grad_ex(self, inst, scheme=0, bnd=0):
        s = self.sizes_ex(inst.N, inst.n, inst.m, scheme, bnd)
        g, mu = np.empty(s["nvar"]), np.empty(s["nvar"])
        _check(self.L.orc_grad_ex(inst.N, inst.n, inst.m, scheme, bnd, _p(_d(inst.q)),
                                  _p(_d(inst.r)), _p(_d(inst.z)), _p(g), _p(mu)), "grad_ex")
        return g, mu

    def cons_ex(self, inst, scheme=0, bnd=0):
        s = self.sizes_ex(inst.N, inst.n, inst.m, scheme, bnd)
        c, mu = np.empty(s["ncon"]), np.empty(s["ncon"])
        _check(self.L.orc_cons_ex(inst.N, inst.n, inst.m, scheme, bnd, _p(_d(inst.A)), _p(_d(inst.B)),
                                  _p(_d(inst.gamma)), _p(_d(inst.z)), _p(c), _p(mu)), "cons_ex")
        return c, mu

    def jac_ex(self, inst, scheme=0, bnd=0):
        s = self.sizes_ex(inst.N, inst.n, inst.m, scheme, bnd)
        v, mu = np.empty(s["nnzj"]), np.empty(s["nnzj"])
        _check(self.L.orc_jac_ex(inst.N, inst.n, inst.m, scheme, bnd, _p(_d(inst.A)), _p(_d(inst.B)),
                                 _p(_d(inst.gamma)), _p(_d(inst.z)), _p(v), _p(mu)), "jac_ex")
        return v, mu

    def hess_ex(self, inst, scheme=0, bnd=0, sigma=None, y=None):
        s = self.sizes_ex(inst.N, inst.n, inst.m, scheme, bnd)
        v, mu = np.empty(s["nnzh"]), np.empty(s["nnzh"])
        sigma = inst.sigma if sigma is None else sigma
        y = inst.y if y is None else y
        _check(self.L.orc_hess_ex(inst.N, inst.n, inst.m, scheme, bnd, _p(_d(inst.A)),
                                  _p(_d(inst.gamma)), _p(_d(inst.q)), _p(_d(inst.r)), _p(_d(inst.z)),
                                  _p(_d(y)), float(sigma), _p(v), _p(mu)), "hess_ex")
        return v, mu

    def pattern_ex(self, N, n, m, scheme=0, bnd=0):
        s = self.sizes_ex(N, n, m, scheme, bnd)
        jr, jc = np.empty(s["nnzj"], np.int32), np.empty(s["nnzj"], np.int32)
        hr, hc = np.empty(s["nnzh"], np.int32), np.empty(s["nnzh"], np.int32)
        _check(self.L.orc_pattern_ex(N, n, m, scheme, bnd, _p(jr), _p(jc), _p(hr), _p(hc)),
               "pattern_ex")
        return jr, jc, hr, hc

    def kkt_ex(self, N, n, m, scheme=0, bnd=0):
        s = self.sizes_ex(N, n, m, scheme, bnd)
        jr, jc, hr, hc = self.pattern_ex(N, n, m, scheme, bnd)
        rowptr = np.empty(s["dim"] + 1, np.int32)
        colind = np.empty(s["nnzh"] + s["nnzj"] + s["dim"], np.int32)
        perm_j = np.empty(s["nnzj"], np.int32)
        perm_h = np.empty(s["nnzh"], np.int32)
        nnzk = np.zeros(1, np.int64)
        _check(self.L.orc_kkt_generic(s["nvar"], s["ncon"], s["nnzj"], s["nnzh"], _p(jr), _p(jc),
                                      _p(hr), _p(hc), _p(rowptr), _p(colind), _p(perm_j),
                                      _p(perm_h), _p(nnzk)), "kkt_generic")
        return rowptr, colind[: int(nnzk[0])].copy(), perm_j, perm_h

    # ---- symmetric reordering of the KKT matrix ----

    def kkt_permute(self, rowptr, colind, perm_j, perm_h, order):
        """Lower CSR of P K P^T for order[new] = old, with the slot maps
        carried over: (rowptr2, colind2, perm_j2, perm_h2, diag2)."""
        dim = len(rowptr) - 1
        nnzk = int(rowptr[-1])
        rp2 = np.empty(dim + 1, np.int32)
        ci2 = np.empty(nnzk, np.int32)
        pj2 = np.empty(len(perm_j), np.int32)
        ph2 = np.empty(len(perm_h), np.int32)
        dg2 = np.empty(dim, np.int32)
        rowptr, colind, perm_j, perm_h, order = (_i32(a) for a in (rowptr, colind, perm_j, perm_h, order))
        _check(self.L.orc_kkt_permute(dim, _p(rowptr), _p(colind), len(perm_j), _p(perm_j),
                                      len(perm_h), _p(perm_h), _p(order), _p(rp2), _p(ci2),
                                      _p(pj2), _p(ph2), _p(dg2)), "kkt_permute")
        return rp2, ci2, pj2, ph2, dg2

    def assemble_mapped(self, nnzk, diag, perm_j, jvals, perm_h, hvals, reg=None):
        out = np.empty(int(nnzk))
        regp = None if reg is None else _d(reg)
        diag, perm_j, perm_h = _i32(diag), _i32(perm_j), _i32(perm_h)
        _check(self.L.orc_assemble_mapped(int(nnzk), len(diag), _p(diag), len(perm_j), _p(perm_j),
                                          _p(_d(jvals)), len(perm_h), _p(perm_h), _p(_d(hvals)),
                                          _p(regp), _p(out)), "assemble_mapped")
        return out

    # ---- quadrotor model (q: a synth.QuadInstance) ----

    def quad_sizes(self, N, bnd=1) -> dict:
        out = np.zeros(5, np.int64)
        _check(self.L.orc_quad_sizes(N, bnd, _p(out)), "quad_sizes")
        return {k: int(v) for k, v in zip(["nvar", "ncon", "nnzj", "nnzh", "dim"], out)}

    def quad_pattern(self, N, bnd=1):
        s = self.quad_sizes(N, bnd)
        jr, jc = np.empty(s["nnzj"], np.int32), np.empty(s["nnzj"], np.int32)
        hr, hc = np.empty(s["nnzh"], np.int32), np.empty(s["nnzh"], np.int32)
        _check(self.L.orc_quad_pattern(N, bnd, _p(jr), _p(jc), _p(hr), _p(hc)), "quad_pattern")
        return jr, jc, hr, hc

    def quad_kkt(self, N, bnd=1):
        s = self.quad_sizes(N, bnd)
        jr, jc, hr, hc = self.quad_pattern(N, bnd)
        rowptr = np.empty(s["dim"] + 1, np.int32)
        colind = np.empty(s["nnzh"] + s["nnzj"] + s["dim"], np.int32)
        perm_j = np.empty(s["nnzj"], np.int32)
        perm_h = np.empty(s["nnzh"], np.int32)
        nnzk = np.zeros(1, np.int64)
        _check(self.L.orc_kkt_generic(s["nvar"], s["ncon"], s["nnzj"], s["nnzh"], _p(jr), _p(jc),
                                      _p(hr), _p(hc), _p(rowptr), _p(colind), _p(perm_j),
                                      _p(perm_h), _p(nnzk)), "kkt_generic")
        return rowptr, colind[: int(nnzk[0])].copy(), perm_j, perm_h

    def quad_obj(self, q):
        out = np.zeros(2)
        _check(self.L.orc_quad_obj(q.N, q.r, _p(_d(q.z)), _p(out)), "quad_obj")
        return float(out[0]), float(out[1])

    def quad_grad(self, q):
        g, mu = np.empty(len(q.z)), np.empty(len(q.z))
        _check(self.L.orc_quad_grad(q.N, q.r, _p(_d(q.z)), _p(g), _p(mu)), "quad_grad")
        return g, mu

    def quad_cons(self, q):
        s = self.quad_sizes(q.N, q.bnd)
        c, mu = np.empty(s["ncon"]), np.empty(s["ncon"])
        _check(self.L.orc_quad_cons(q.N, q.bnd, q.g, _p(_d(q.z)), _p(c), _p(mu)), "quad_cons")
        return c, mu

    def quad_jac(self, q):
        s = self.quad_sizes(q.N, q.bnd)
        v, mu = np.empty(s["nnzj"]), np.empty(s["nnzj"])
        _check(self.L.orc_quad_jac(q.N, q.bnd, _p(_d(q.z)), _p(v), _p(mu)), "quad_jac")
        return v, mu

    def quad_hess(self, q, sigma=None, y=None):
        s = self.quad_sizes(q.N, q.bnd)
        v, mu = np.empty(s["nnzh"]), np.empty(s["nnzh"])
        sigma = q.sigma if sigma is None else sigma
        y = q.y if y is None else y
        _check(self.L.orc_quad_hess(q.N, q.r, _p(_d(q.z)), _p(_d(y)), float(sigma), _p(v), _p(mu)),
               "quad_hess")
        return v, mu

    # Lagrangian derivatives of the quadrotor model, written out over the
    # arrays above as for the synthetic family (the model has no coefficient
    # parameters, so there is no dL/dtheta).
    def quad_lagrangian(self, q, sigma=None, y=None):
        sigma = q.sigma if sigma is None else sigma
        y = _d(q.y if y is None else y)
        f, fmu = self.quad_obj(q)
        c, cmu = self.quad_cons(q)
        return sigma * f + math.fsum(y * c), abs(sigma) * fmu + float(np.abs(y) @ cmu)

    def quad_lag_grad(self, q, sigma=None, y=None):
        sigma = q.sigma if sigma is None else sigma
        jr, jc, _, _ = self.quad_pattern(q.N, q.bnd)
        return _grad_plus_jt_y(sigma, self.quad_grad(q), self.quad_jac(q), jr, jc,
                               _d(q.y if y is None else y))

    def quad_hvp(self, q, v, sigma=None, y=None):
        _, _, hr, hc = self.quad_pattern(q.N, q.bnd)
        return _sym_lower_mv(self.quad_hess(q, sigma, y), hr, hc, _d(v))

    def quad_jvp(self, q, v):
        jr, jc, _, _ = self.quad_pattern(q.N, q.bnd)
        return _coo_mv(self.quad_jac(q), jr, jc, _d(v), self.quad_sizes(q.N, q.bnd)["ncon"])


def _grad_plus_jt_y(sigma, grad, jac, jr, jc, y):
    """sigma grad f + J^T y from COO (values, mu) arrays, and its mu: a
    scatter-add over the entries in COO order."""
    g, gmu = grad
    jv, jmu = jac
    nv = len(g)
    out = sigma * g + np.bincount(jc, weights=jv * y[jr], minlength=nv)
    mu = abs(sigma) * gmu + np.bincount(jc, weights=jmu * np.abs(y[jr]), minlength=nv)
    return out, mu


def _sym_lower_mv(hess, hr, hc, v):
    """H v for the symmetric H whose lower triangle is the COO (values, mu)
    pair hess, and its mu."""
    hv, hmu = hess
    nv = len(v)
    off = hr != hc
    out = (np.bincount(hr, weights=hv * v[hc], minlength=nv)
           + np.bincount(hc[off], weights=hv[off] * v[hr[off]], minlength=nv))
    mu = (np.bincount(hr, weights=hmu * np.abs(v[hc]), minlength=nv)
          + np.bincount(hc[off], weights=hmu[off] * np.abs(v[hr[off]]), minlength=nv))
    return out, mu


def _coo_mv(jac, jr, jc, v, rows):
    """J v from COO (values, mu) arrays, and its mu."""
    jv, jmu = jac
    return (np.bincount(jr, weights=jv * v[jc], minlength=rows),
            np.bincount(jr, weights=jmu * np.abs(v[jc]), minlength=rows))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments")


DEFAULT = Oracle(LIB)

set_threads = DEFAULT.set_threads
get_threads = DEFAULT.get_threads
sizes = DEFAULT.sizes
obj = DEFAULT.obj
grad = DEFAULT.grad
cons = DEFAULT.cons
jac = DEFAULT.jac
hess = DEFAULT.hess
pattern = DEFAULT.pattern
kkt = DEFAULT.kkt
assemble = DEFAULT.assemble
lagrangian = DEFAULT.lagrangian
lag_grad = DEFAULT.lag_grad
hvp = DEFAULT.hvp
jvp = DEFAULT.jvp
coef_grad = DEFAULT.coef_grad
lagrangian_ex = DEFAULT.lagrangian_ex
lag_grad_ex = DEFAULT.lag_grad_ex
hvp_ex = DEFAULT.hvp_ex
jvp_ex = DEFAULT.jvp_ex
coef_grad_ex = DEFAULT.coef_grad_ex
coef_mixed_ex = DEFAULT.coef_mixed_ex
coef_adjoint_ex = DEFAULT.coef_adjoint_ex
sizes_ex = DEFAULT.sizes_ex
obj_ex = DEFAULT.obj_ex
grad_ex = DEFAULT.grad_ex
cons_ex = DEFAULT.cons_ex
jac_ex = DEFAULT.jac_ex
hess_ex = DEFAULT.hess_ex
pattern_ex = DEFAULT.pattern_ex
kkt_ex = DEFAULT.kkt_ex
kkt_permute = DEFAULT.kkt_permute
assemble_mapped = DEFAULT.assemble_mapped
quad_sizes = DEFAULT.quad_sizes
quad_pattern = DEFAULT.quad_pattern
quad_kkt = DEFAULT.quad_kkt
quad_obj = DEFAULT.quad_obj
quad_grad = DEFAULT.quad_grad
quad_cons = DEFAULT.quad_cons
quad_jac = DEFAULT.quad_jac
quad_hess = DEFAULT.quad_hess
quad_lagrangian = DEFAULT.quad_lagrangian
quad_lag_grad = DEFAULT.quad_lag_grad
quad_hvp = DEFAULT.quad_hvp
quad_jvp = DEFAULT.quad_jvp


def build_variant(src_text: str, out_path: str) -> "Oracle":
    """Compile an edited copy of the oracle source (mutation tests) and load it."""
    c_path = out_path[:-3] + ".c" if out_path.endswith(".so") else out_path + ".c"
    with open(c_path, "w") as fh:
        fh.write(src_text)
    subprocess.check_call(["gcc", *CFLAGS, c_path, "-o", out_path, "-lm"])
    return Oracle(out_path)
