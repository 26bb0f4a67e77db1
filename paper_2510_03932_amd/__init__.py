"""MI355X (gfx950) evaluation of a trapezoidal direct-transcription NLP.

Thin Python binding over the C ABI in ``include/ocp_eval.h`` (``libocpeval.so``
built in-tree by ``python -m paper_2510_03932_amd.build``).  Argument
marshalling only: every evaluation runs in the library's HIP kernels on the
caller's current torch stream; PyTorch only provides device memory and
streams.  There is no CPU fallback: if the library is missing, every call
raises.

    prob = Problem(N, n, m, A, B, gamma, q, r)      # coefficients: host arrays
    g = prob.grad(z); c = prob.cons(z); jv = prob.jac(z)
    hv = prob.hess(z, y, sigma)
    rowptr, colind, perm_j, perm_h = kkt_pattern(N, n, m)   # host, once
    kkt = prob.assemble_kkt(perm_j_dev, perm_h_dev, rowptr_dev, jv, hv, reg)
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libocpeval.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ocp_eval.h")

OCP_OK, OCP_ERR_ARG, OCP_ERR_OVERFLOW, OCP_ERR_HIP, OCP_ERR_ALLOC = 0, 1, 2, 3, 4
MAX_DIM = 32


class OcpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Sizes(ctypes.Structure):
    _fields_ = [("nvar", ctypes.c_int64), ("ncon", ctypes.c_int64), ("nnzj", ctypes.c_int64),
                ("nnzh", ctypes.c_int64), ("nnzk", ctypes.c_int64), ("dim", ctypes.c_int64),
                ("npair", ctypes.c_int32), ("T", ctypes.c_int32), ("S", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded C library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OcpError(OCP_ERR_HIP, f"HIP library not built: {LIB_PATH} is missing "
                                        "(run python -m paper_2510_03932_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
        L.ocp_sizes.argtypes = [i64, i32, i32, ctypes.POINTER(Sizes)]
        L.ocp_build_pattern.argtypes = [i64, i32, i32, vp, vp, vp, vp]
        L.ocp_build_kkt.argtypes = [i64, i32, i32, vp, vp, vp, vp]
        L.ocp_create.argtypes = [i64, i32, i32, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.ocp_destroy.argtypes = [vp]
        L.ocp_destroy.restype = None
        L.ocp_problem_sizes.argtypes = [vp, ctypes.POINTER(Sizes)]
        L.ocp_eval_obj.argtypes = [vp, vp, vp, vp]
        L.ocp_eval_grad.argtypes = [vp, vp, vp, vp]
        L.ocp_eval_cons.argtypes = [vp, vp, vp, vp]
        L.ocp_eval_jac.argtypes = [vp, vp, vp, vp]
        L.ocp_eval_hess.argtypes = [vp, vp, vp, dbl, vp, vp]
        L.ocp_assemble_kkt.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ocp_last_error.restype = ctypes.c_char_p
        missing = [name for name in exported_names() if not hasattr(L, name)]
        if missing:
            raise OcpError(OCP_ERR_HIP, f"{LIB_PATH} lacks {missing}: rebuild it")
        _lib = L
    return _lib


def exported_names() -> list[str]:
    """Entry points declared in the public header."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(ocp_\w+)\s*\(", text, re.M)))


def _check(rc: int, what: str):
    if rc != OCP_OK:
        msg = lib().ocp_last_error().decode()
        raise OcpError(rc, f"{what}: {msg}")


def _hp(a: np.ndarray | None):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def sizes(N: int, n: int, m: int) -> dict:
    s = Sizes()
    _check(lib().ocp_sizes(N, n, m, ctypes.byref(s)), "ocp_sizes")
    return s.as_dict()


def pattern(N: int, n: int, m: int, jac: bool = True, hess: bool = True):
    """Host COO patterns (jrow, jcol, hrow, hcol), int32; skipped parts are None."""
    s = sizes(N, n, m)
    jrow = np.empty(s["nnzj"], np.int32) if jac else None
    jcol = np.empty(s["nnzj"], np.int32) if jac else None
    hrow = np.empty(s["nnzh"], np.int32) if hess else None
    hcol = np.empty(s["nnzh"], np.int32) if hess else None
    _check(lib().ocp_build_pattern(N, n, m, _hp(jrow), _hp(jcol), _hp(hrow), _hp(hcol)),
           "ocp_build_pattern")
    return jrow, jcol, hrow, hcol


def kkt_pattern(N: int, n: int, m: int, rowptr=True, colind=True, perm_j=True, perm_h=True):
    """Host KKT structure (rowptr, colind, perm_j, perm_h), int32; skipped parts are None."""
    s = sizes(N, n, m)
    rp = np.empty(s["dim"] + 1, np.int32) if rowptr else None
    ci = np.empty(s["nnzk"], np.int32) if colind else None
    pj = np.empty(s["nnzj"], np.int32) if perm_j else None
    ph = np.empty(s["nnzh"], np.int32) if perm_h else None
    _check(lib().ocp_build_kkt(N, n, m, _hp(rp), _hp(ci), _hp(pj), _hp(ph)), "ocp_build_kkt")
    return rp, ci, pj, ph


def _torch():
    import torch
    return torch


class Problem:
    """One transcribed OCP instance bound to a GPU (the current torch device)."""

    def __init__(self, N, n, m, A, B, gamma, q, r, device=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise OcpError(OCP_ERR_HIP, "no GPU visible: this library runs only on gfx950 devices")
        self.N, self.n, self.m = int(N), int(n), int(m)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        f64 = lambda a, shape: np.ascontiguousarray(np.asarray(a, np.float64).reshape(shape))
        A = f64(A, (n, n))
        B = f64(B, (n, m)) if m else np.zeros((n, 0))
        gamma, q = f64(gamma, (n,)), f64(q, (n,))
        r = f64(r, (m,)) if m else np.zeros(0)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().ocp_create(self.N, self.n, self.m, _hp(A), _hp(B) if m else None,
                                    _hp(gamma), _hp(q), _hp(r) if m else None, ctypes.byref(h)),
                   "ocp_create")
        self._h = h
        s = Sizes()
        _check(lib().ocp_problem_sizes(self._h, ctypes.byref(s)), "ocp_problem_sizes")
        self.sizes = s.as_dict()

    @classmethod
    def from_instance(cls, inst, device=None):
        return cls(inst.N, inst.n, inst.m, inst.A, inst.B, inst.gamma, inst.q, inst.r, device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ocp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- marshalling helpers ---------------------------------------------------
    def _dev(self, t, numel, dtype, what):
        torch = _torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{what}: expected a torch tensor on {self.device}")
        if t.device != self.device:
            raise ValueError(f"{what}: tensor is on {t.device}, problem on {self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{what}: dtype {t.dtype}, expected {dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{what}: tensor must be contiguous")
        if t.numel() != numel:
            raise ValueError(f"{what}: {t.numel()} elements, expected {numel}")
        return ctypes.c_void_p(t.data_ptr())

    def _out(self, out, numel, what):
        torch = _torch()
        if out is None:
            out = torch.empty(numel, dtype=torch.float64, device=self.device)
        return out, self._dev(out, numel, torch.float64, what)

    def _stream(self):
        return ctypes.c_void_p(_torch().cuda.current_stream(self.device).cuda_stream)

    # -- evaluations -------------------------------------------------------------
    def obj(self, z, out=None):
        torch = _torch()
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        out, op = self._out(out, 1, "obj")
        _check(lib().ocp_eval_obj(self._h, zp, op, self._stream()), "ocp_eval_obj")
        return out

    def grad(self, z, out=None):
        torch = _torch()
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        out, op = self._out(out, self.sizes["nvar"], "grad")
        _check(lib().ocp_eval_grad(self._h, zp, op, self._stream()), "ocp_eval_grad")
        return out

    def cons(self, z, out=None):
        torch = _torch()
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        out, op = self._out(out, self.sizes["ncon"], "cons")
        _check(lib().ocp_eval_cons(self._h, zp, op, self._stream()), "ocp_eval_cons")
        return out

    def jac(self, z, out=None):
        torch = _torch()
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        out, op = self._out(out, self.sizes["nnzj"], "jac")
        _check(lib().ocp_eval_jac(self._h, zp, op, self._stream()), "ocp_eval_jac")
        return out

    def hess(self, z, y, sigma=1.0, out=None):
        torch = _torch()
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        yp = self._dev(y, self.sizes["ncon"], torch.float64, "y")
        out, op = self._out(out, self.sizes["nnzh"], "hess")
        _check(lib().ocp_eval_hess(self._h, zp, yp, float(sigma), op, self._stream()),
               "ocp_eval_hess")
        return out

    def assemble_kkt(self, perm_j, perm_h, rowptr, jvals, hvals, reg=None, out=None):
        torch = _torch()
        s = self.sizes
        pj = self._dev(perm_j, s["nnzj"], torch.int32, "perm_j")
        ph = self._dev(perm_h, s["nnzh"], torch.int32, "perm_h")
        rp = self._dev(rowptr, s["dim"] + 1, torch.int32, "rowptr")
        jp = self._dev(jvals, s["nnzj"], torch.float64, "jvals")
        hp = self._dev(hvals, s["nnzh"], torch.float64, "hvals")
        gp = None if reg is None else self._dev(reg, s["dim"], torch.float64, "reg")
        out, op = self._out(out, s["nnzk"], "kkt")
        _check(lib().ocp_assemble_kkt(self._h, pj, ph, rp, jp, hp, gp, op, self._stream()),
               "ocp_assemble_kkt")
        return out
