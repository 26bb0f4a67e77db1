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


class Options(ctypes.Structure):
    """Transcription options: scheme 0 trapezoidal / 1 forward Euler; boundary
    0 none / 1 initial-state rows / 2 initial- and final-state rows."""
    _fields_ = [("scheme", ctypes.c_int32), ("boundary", ctypes.c_int32)]


SCHEMES = {"trapezoidal": 0, "euler": 1}


def _opts(scheme=0, boundary=0):
    scheme = SCHEMES.get(scheme, scheme) if isinstance(scheme, str) else scheme
    return Options(int(scheme), int(boundary))


class BatchConfig(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("pair", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("order", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


EVAL_JAC, EVAL_HESS, EVAL_OBJ, EVAL_GRAD, EVAL_CONS, EVAL_KKT = 1, 2, 4, 8, 16, 32
EVAL_ALL = 63


class BatchIO(ctypes.Structure):
    """ocp_batch_io: the device arrays of one batched evaluation."""
    _fields_ = [("z", ctypes.c_void_p), ("y", ctypes.c_void_p), ("reg", ctypes.c_void_p),
                ("sigma", ctypes.c_double), ("obj", ctypes.c_void_p), ("grad", ctypes.c_void_p),
                ("cons", ctypes.c_void_p), ("jac", ctypes.c_void_p), ("hess", ctypes.c_void_p),
                ("kkt", ctypes.c_void_p)]


AUTOTUNE_SHAPES = [{"block": b, "pair": p, "wgs_per_cu": w, "order": o}
                   for b in (128, 256) for p in (0, 1) for w in (1, 2, 4, 8, 16, 32, 0) for o in (0, 1)]
MODES = {"persistent": 0, "per_instance": 1}

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
        L.ocp_sizes_ex.argtypes = [i64, i32, i32, ctypes.POINTER(Options), ctypes.POINTER(Sizes)]
        L.ocp_build_pattern_ex.argtypes = [i64, i32, i32, ctypes.POINTER(Options), vp, vp, vp, vp]
        L.ocp_build_kkt_ex.argtypes = [i64, i32, i32, ctypes.POINTER(Options), vp, vp, vp, vp]
        L.ocp_create_ex.argtypes = [i64, i32, i32, ctypes.POINTER(Options), vp, vp, vp, vp, vp,
                                    ctypes.POINTER(vp)]
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
        L.ocp_quad_sizes.argtypes = [i64, i32, ctypes.POINTER(Sizes)]
        L.ocp_stage_order.argtypes = [i64, i32, i32, ctypes.POINTER(Options), vp]
        L.ocp_quad_stage_order.argtypes = [i64, i32, vp]
        L.ocp_kkt_permute.argtypes = [i64, vp, vp, i64, vp, i64, vp, vp, vp, vp, vp, vp, vp]
        L.ocp_assemble_kkt_mapped.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ocp_mapped_plan_size.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.ocp_mapped_plan.argtypes = [vp, vp, vp, vp, vp, vp]
        L.ocp_eval_kkt.argtypes = [vp, vp, vp, dbl, vp, vp, vp]
        L.ocp_quad_pattern.argtypes = [i64, i32, vp, vp, vp, vp]
        L.ocp_quad_kkt.argtypes = [i64, i32, vp, vp, vp, vp]
        L.ocp_quad_create.argtypes = [i64, i32, dbl, dbl, ctypes.POINTER(vp)]
        L.ocp_set_coefficients.argtypes = [vp, vp, vp, vp, vp]
        L.ocp_eval_lagrangian.argtypes = [vp, vp, vp, dbl, vp, vp]
        L.ocp_eval_lag_grad.argtypes = [vp, vp, vp, dbl, vp, vp]
        L.ocp_eval_hvp.argtypes = [vp, vp, vp, dbl, vp, vp, vp]
        L.ocp_eval_jvp.argtypes = [vp, vp, vp, vp, vp]
        L.ocp_eval_coef_grad.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.ocp_eval_coef_grad_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.ocp_eval_coef_mixed.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.ocp_eval_coef_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ocp_eval_lagrangian_backward.argtypes = [vp, vp, vp, dbl, vp, vp, vp, vp, vp, vp, vp]
        L.ocp_batch_create.argtypes = [i32, vp, i32, i32, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.ocp_batch_destroy.argtypes = [vp]
        L.ocp_batch_destroy.restype = None
        L.ocp_batch_offsets.argtypes = [vp, vp, vp, vp, vp]
        L.ocp_batch_get_config.argtypes = [vp, ctypes.POINTER(BatchConfig)]
        L.ocp_batch_set_config.argtypes = [vp, ctypes.POINTER(BatchConfig)]
        L.ocp_batch_eval.argtypes = [vp, i32, i32, vp, vp, dbl, vp, vp, vp]
        L.ocp_batch_graph_create.argtypes = [vp, i32, i32, vp, vp, dbl, vp, vp, ctypes.POINTER(vp)]
        L.ocp_graph_launch.argtypes = [vp, vp]
        L.ocp_graph_destroy.argtypes = [vp]
        L.ocp_graph_destroy.restype = None
        L.ocp_batch_autotune.argtypes = [vp, i32, vp, vp, dbl, vp, vp, i32, vp,
                                         ctypes.POINTER(BatchConfig), ctypes.POINTER(ctypes.c_float),
                                         vp]
        L.ocp_batch_create_ex.argtypes = [i32, vp, i32, i32, ctypes.POINTER(Options), vp, vp, vp, vp, vp,
                                          ctypes.POINTER(vp)]
        L.ocp_batch_offsets_ex.argtypes = [vp, vp, vp]
        L.ocp_batch_prepare.argtypes = [vp, i32]
        L.ocp_batch_eval_io.argtypes = [vp, i32, i32, ctypes.POINTER(BatchIO), vp]
        L.ocp_batch_graph_create_io.argtypes = [vp, i32, i32, ctypes.POINTER(BatchIO), ctypes.POINTER(vp)]
        L.ocp_batch_autotune_io.argtypes = [vp, i32, ctypes.POINTER(BatchIO), i32, vp,
                                            ctypes.POINTER(BatchConfig), ctypes.POINTER(ctypes.c_float), vp]
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


def sizes(N: int, n: int, m: int, scheme=0, boundary=0) -> dict:
    s = Sizes()
    o = _opts(scheme, boundary)
    _check(lib().ocp_sizes_ex(N, n, m, ctypes.byref(o), ctypes.byref(s)), "ocp_sizes")
    return s.as_dict()


def pattern(N: int, n: int, m: int, jac: bool = True, hess: bool = True, scheme=0, boundary=0):
    """Host COO patterns (jrow, jcol, hrow, hcol), int32; skipped parts are None."""
    s = sizes(N, n, m, scheme, boundary)
    jrow = np.empty(s["nnzj"], np.int32) if jac else None
    jcol = np.empty(s["nnzj"], np.int32) if jac else None
    hrow = np.empty(s["nnzh"], np.int32) if hess else None
    hcol = np.empty(s["nnzh"], np.int32) if hess else None
    o = _opts(scheme, boundary)
    _check(lib().ocp_build_pattern_ex(N, n, m, ctypes.byref(o), _hp(jrow), _hp(jcol), _hp(hrow),
                                      _hp(hcol)), "ocp_build_pattern")
    return jrow, jcol, hrow, hcol


def kkt_pattern(N: int, n: int, m: int, rowptr=True, colind=True, perm_j=True, perm_h=True,
                scheme=0, boundary=0):
    """Host KKT structure (rowptr, colind, perm_j, perm_h), int32; skipped parts are None."""
    s = sizes(N, n, m, scheme, boundary)
    rp = np.empty(s["dim"] + 1, np.int32) if rowptr else None
    ci = np.empty(s["nnzk"], np.int32) if colind else None
    pj = np.empty(s["nnzj"], np.int32) if perm_j else None
    ph = np.empty(s["nnzh"], np.int32) if perm_h else None
    o = _opts(scheme, boundary)
    _check(lib().ocp_build_kkt_ex(N, n, m, ctypes.byref(o), _hp(rp), _hp(ci), _hp(pj), _hp(ph)),
           "ocp_build_kkt")
    return rp, ci, pj, ph


# ---- symmetric reordering of the KKT matrix --------------------------------------

def stage_order(N: int, n: int, m: int, scheme=0, boundary=0) -> np.ndarray:
    """Node-grouped fill-reducing ordering (order[new] = old), int32."""
    s = sizes(N, n, m, scheme, boundary)
    order = np.empty(s["dim"], np.int32)
    o = _opts(scheme, boundary)
    _check(lib().ocp_stage_order(int(N), int(n), int(m), ctypes.byref(o), _hp(order)), "ocp_stage_order")
    return order


def quad_stage_order(N: int, boundary: int = 1) -> np.ndarray:
    s = quad_sizes(N, boundary)
    order = np.empty(s["dim"], np.int32)
    _check(lib().ocp_quad_stage_order(int(N), int(boundary), _hp(order)), "ocp_quad_stage_order")
    return order


def kkt_permute(rowptr, colind, perm_j, perm_h, order):
    """Lower CSR of P K P^T with the slot maps carried over:
    (rowptr2, colind2, perm_j2, perm_h2, diag2), all int32 host arrays."""
    i32 = lambda a: np.ascontiguousarray(a, np.int32)
    rowptr, colind, perm_j, perm_h, order = (i32(a) for a in (rowptr, colind, perm_j, perm_h, order))
    dim = len(rowptr) - 1
    if len(order) != dim:
        raise ValueError(f"order has {len(order)} entries, the KKT matrix {dim} rows")
    nnzk = int(rowptr[-1])
    rp2 = np.empty(dim + 1, np.int32)
    ci2 = np.empty(nnzk, np.int32)
    pj2 = np.empty(len(perm_j), np.int32)
    ph2 = np.empty(len(perm_h), np.int32)
    dg2 = np.empty(dim, np.int32)
    _check(lib().ocp_kkt_permute(dim, _hp(rowptr), _hp(colind), len(perm_j), _hp(perm_j), len(perm_h),
                                 _hp(perm_h), _hp(order), _hp(rp2), _hp(ci2), _hp(pj2), _hp(ph2),
                                 _hp(dg2)), "ocp_kkt_permute")
    return rp2, ci2, pj2, ph2, dg2


# ---- the quadrotor model (paper Appendix A) ----------------------------------

QUAD_G, QUAD_R = 9.8, 0.1  # the paper's gravity and control weight


def quad_sizes(N: int, boundary: int = 1) -> dict:
    out = Sizes()
    _check(lib().ocp_quad_sizes(int(N), int(boundary), ctypes.byref(out)), "ocp_quad_sizes")
    return out.as_dict()


def quad_pattern(N: int, boundary: int = 1, jac: bool = True, hess: bool = True):
    """Host COO patterns (jrow, jcol, hrow, hcol) of the quadrotor NLP, int32."""
    s = quad_sizes(N, boundary)
    jr = np.empty(s["nnzj"], np.int32) if jac else None
    jc = np.empty(s["nnzj"], np.int32) if jac else None
    hr = np.empty(s["nnzh"], np.int32) if hess else None
    hc = np.empty(s["nnzh"], np.int32) if hess else None
    _check(lib().ocp_quad_pattern(int(N), int(boundary), _hp(jr), _hp(jc), _hp(hr), _hp(hc)),
           "ocp_quad_pattern")
    return jr, jc, hr, hc


def quad_kkt_pattern(N: int, boundary: int = 1, rowptr=True, colind=True, perm_j=True, perm_h=True):
    """Host KKT structure (rowptr, colind, perm_j, perm_h) of the quadrotor NLP."""
    s = quad_sizes(N, boundary)
    rp = np.empty(s["dim"] + 1, np.int32) if rowptr else None
    ci = np.empty(s["nnzk"], np.int32) if colind else None
    pj = np.empty(s["nnzj"], np.int32) if perm_j else None
    ph = np.empty(s["nnzh"], np.int32) if perm_h else None
    _check(lib().ocp_quad_kkt(int(N), int(boundary), _hp(rp), _hp(ci), _hp(pj), _hp(ph)),
           "ocp_quad_kkt")
    return rp, ci, pj, ph


def _torch():
    import torch
    return torch


def _raw_stream(device):
    """The raw HIP stream of torch's current stream on `device` (a
    torch.device with an index), as a ctypes pointer.  torch's internal query
    returns the handle without building a Stream object, which saves about
    2 us of host time per library call; the public call is the fallback."""
    torch = _torch()
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None and device.index is not None:
        return ctypes.c_void_p(raw(device.index))
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Problem:
    """One transcribed OCP instance bound to a GPU (the current torch device)."""

    def __init__(self, N, n, m, A, B, gamma, q, r, device=None, scheme=0, boundary=0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise OcpError(OCP_ERR_HIP, "no GPU visible: this library runs only on gfx950 devices")
        self.N, self.n, self.m = int(N), int(n), int(m)
        self.options = _opts(scheme, boundary)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        f64 = lambda a, shape: np.ascontiguousarray(np.asarray(a, np.float64).reshape(shape))
        A = f64(A, (n, n))
        B = f64(B, (n, m)) if m else np.zeros((n, 0))
        gamma, q = f64(gamma, (n,)), f64(q, (n,))
        r = f64(r, (m,)) if m else np.zeros(0)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().ocp_create_ex(self.N, self.n, self.m, ctypes.byref(self.options), _hp(A),
                                       _hp(B) if m else None, _hp(gamma), _hp(q),
                                       _hp(r) if m else None, ctypes.byref(h)), "ocp_create")
        self._h = h
        s = Sizes()
        _check(lib().ocp_problem_sizes(self._h, ctypes.byref(s)), "ocp_problem_sizes")
        self.sizes = s.as_dict()

    @classmethod
    def from_instance(cls, inst, device=None):
        return cls(inst.N, inst.n, inst.m, inst.A, inst.B, inst.gamma, inst.q, inst.r, device,
                   scheme=getattr(inst, "scheme", 0), boundary=getattr(inst, "bnd", 0))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ocp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the problem's sparsity structure (host) ----------------------------------
    def pattern(self, jac: bool = True, hess: bool = True):
        """This problem's COO patterns (jrow, jcol, hrow, hcol): the module's
        pattern() for the problem's sizes, scheme and boundary option."""
        return pattern(self.N, self.n, self.m, jac, hess, self.options.scheme, self.options.boundary)

    def kkt_pattern(self, rowptr=True, colind=True, perm_j=True, perm_h=True):
        """This problem's KKT structure (rowptr, colind, perm_j, perm_h): the
        module's kkt_pattern() for the problem's sizes and options."""
        return kkt_pattern(self.N, self.n, self.m, rowptr, colind, perm_j, perm_h, self.options.scheme,
                           self.options.boundary)

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
        return _raw_stream(self.device)

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

    def eval_kkt(self, z, y, sigma=1.0, reg=None, out=None):
        """Jacobian and Hessian evaluated straight into the KKT values (the
        layout of kkt_pattern), the fused form of jac + hess + assemble_kkt."""
        torch = _torch()
        s = self.sizes
        zp = self._dev(z, s["nvar"], torch.float64, "z")
        yp = self._dev(y, s["ncon"], torch.float64, "y")
        gp = None if reg is None else self._dev(reg, s["dim"], torch.float64, "reg")
        out, op = self._out(out, s["nnzk"], "kkt")
        _check(lib().ocp_eval_kkt(self._h, zp, yp, float(sigma), gp, op, self._stream()), "ocp_eval_kkt")
        return out

    def mapped_plan(self, perm_j, perm_h, diag):
        """Per-tile CSR ranges of slot maps, for assemble_kkt_mapped (int32 device tensor)."""
        torch = _torch()
        s = self.sizes
        pj = self._dev(perm_j, s["nnzj"], torch.int32, "perm_j")
        ph = self._dev(perm_h, s["nnzh"], torch.int32, "perm_h")
        dg = self._dev(diag, s["dim"], torch.int32, "diag")
        cnt = ctypes.c_int64()
        _check(lib().ocp_mapped_plan_size(self._h, ctypes.byref(cnt)), "ocp_mapped_plan_size")
        plan = torch.empty(cnt.value, dtype=torch.int32, device=self.device)
        _check(lib().ocp_mapped_plan(self._h, pj, ph, dg, ctypes.c_void_p(plan.data_ptr()), self._stream()),
               "ocp_mapped_plan")
        return plan

    def assemble_kkt_mapped(self, perm_j, perm_h, diag, jvals, hvals, reg=None, out=None, plan=None):
        """Assembly through slot maps alone (any ordering, e.g. from kkt_permute);
        plan (from mapped_plan for the same maps) skips a pass over the maps."""
        torch = _torch()
        s = self.sizes
        pj = self._dev(perm_j, s["nnzj"], torch.int32, "perm_j")
        ph = self._dev(perm_h, s["nnzh"], torch.int32, "perm_h")
        dg = self._dev(diag, s["dim"], torch.int32, "diag")
        jp = self._dev(jvals, s["nnzj"], torch.float64, "jvals")
        hp = self._dev(hvals, s["nnzh"], torch.float64, "hvals")
        gp = None if reg is None else self._dev(reg, s["dim"], torch.float64, "reg")
        pl = None
        if plan is not None:
            cnt = ctypes.c_int64()
            _check(lib().ocp_mapped_plan_size(self._h, ctypes.byref(cnt)), "ocp_mapped_plan_size")
            pl = self._dev(plan, cnt.value, torch.int32, "plan")
        out, op = self._out(out, s["nnzk"], "kkt")
        _check(lib().ocp_assemble_kkt_mapped(self._h, pj, ph, dg, pl, jp, hp, gp, op, self._stream()),
               "ocp_assemble_kkt_mapped")
        return out

    # -- Lagrangian derivatives ---------------------------------------------------
    def set_coefficients(self, A, B, gamma):
        """Copy device tensors A (n, n), B (n, m), gamma (n,) into the handle
        (stream-ordered on the current stream)."""
        torch = _torch()
        n, m = self.n, self.m
        # the contiguous copies stay referenced until the copies are queued:
        # a freed temporary could be handed to the next temporary's copy kernel
        A, gamma = A.contiguous(), gamma.contiguous()
        B = B.contiguous() if m else None
        Ap = self._dev(A, n * n, torch.float64, "A")
        Bp = self._dev(B, n * m, torch.float64, "B") if m else None
        gp = self._dev(gamma, n, torch.float64, "gamma")
        _check(lib().ocp_set_coefficients(self._h, Ap, Bp, gp, self._stream()), "ocp_set_coefficients")
        self._coef_key = None  # an upload the autograd functions did not make

    def lagrangian(self, z, y, sigma=1.0, out=None):
        torch = _torch()
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        yp = self._dev(y, self.sizes["ncon"], torch.float64, "y")
        out, op = self._out(out, 1, "L")
        _check(lib().ocp_eval_lagrangian(self._h, zp, yp, float(sigma), op, self._stream()),
               "ocp_eval_lagrangian")
        return out

    def lag_grad(self, z, y, sigma=1.0, out=None):
        torch = _torch()
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        yp = self._dev(y, self.sizes["ncon"], torch.float64, "y")
        out, op = self._out(out, self.sizes["nvar"], "grad_z L")
        _check(lib().ocp_eval_lag_grad(self._h, zp, yp, float(sigma), op, self._stream()),
               "ocp_eval_lag_grad")
        return out

    def hvp(self, z, y, v, sigma=1.0, out=None):
        torch = _torch()
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        yp = self._dev(y, self.sizes["ncon"], torch.float64, "y")
        vp = self._dev(v, self.sizes["nvar"], torch.float64, "v")
        out, op = self._out(out, self.sizes["nvar"], "H v")
        _check(lib().ocp_eval_hvp(self._h, zp, yp, float(sigma), vp, op, self._stream()),
               "ocp_eval_hvp")
        return out

    def jvp(self, z, v, out=None):
        torch = _torch()
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        vp = self._dev(v, self.sizes["nvar"], torch.float64, "v")
        out, op = self._out(out, self.sizes["ncon"], "J v")
        _check(lib().ocp_eval_jvp(self._h, zp, vp, op, self._stream()), "ocp_eval_jvp")
        return out

    def coef_grad(self, z, y, noalloc=False, out=None):
        """(dL/dA (n, n), dL/dB (n, m), dL/dgamma (n,)) as device tensors.
        noalloc=True calls the allocation-free entry point (its partial sums
        in the library's fixed scratch array instead of the handle's
        workspace; bitwise the same result).  out: optional (gA, gB, gamma)
        contiguous float64 tensors of n * n, n * m and n elements on the
        problem's device, written in place and returned."""
        torch = _torch()
        n, m = self.n, self.m
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        yp = self._dev(y, self.sizes["ncon"], torch.float64, "y")
        if out is None:
            f64 = dict(dtype=torch.float64, device=self.device)
            gA, gB, gg = torch.empty(n, n, **f64), torch.empty(n, m, **f64), torch.empty(n, **f64)
        else:
            gA, gB, gg = out
            self._dev(gA, n * n, torch.float64, "out[0]")
            self._dev(gB, n * m, torch.float64, "out[1]")
            self._dev(gg, n, torch.float64, "out[2]")
        fn = "ocp_eval_coef_grad_noalloc" if noalloc else "ocp_eval_coef_grad"
        _check(getattr(lib(), fn)(self._h, zp, yp, ctypes.c_void_p(gA.data_ptr()),
                                  ctypes.c_void_p(gB.data_ptr()) if m else None,
                                  ctypes.c_void_p(gg.data_ptr()), self._stream()), fn)
        return gA, gB, gg

    def coef_mixed(self, z, y, v, out=None):
        """The derivative of coef_grad(z, y) along the direction v of z (nvar
        doubles): d/d(A, B, gamma) of v^T grad_z L, as (n, n), (n, m) and (n,)
        device tensors (or written into out, as for coef_grad)."""
        torch = _torch()
        n, m = self.n, self.m
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        yp = self._dev(y, self.sizes["ncon"], torch.float64, "y")
        vp_ = self._dev(v, self.sizes["nvar"], torch.float64, "v")
        if out is None:
            f64 = dict(dtype=torch.float64, device=self.device)
            gA, gB, gg = torch.empty(n, n, **f64), torch.empty(n, m, **f64), torch.empty(n, **f64)
        else:
            gA, gB, gg = out
            self._dev(gA, n * n, torch.float64, "out[0]")
            self._dev(gB, n * m, torch.float64, "out[1]")
            self._dev(gg, n, torch.float64, "out[2]")
        _check(lib().ocp_eval_coef_mixed(self._h, zp, yp, vp_, ctypes.c_void_p(gA.data_ptr()),
                                          ctypes.c_void_p(gB.data_ptr()) if m else None,
                                          ctypes.c_void_p(gg.data_ptr()), self._stream()),
               "ocp_eval_coef_mixed")
        return gA, gB, gg

    def lagrangian_backward(self, z, y, sigma, gL, want_z=True, want_y=True, want_coef=False):
        """One backward pass of L in one library call: (gz, gy, coef) =
        gL times (grad_z L, c(z), (dL/dA, dL/dB, dL/dgamma)), gL being a
        one-element float64 device tensor (the incoming gradient); an output
        not wanted is None."""
        torch = _torch()
        n, m = self.n, self.m
        if not (want_z or want_y or want_coef):
            raise ValueError("lagrangian_backward: no output is wanted")
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        yp = self._dev(y, self.sizes["ncon"], torch.float64, "y")
        gp = self._dev(gL, 1, torch.float64, "gL")
        gz = gy = coef = None
        zo = yo = ap = bp = cp = None
        if want_z:
            gz, zo = self._out(None, self.sizes["nvar"], "gz")
        if want_y:
            gy, yo = self._out(None, self.sizes["ncon"], "gy")
        if want_coef:
            f64 = dict(dtype=torch.float64, device=self.device)
            coef = (torch.empty(n, n, **f64), torch.empty(n, m, **f64), torch.empty(n, **f64))
            ap, cp = ctypes.c_void_p(coef[0].data_ptr()), ctypes.c_void_p(coef[2].data_ptr())
            bp = ctypes.c_void_p(coef[1].data_ptr()) if m else None
        _check(lib().ocp_eval_lagrangian_backward(self._h, zp, yp, float(sigma), gp, zo, yo, ap, bp, cp,
                                                  self._stream()), "ocp_eval_lagrangian_backward")
        return gz, gy, coef

    def coef_adjoint(self, z, y, tA, tB, tgamma, want_z=True, want_y=True, out_z=None, out_y=None):
        """The adjoint of coef_grad(z, y): for cotangents tA (n, n), tB (n, m)
        and tgamma (n,) of its three outputs, the gradients of
        tA . dL/dA + tB . dL/dB + tgamma . dL/dgamma in z (nvar doubles) and
        in y (ncon doubles), as (gz, gy); an output not wanted is None.  The
        handle's coefficients are neither read nor changed."""
        torch = _torch()
        n, m = self.n, self.m
        if not (want_z or want_y):
            raise ValueError("coef_adjoint: neither output is wanted")
        zp = self._dev(z, self.sizes["nvar"], torch.float64, "z")
        yp = self._dev(y, self.sizes["ncon"], torch.float64, "y")
        ap = self._dev(tA, n * n, torch.float64, "tA")
        bp = self._dev(tB, n * m, torch.float64, "tB") if m else None
        gp = self._dev(tgamma, n, torch.float64, "tgamma")
        gz = gy = None
        zo = yo = None
        if want_z:
            gz, zo = self._out(out_z, self.sizes["nvar"], "gz")
        if want_y:
            gy, yo = self._out(out_y, self.sizes["ncon"], "gy")
        _check(lib().ocp_eval_coef_adjoint(self._h, zp, yp, ap, bp, gp, zo, yo, self._stream()),
               "ocp_eval_coef_adjoint")
        return gz, gy


class QuadrotorProblem(Problem):
    """The quadrotor model on a GPU: the evaluations and the assembly of
    Problem, with the quadrotor's layouts (see ``quad_sizes``)."""

    def __init__(self, N, boundary=1, g=QUAD_G, r=QUAD_R, device=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise OcpError(OCP_ERR_HIP, "no GPU visible: this library runs only on gfx950 devices")
        self.N, self.n, self.m = int(N), 9, 4
        self.boundary = int(boundary)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().ocp_quad_create(self.N, self.boundary, float(g), float(r), ctypes.byref(h)),
                   "ocp_quad_create")
        self._h = h
        s = Sizes()
        _check(lib().ocp_problem_sizes(self._h, ctypes.byref(s)), "ocp_problem_sizes")
        self.sizes = s.as_dict()

    @classmethod
    def from_instance(cls, q, device=None):
        return cls(q.N, q.bnd, q.g, q.r, device)

    def pattern(self, jac: bool = True, hess: bool = True):
        """The quadrotor NLP's COO patterns (module quad_pattern())."""
        return quad_pattern(self.N, self.boundary, jac, hess)

    def kkt_pattern(self, rowptr=True, colind=True, perm_j=True, perm_h=True):
        """The quadrotor NLP's KKT structure (module quad_kkt_pattern())."""
        return quad_kkt_pattern(self.N, self.boundary, rowptr, colind, perm_j, perm_h)


def _autotune_cache_path() -> str:
    return os.environ.get("OCP_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2510_03932_amd",
                                       "autotune.json"))


class Graph:
    """An instantiated HIP graph of one batched evaluation (pointers bound at
    capture).  launch() replays it on the current torch stream."""

    def __init__(self, handle, device, keep, owner=None):
        self._h = handle
        self.device = device
        self._keep = keep  # tensors the graph reads or writes stay alive with it
        self._owner = owner  # the batch whose coefficients the graph reads

    def launch(self):
        if self._owner is not None and not self._owner._h.value:
            raise OcpError(OCP_ERR_ARG, "ocp_graph_launch: the graph's batch has been closed")
        stream = _raw_stream(self.device)
        _check(lib().ocp_graph_launch(self._h, stream), "ocp_graph_launch")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ocp_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent instances (own N_b, A, B, gamma, q, r; shared n, m)
    evaluated together.  Packed arrays hold each instance's single-instance
    array back to back; ``offsets`` gives the starts."""

    def __init__(self, Ns, n, m, A, B, gamma, q, r, device=None, scheme=0, boundary=0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise OcpError(OCP_ERR_HIP, "no GPU visible: this library runs only on gfx950 devices")
        Ns = np.ascontiguousarray(np.asarray(Ns, np.int64))
        self.count, self.n, self.m = int(len(Ns)), int(n), int(m)
        self.options = _opts(scheme, boundary)
        self.Ns = Ns
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        c = self.count
        f64 = lambda a, shape: np.ascontiguousarray(np.asarray(a, np.float64).reshape(shape))
        A = f64(A, (c, n, n))
        B = f64(B, (c, n, m)) if m else np.zeros((c, n, 0))
        gamma, q = f64(gamma, (c, n)), f64(q, (c, n))
        r = f64(r, (c, m)) if m else np.zeros((c, 0))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().ocp_batch_create_ex(c, _hp(Ns), self.n, self.m, ctypes.byref(self.options), _hp(A),
                                             _hp(B) if m else None, _hp(gamma), _hp(q),
                                             _hp(r) if m else None, ctypes.byref(h)), "ocp_batch_create")
        self._h = h
        offs = [np.zeros(c + 1, np.int64) for _ in range(6)]
        _check(lib().ocp_batch_offsets(self._h, *(_hp(o) for o in offs[:4])), "ocp_batch_offsets")
        _check(lib().ocp_batch_offsets_ex(self._h, _hp(offs[4]), _hp(offs[5])), "ocp_batch_offsets_ex")
        self.offsets = dict(zip(("z", "c", "jac", "hess", "kkt", "dim"), offs))
        self.tuning = None  # the autotuner's table of (shape, ms), once tuned

    @classmethod
    def from_instances(cls, insts, device=None, scheme=0, boundary=0):
        n, m = insts[0].n, insts[0].m
        return cls([i.N for i in insts], n, m, np.stack([i.A for i in insts]),
                   np.stack([i.B for i in insts]), np.stack([i.gamma for i in insts]),
                   np.stack([i.q for i in insts]), np.stack([i.r for i in insts]), device,
                   scheme=scheme, boundary=boundary)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ocp_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def config(self) -> dict:
        c = BatchConfig()
        _check(lib().ocp_batch_get_config(self._h, ctypes.byref(c)), "ocp_batch_get_config")
        return c.as_dict()

    @config.setter
    def config(self, cfg: dict):
        c = BatchConfig(int(cfg["block"]), int(cfg["pair"]), int(cfg["wgs_per_cu"]), int(cfg["order"]))
        _check(lib().ocp_batch_set_config(self._h, ctypes.byref(c)), "ocp_batch_set_config")

    def _args(self, z, y, jac, hess, what):
        torch = _torch()
        tot = {k: int(v[-1]) for k, v in self.offsets.items()}
        chk = self._dev  # the same tensor checks as a single problem
        zp = chk(z, tot["z"], torch.float64, "z")
        yp = chk(y, tot["c"], torch.float64, "y") if (what & EVAL_HESS) else None
        if (what & EVAL_JAC) and jac is None:
            jac = torch.empty(tot["jac"], dtype=torch.float64, device=self.device)
        if (what & EVAL_HESS) and hess is None:
            hess = torch.empty(tot["hess"], dtype=torch.float64, device=self.device)
        jp = chk(jac, tot["jac"], torch.float64, "jac") if (what & EVAL_JAC) else None
        hp = chk(hess, tot["hess"], torch.float64, "hess") if (what & EVAL_HESS) else None
        return zp, yp, jp, hp, jac, hess

    _dev = Problem._dev

    def eval(self, z, y=None, sigma=1.0, jac=None, hess=None, what=EVAL_JAC | EVAL_HESS,
             mode="persistent"):
        """Packed Jacobian and/or Hessian values of every instance: (jac, hess)."""
        zp, yp, jp, hp, jac, hess = self._args(z, y, jac, hess, what)
        stream = _raw_stream(self.device)
        _check(lib().ocp_batch_eval(self._h, what, MODES[mode], zp, yp, float(sigma), jp, hp, stream),
               "ocp_batch_eval")
        return jac, hess

    def graph(self, z, y=None, sigma=1.0, jac=None, hess=None, what=EVAL_JAC | EVAL_HESS,
              mode="persistent"):
        """Capture one evaluation into a HIP graph: returns (Graph, jac, hess)."""
        zp, yp, jp, hp, jac, hess = self._args(z, y, jac, hess, what)
        g = ctypes.c_void_p()
        with _torch().cuda.device(self.device):
            _check(lib().ocp_batch_graph_create(self._h, what, MODES[mode], zp, yp, float(sigma), jp,
                                                hp, ctypes.byref(g)), "ocp_batch_graph_create")
        # the graph also reads this batch's coefficients and offset table
        return Graph(g, self.device, (z, y, jac, hess), owner=self), jac, hess

    # -- whole interior-point step ---------------------------------------------
    _STEP_OUT = (("obj", EVAL_OBJ, None), ("grad", EVAL_GRAD, "z"), ("cons", EVAL_CONS, "c"),
                 ("jac", EVAL_JAC, "jac"), ("hess", EVAL_HESS, "hess"), ("kkt", EVAL_KKT, "kkt"))

    def _io(self, z, y, sigma, reg, what, out):
        """The BatchIO of one step and the output tensors (allocated where
        `out` lacks them; None for parts not requested)."""
        torch = _torch()
        tot = {k: int(v[-1]) for k, v in self.offsets.items()}
        chk = self._dev
        io = BatchIO()
        io.z = chk(z, tot["z"], torch.float64, "z")
        if what & (EVAL_HESS | EVAL_KKT) or y is not None:
            io.y = chk(y, tot["c"], torch.float64, "y") if y is not None else None
        if reg is not None:
            io.reg = chk(reg, tot["dim"], torch.float64, "reg")
        io.sigma = float(sigma)
        out = dict(out or {})
        res = {}
        for name, bit, key in self._STEP_OUT:
            if not what & bit:
                res[name] = None
                continue
            size = self.count if key is None else tot[key]
            t = out.get(name)
            if t is None:
                t = torch.empty(size, dtype=torch.float64, device=self.device)
            setattr(io, name, chk(t, size, torch.float64, name))
            res[name] = t
        return io, res

    def step(self, z, y=None, sigma=1.0, reg=None, what=EVAL_ALL, mode="persistent", out=None):
        """Evaluate the parts of an interior-point step that `what` selects
        (EVAL_OBJ, EVAL_GRAD, EVAL_CONS, EVAL_JAC, EVAL_HESS, EVAL_KKT) for
        every instance; returns {"obj", "grad", "cons", "jac", "hess", "kkt"}
        (packed device tensors, None where not requested)."""
        io, res = self._io(z, y, sigma, reg, what, out)
        stream = _raw_stream(self.device)
        _check(lib().ocp_batch_eval_io(self._h, int(what), MODES[mode], ctypes.byref(io), stream),
               "ocp_batch_eval_io")
        return res

    def prepare(self, what=EVAL_ALL):
        """Build the persistent tile lists of `what` now (so that a later
        evaluation or capture allocates nothing)."""
        _check(lib().ocp_batch_prepare(self._h, int(what)), "ocp_batch_prepare")

    def step_graph(self, z, y=None, sigma=1.0, reg=None, what=EVAL_ALL, mode="persistent", out=None):
        """Capture one step into a HIP graph: returns the Graph (its outputs
        are the tensors of `out`, allocated where missing, in graph.outputs)."""
        io, res = self._io(z, y, sigma, reg, what, out)
        g = ctypes.c_void_p()
        with _torch().cuda.device(self.device):
            _check(lib().ocp_batch_graph_create_io(self._h, int(what), MODES[mode], ctypes.byref(io),
                                                   ctypes.byref(g)), "ocp_batch_graph_create_io")
        graph = Graph(g, self.device, (z, y, reg, *res.values()), owner=self)
        graph.outputs = res
        return graph

    def autotune_step(self, z, y=None, sigma=1.0, reg=None, what=EVAL_ALL, reps=5, out=None):
        """Time every tile shape on the step `what` and keep the fastest:
        returns (config, ms per step, table)."""
        torch = _torch()
        io, res = self._io(z, y, sigma, reg, what, out)
        best = BatchConfig()
        ms = ctypes.c_float()
        table = np.zeros(len(AUTOTUNE_SHAPES), np.float32)
        stream = _raw_stream(self.device)
        _check(lib().ocp_batch_autotune_io(self._h, int(what), ctypes.byref(io), int(reps), stream,
                                           ctypes.byref(best), ctypes.byref(ms), _hp(table)),
               "ocp_batch_autotune_io")
        tab = [dict(shape, ms=float(t)) for shape, t in zip(AUTOTUNE_SHAPES, table)]
        return best.as_dict(), float(ms.value), tab

    def autotune(self, z, y=None, sigma=1.0, jac=None, hess=None, what=EVAL_JAC | EVAL_HESS,
                 reps=5, cache: str | None = None, use_cache=True):
        """Pick the fastest tile shape of the persistent launch (timed in the
        library), remember it in a JSON cache keyed by device, shape and work,
        and set it.  Returns (config, ms per evaluation)."""
        import json
        torch = _torch()
        key = "|".join([torch.cuda.get_device_name(self.device), f"n{self.n}", f"m{self.m}",
                        f"count{self.count}", f"sumN{int(self.Ns.sum())}", f"what{what}"])
        path = cache or _autotune_cache_path()
        db = {}
        if use_cache and os.path.exists(path):
            try:
                db = json.load(open(path))
            except (OSError, ValueError):
                db = {}
        if use_cache and key in db:
            self.config = db[key]["config"]
            self.tuning = db[key].get("table")
            return db[key]["config"], float(db[key]["ms"])
        zp, yp, jp, hp, jac, hess = self._args(z, y, jac, hess, what)
        best = BatchConfig()
        ms = ctypes.c_float()
        table = np.zeros(len(AUTOTUNE_SHAPES), np.float32)
        stream = _raw_stream(self.device)
        _check(lib().ocp_batch_autotune(self._h, what, zp, yp, float(sigma), jp, hp, int(reps), stream,
                                        ctypes.byref(best), ctypes.byref(ms), _hp(table)),
               "ocp_batch_autotune")
        cfg = best.as_dict()
        self.tuning = [dict(shape, ms=float(t)) for shape, t in zip(AUTOTUNE_SHAPES, table)]
        db[key] = {"config": cfg, "ms": float(ms.value), "table": self.tuning}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(db, fh, indent=1)
            os.replace(tmp, path)
        except OSError:
            pass  # an unwritable cache only costs a re-tune next time
        return cfg, float(ms.value)
