"""The allocation-free coefficient gradient, called through the C ABI: its
output equals ocp_eval_coef_grad's bit for bit (same kernels, same reduction
order), on two calls in a row, the second on a smaller problem, and it meets
the oracle's bar (|gpu - oracle| <= 1e-12 mu).  A problem whose partial sums
exceed the fixed scratch array is refused before any HIP call."""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import check_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ocp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_03932_amd as ocp
    L = ocp.lib()
    vp = ctypes.c_void_p
    L.ocp_eval_coef_grad_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    return ocp


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _coef_grad(ocp, prob, z, y, fn):
    """dL/d(A, B, gamma) through the C entry point `fn` on the current stream."""
    n, m = prob.n, prob.m
    f64 = dict(dtype=torch.float64, device=z.device)
    gA, gB, gg = torch.empty(n, n, **f64), torch.empty(n, max(m, 1), **f64), torch.empty(n, **f64)
    # poison the outputs so a call that writes nothing cannot pass
    for t in (gA, gB, gg):
        t.fill_(float("nan"))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(ocp.lib(), fn)(prob._h, _ptr(z), _ptr(y), _ptr(gA), _ptr(gB) if m else None,
                                _ptr(gg), stream)
    if rc != 0:
        raise ocp.OcpError(rc, ocp.lib().ocp_last_error().decode())
    torch.cuda.synchronize()
    return gA.cpu().numpy(), gB[:, :m].cpu().numpy(), gg.cpu().numpy()


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


@pytest.mark.parametrize("first,second", [((200_000, 8, 4), (5_000, 4, 2)),
                                          ((1_000_000, 16, 8), (777, 5, 3))])
def test_noalloc_matches_workspace_entry_point(ocp, first, second):
    dev = torch.device("cuda", 0)
    for (N, n, m), seed in ((first, 3), (second, 4)):
        _say(f"[no-alloc] N={N} n={n} m={m} seed={seed}")
        inst = synth.make_instance(N, n, m, seed=seed)
        prob = ocp.Problem.from_instance(inst, dev)
        z = torch.from_numpy(inst.z).to(dev)
        y = torch.from_numpy(inst.y).to(dev)
        ref = _coef_grad(ocp, prob, z, y, "ocp_eval_coef_grad")
        got = _coef_grad(ocp, prob, z, y, "ocp_eval_coef_grad_noalloc")
        for name, a, b in zip(("dL/dA", "dL/dB", "dL/dgamma"), got, ref):
            assert np.array_equal(_bits(a), _bits(b)), f"{name} differs from ocp_eval_coef_grad"
        if N <= 200_000:
            (oA, oB, og), (mA, mB, mg) = oracle.coef_grad(inst)
            check_close(got[0], oA, mA, what=f"no-alloc dL/dA N={N}")
            check_close(got[1], oB, mB, what=f"no-alloc dL/dB N={N}")
            check_close(got[2], og, mg, what=f"no-alloc dL/dgamma N={N}")
        prob.close()


def test_noalloc_refuses_problems_beyond_the_scratch_array(ocp):
    dev = torch.device("cuda", 0)
    # n = 32, m = 32: 32 * 65 partial rows per workgroup, 1024 workgroups at
    # N + 1 >= 65536 nodes -> 2,129,920 doubles > 524,288
    N, n, m = 70_000, 32, 32
    _say(f"[no-alloc] refusal N={N} n={n} m={m}")
    inst = synth.make_instance(N, n, m, seed=5)
    prob = ocp.Problem.from_instance(inst, dev)
    z = torch.from_numpy(inst.z).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    with pytest.raises(ocp.OcpError) as exc:
        _coef_grad(ocp, prob, z, y, "ocp_eval_coef_grad_noalloc")
    assert exc.value.code == 1 and "scratch" in str(exc.value)
    # the workspace entry point still serves it, and the library stays usable
    ref = _coef_grad(ocp, prob, z, y, "ocp_eval_coef_grad")
    assert all(np.all(np.isfinite(a)) for a in ref)
    prob.close()
