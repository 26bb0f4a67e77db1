"""The largest problems the int32 index space allows (every KKT position
below 2^31): n = 16, m = 8 at N = 2,606,189 (2.1e9 KKT values, about 60 GB
of device memory with the checks) and n = 2, m = 1 at N = 119,304,647
(1.2e8 nodes).  Index arithmetic that overflows 32 bits anywhere in the
evaluation or the assembly shows up only here.  The checks: the oracle on
node ranges at both ends of the grid (values within 1e-12 mu), the objective
in full, the assembly against its definition on sampled and on the last
Jacobian entries, every Hessian entry and every constraint diagonal, and the
fused evaluation against the separate path on the whole KKT array."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import check_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

INT32_MAX = 2**31 - 1


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ocp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_03932_amd as ocp
    ocp.lib()
    return ocp


def _largest_N(ocp, n, m):
    """Largest N the library accepts for (n, m): nnzk = nnzh + nnzj + ncon
    grows by S + nT + n per interval."""
    s1 = ocp.sizes(1, n, m)
    per = s1["S"] + n * s1["T"] + n
    N = (INT32_MAX - s1["S"]) // per
    s = ocp.sizes(N, n, m)
    assert s["nnzk"] <= INT32_MAX < s["nnzk"] + per
    with pytest.raises(ocp.OcpError) as e:
        ocp.sizes(N + 1, n, m)
    assert e.value.code == ocp.OCP_ERR_OVERFLOW
    return N


def _close_on_device(a, b):
    """|a - b| <= 1e-12 (|a| + |b|) + 1e-18 element-wise, in chunks."""
    step = 1 << 27
    for i in range(0, a.numel(), step):
        x, y = a[i:i + step], b[i:i + step]
        assert bool(((x - y).abs() <= 1e-12 * (x.abs() + y.abs()) + 1e-18).all()), i


@pytest.mark.parametrize("n,m", [(16, 8), (2, 1)])
def test_largest_int32_problem(ocp, n, m):
    N = _largest_N(ocp, n, m)
    _say(f"[limits] N={N} n={n} m={m}: drawing the instance")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=0)
    prob = ocp.Problem.from_instance(inst, dev)
    s = prob.sizes
    T, S = s["T"], s["S"]
    z = torch.from_numpy(inst.z).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    ends = [(0, 512), (N - 512, N)]

    _say("[limits] obj, grad, cons")
    f, fmu = oracle.obj(inst)
    check_close(prob.obj(z).cpu().numpy(), np.array([f]), np.array([fmu]), what="obj")
    g = prob.grad(z).view(n + m, N + 1)
    for k0, k1 in ends:
        want, mu = oracle.grad(inst, k0, k1 + 1)
        check_close(g[:, k0:k1 + 1].cpu().numpy().ravel(), want, mu, what=f"grad {k0}")
    del g
    c = prob.cons(z).view(n, N)
    for k0, k1 in ends:
        want, mu = oracle.cons(inst, k0, k1)
        check_close(c[:, k0:k1].cpu().numpy().ravel(), want, mu, what=f"cons {k0}")
    del c

    _say("[limits] jac, hess")
    jv = prob.jac(z)
    for k0, k1 in ends:
        want, mu = oracle.jac(inst, k0, k1)
        check_close(jv.view(n * T, N)[:, k0:k1].cpu().numpy().ravel(), want, mu, what=f"jac {k0}")
    hv = prob.hess(z, y, inst.sigma)
    for k0, k1 in [(0, 512), (N - 511, N + 1)]:
        want, mu = oracle.hess(inst, k0, k1)
        check_close(hv.view(S, N + 1)[:, k0:k1].cpu().numpy().ravel(), want, mu, what=f"hess {k0}")

    _say("[limits] KKT pattern and assembly")
    rowptr, _, perm_j, perm_h = ocp.kkt_pattern(N, n, m, colind=False)
    assert int(rowptr[-1]) == s["nnzk"]
    pj = torch.from_numpy(perm_j).to(dev)
    del perm_j
    ph, rp = torch.from_numpy(perm_h).to(dev), torch.from_numpy(rowptr).to(dev)
    del perm_h, rowptr
    reg = torch.linspace(1e-8, 2e-8, s["dim"], dtype=torch.float64, device=dev)
    kkt = prob.assemble_kkt(pj, ph, rp, jv, hv, reg)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    e = torch.from_numpy(np.concatenate([rng.integers(0, s["nnzj"], 2_000_000),
                                         np.arange(s["nnzj"] - 1_000_000, s["nnzj"])])).to(dev)
    assert torch.equal(kkt[pj[e].long()].view(torch.int64), jv[e].view(torch.int64))
    del e
    hrow = torch.from_numpy(ocp.pattern(N, n, m, jac=False)[2]).to(dev).long()
    hcol = torch.from_numpy(ocp.pattern(N, n, m, jac=False)[3]).to(dev).long()
    want_h = torch.where(hcol == hrow, hv + reg[hrow], hv)
    assert torch.equal(kkt[ph.long()].view(torch.int64), want_h.view(torch.int64))
    del hrow, hcol, want_h
    d = torch.arange(s["nvar"], s["dim"], device=dev)
    assert torch.equal(kkt[(rp[d + 1] - 1).long()].view(torch.int64), reg[d].view(torch.int64))
    del d, pj, ph, jv, hv
    torch.cuda.empty_cache()

    _say("[limits] fused evaluation into the KKT")
    fused = prob.eval_kkt(z, y, inst.sigma, reg)
    torch.cuda.synchronize()
    _close_on_device(fused, kkt)
    del fused, kkt, reg
    prob.close()
    torch.cuda.empty_cache()
