"""GPU parity: every entry point of the C ABI (through the Python binding)
against the CPU oracle, element by element, on the same seeded inputs.

Bar: values within 1e-12 * mu (mu = sum of |terms| of each entry, from the
oracle), equality where mu = 0; KKT assembly bit-exact given the same inputs;
repeated evaluations bitwise identical.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import REL, check_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (N, n, m): the 1000-interval parity workload, ragged tails (odd N, N not a
# multiple of the workgroup), the degenerate sizes, and the maximum dimensions.
SHAPES = [
    (1000, 4, 2),
    (777, 5, 3),
    (1, 1, 0),
    (1, 1, 1),
    (2, 2, 1),
    (3, 3, 0),
    (2, 1, 3),
    (255, 2, 0),
    (256, 3, 1),
    (257, 16, 8),
    (1023, 6, 3),
    (4097, 8, 4),
    (513, 32, 32),
    (100, 17, 0),
    (50, 2, 9),
    (33, 5, 20),
]


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


def _evaluate(ocp, inst, sigma=None):
    dev = torch.device("cuda", 0)
    prob = ocp.Problem.from_instance(inst, dev)
    z = torch.from_numpy(inst.z).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    sigma = inst.sigma if sigma is None else sigma
    out = dict(obj=prob.obj(z), grad=prob.grad(z), cons=prob.cons(z), jac=prob.jac(z),
               hess=prob.hess(z, y, sigma))
    torch.cuda.synchronize()
    return prob, {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("N,n,m", SHAPES)
def test_values_match_oracle(ocp, N, n, m):
    _say(f"[parity] N={N} n={n} m={m}")
    inst = synth.make_instance(N, n, m, seed=0)
    prob, got = _evaluate(ocp, inst)
    f, fmu = oracle.obj(inst)
    # the objective sums N+1 nodes in a different (tree) order than the oracle's
    # compensated sum: rounding of a sum of nonnegative terms grows like
    # log2(N) eps, far inside the bar
    check_close(got["obj"], np.array([f]), np.array([fmu]), what="obj")
    for name, fn in (("grad", oracle.grad), ("cons", oracle.cons), ("jac", oracle.jac),
                     ("hess", oracle.hess)):
        want, mu = fn(inst)
        check_close(got[name], want, mu, what=name)
    prob.close()


@pytest.mark.parametrize("N,n,m", [(1000, 4, 2), (777, 5, 3), (1, 1, 0), (2, 2, 1), (513, 32, 32)])
@pytest.mark.parametrize("with_reg", [False, True])
def test_assemble_kkt_bit_exact(ocp, N, n, m, with_reg):
    _say(f"[assemble] N={N} n={n} m={m} reg={with_reg}")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=1)
    prob, got = _evaluate(ocp, inst)
    rowptr, colind, perm_j, perm_h = ocp.kkt_pattern(N, n, m)
    s = prob.sizes
    reg = np.random.default_rng(5).normal(size=s["dim"]) if with_reg else None
    kkt = prob.assemble_kkt(torch.from_numpy(perm_j).to(dev), torch.from_numpy(perm_h).to(dev),
                            torch.from_numpy(rowptr).to(dev), torch.from_numpy(got["jac"]).to(dev),
                            torch.from_numpy(got["hess"]).to(dev),
                            None if reg is None else torch.from_numpy(reg).to(dev))
    kkt = kkt.cpu().numpy()
    want = oracle.assemble(rowptr, perm_j, got["jac"], perm_h, got["hess"], reg)
    assert np.array_equal(kkt.view(np.uint64), want.view(np.uint64))
    prob.close()


@pytest.mark.parametrize("N,n,m", [(1000, 4, 2), (130, 32, 32), (77, 3, 1)])
@pytest.mark.parametrize("scope", ["within_rows", "global"])
def test_assemble_generic_slot_map(ocp, N, n, m, scope):
    """assemble_kkt reads the slot maps instead of assuming their closed form:
    shuffle the Jacobian/Hessian slots (constraint diagonals fixed) either
    within each CSR row (every tile still covers its range exactly) or over the
    whole matrix (tiles fall back to direct stores).  Without reg the result
    must equal the oracle's plain scatter bit for bit."""
    _say(f"[assemble-generic] N={N} n={n} m={m} {scope}")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=8)
    prob, got = _evaluate(ocp, inst)
    rowptr, _, perm_j, perm_h = ocp.kkt_pattern(N, n, m, colind=False)
    s = prob.sizes
    rng = np.random.default_rng(11)
    movable = np.concatenate([perm_h, perm_j])
    pi = np.arange(s["nnzk"], dtype=np.int64)
    if scope == "global":
        pi[movable] = movable[rng.permutation(len(movable))]
    else:
        rows = np.repeat(np.arange(s["dim"]), np.diff(rowptr))
        for d in rng.choice(s["dim"], size=min(s["dim"], 2000), replace=False):
            slots = np.arange(rowptr[d], rowptr[d + 1])
            slots = slots[np.isin(slots, movable)]
            pi[slots] = rng.permutation(slots)
        assert np.all(rows[pi] == rows)
    pj2 = pi[perm_j].astype(np.int32)
    ph2 = pi[perm_h].astype(np.int32)
    kkt = prob.assemble_kkt(torch.from_numpy(pj2).to(dev), torch.from_numpy(ph2).to(dev),
                            torch.from_numpy(rowptr).to(dev), torch.from_numpy(got["jac"]).to(dev),
                            torch.from_numpy(got["hess"]).to(dev))
    want = oracle.assemble(rowptr, pj2, got["jac"], ph2, got["hess"], None)
    assert np.array_equal(kkt.cpu().numpy().view(np.uint64), want.view(np.uint64))
    prob.close()


def test_assemble_overwrites_output(ocp):
    """Each call fully overwrites its output: garbage in the buffer beforehand
    must not survive."""
    dev = torch.device("cuda", 0)
    N, n, m = 300, 4, 2
    inst = synth.make_instance(N, n, m, seed=2)
    prob, got = _evaluate(ocp, inst)
    rowptr, _, perm_j, perm_h = ocp.kkt_pattern(N, n, m, colind=False)
    args = [torch.from_numpy(a).to(dev) for a in (perm_j, perm_h, rowptr, got["jac"], got["hess"])]
    out = torch.full((prob.sizes["nnzk"],), float("nan"), dtype=torch.float64, device=dev)
    prob.assemble_kkt(*args, out=out)
    want = oracle.assemble(rowptr, perm_j, got["jac"], perm_h, got["hess"], None)
    assert np.array_equal(out.cpu().numpy().view(np.uint64), want.view(np.uint64))
    prob.close()


@pytest.mark.parametrize("N,n,m", [(1000, 4, 2), (4097, 8, 4)])
def test_deterministic_and_layout_independent(ocp, N, n, m):
    """Two runs are bitwise equal, and the paired-store Jacobian path (aligned
    output, even N) gives bitwise the same values as the single-store path
    (output shifted by one double)."""
    _say(f"[determinism] N={N} n={n} m={m}")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=3)
    prob = ocp.Problem.from_instance(inst, dev)
    z = torch.from_numpy(inst.z).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    a = [prob.obj(z), prob.grad(z), prob.cons(z), prob.jac(z), prob.hess(z, y, 1.0)]
    b = [prob.obj(z), prob.grad(z), prob.cons(z), prob.jac(z), prob.hess(z, y, 1.0)]
    for u, v in zip(a, b):
        assert torch.equal(u.view(torch.int64), v.view(torch.int64))
    nnzj = prob.sizes["nnzj"]
    buf = torch.empty(nnzj + 1, dtype=torch.float64, device=dev)
    shifted = prob.jac(z, out=buf[1:])
    assert shifted.data_ptr() % 16 == 8
    assert torch.equal(shifted.view(torch.int64), a[3].view(torch.int64))
    prob.close()


def test_sigma_and_multiplier_scaling(ocp):
    """sigma = 0 removes the cost from the Hessian; y = 0 leaves only the cost."""
    dev = torch.device("cuda", 0)
    N, n, m = 200, 5, 2
    inst = synth.make_instance(N, n, m, seed=4)
    prob = ocp.Problem.from_instance(inst, dev)
    z = torch.from_numpy(inst.z).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    for sigma, yy in ((0.0, inst.y), (2.5, np.zeros_like(inst.y))):
        got = prob.hess(z, torch.from_numpy(yy).to(dev), sigma).cpu().numpy()
        want, mu = oracle.hess(inst, sigma=sigma, y=yy)
        check_close(got, want, mu, what=f"hess sigma={sigma}")
    prob.close()


def test_binding_rejects_bad_tensors(ocp):
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(10, 2, 1)
    prob = ocp.Problem.from_instance(inst, dev)
    z = torch.from_numpy(inst.z).to(dev)
    with pytest.raises(TypeError):
        prob.grad(z.float())
    with pytest.raises(ValueError):
        prob.grad(z[:-1])
    with pytest.raises(ValueError):
        prob.grad(z.cpu())
    with pytest.raises(ValueError):
        prob.cons(torch.empty(2 * len(inst.z), dtype=torch.float64, device=dev)[::2])
    prob.close()


# ---- the 1e5-interval workload: full arrays ---------------------------------

def test_ipm_loop_workload_full_arrays(ocp):
    N, n, m = synth.IPM_LOOP
    _say(f"[ipm-loop] N={N} n={n} m={m}")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=0)
    prob = ocp.Problem.from_instance(inst, dev)
    rowptr, _, perm_j, perm_h = ocp.kkt_pattern(N, n, m, colind=False)
    pj, ph, rp = (torch.from_numpy(a).to(dev) for a in (perm_j, perm_h, rowptr))
    for it in (0, 49):  # first and last point of the 50-iteration loop the benchmark times
        z, y = synth.device_point(torch, dev, N, n, m, 1000 + it)
        inst.z = z.cpu().numpy()
        inst.y = y.cpu().numpy()
        c, jv, hv = prob.cons(z), prob.jac(z), prob.hess(z, y, 1.0)
        reg = torch.linspace(-1.0, 1.0, prob.sizes["dim"], dtype=torch.float64, device=dev)
        kkt = prob.assemble_kkt(pj, ph, rp, jv, hv, reg)
        torch.cuda.synchronize()
        for name, got, fn in (("cons", c, oracle.cons), ("jac", jv, oracle.jac),
                              ("hess", hv, oracle.hess)):
            want, mu = fn(inst)
            check_close(got.cpu().numpy(), want, mu, what=f"{name} it={it}")
        want = oracle.assemble(rowptr, perm_j, jv.cpu().numpy(), perm_h, hv.cpu().numpy(),
                               reg.cpu().numpy())
        assert np.array_equal(kkt.cpu().numpy().view(np.uint64), want.view(np.uint64))
    prob.close()


# ---- the 1e6-interval, n = 16, m = 8 workload: sampled node ranges ----------

@pytest.fixture(scope="module")
def large(ocp):
    N, n, m = synth.LARGE
    _say(f"[large] building N={N} n={n} m={m}")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=0)
    prob = ocp.Problem.from_instance(inst, dev)
    z = torch.from_numpy(inst.z).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    yield inst, prob, z, y
    prob.close()
    torch.cuda.empty_cache()


RANGES = [(0, 2048), (499_000, 501_000), (1_000_000 - 2048, 1_000_000)]


def test_large_values_sampled(large):
    inst, prob, z, y = large
    N, n, m = inst.N, inst.n, inst.m
    T, S = 2 * n + 2 * m, prob.sizes["S"]
    _say("[large] values")
    f, fmu = oracle.obj(inst)
    check_close(prob.obj(z).cpu().numpy(), np.array([f]), np.array([fmu]), what="obj")
    g = prob.grad(z).view(n + m, N + 1)
    c = prob.cons(z).view(n, N)
    for k0, k1 in RANGES:
        want, mu = oracle.grad(inst, k0, k1 + 1)
        check_close(g[:, k0:k1 + 1].cpu().numpy().ravel(), want, mu, what=f"grad {k0}")
        want, mu = oracle.cons(inst, k0, k1)
        check_close(c[:, k0:k1].cpu().numpy().ravel(), want, mu, what=f"cons {k0}")
    del g, c
    jv = prob.jac(z).view(n * T, N)
    for k0, k1 in RANGES:
        want, mu = oracle.jac(inst, k0, k1)
        check_close(jv[:, k0:k1].cpu().numpy().ravel(), want, mu, what=f"jac {k0}")
    del jv
    hv = prob.hess(z, y, inst.sigma).view(S, N + 1)
    for k0, k1 in RANGES + [(N - 10, N + 1)]:
        want, mu = oracle.hess(inst, k0, k1)
        check_close(hv[:, k0:k1].cpu().numpy().ravel(), want, mu, what=f"hess {k0}")
    del hv
    torch.cuda.empty_cache()


def test_large_assemble_sampled(ocp, large):
    """Full-size assembly, checked at 2e6 sampled Jacobian entries, every
    Hessian entry and every constraint diagonal against the scatter's definition."""
    inst, prob, z, y = large
    _say("[large] assemble")
    dev = z.device
    s = prob.sizes
    rowptr, _, perm_j, perm_h = ocp.kkt_pattern(inst.N, inst.n, inst.m, colind=False)
    pj = torch.from_numpy(perm_j).to(dev)
    del perm_j
    ph, rp = torch.from_numpy(perm_h).to(dev), torch.from_numpy(rowptr).to(dev)
    reg = torch.from_numpy(np.random.default_rng(6).normal(size=s["dim"])).to(dev)
    jv = prob.jac(z)
    hv = prob.hess(z, y, inst.sigma)
    kkt = prob.assemble_kkt(pj, ph, rp, jv, hv, reg)
    torch.cuda.synchronize()
    e = torch.from_numpy(np.random.default_rng(7).integers(0, s["nnzj"], 2_000_000)).to(dev)
    assert torch.equal(kkt[pj[e].long()].view(torch.int64), jv[e].view(torch.int64))
    # Hessian entries: diagonal slots get hess + reg in one add
    hrow = torch.from_numpy(ocp.pattern(inst.N, inst.n, inst.m, jac=False)[2]).to(dev).long()
    hcol_is_diag = torch.from_numpy(ocp.pattern(inst.N, inst.n, inst.m, jac=False)[3]).to(dev).long() == hrow
    want_h = torch.where(hcol_is_diag, hv + reg[hrow], hv)
    assert torch.equal(kkt[ph.long()].view(torch.int64), want_h.view(torch.int64))
    d = torch.arange(s["nvar"], s["dim"], device=dev)
    assert torch.equal(kkt[(rp[d + 1] - 1).long()].view(torch.int64), reg[d].view(torch.int64))
    del kkt, pj, jv, hv
    torch.cuda.empty_cache()
