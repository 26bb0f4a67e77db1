"""GPU parity of the KKT assembly through slot maps (ocp_assemble_kkt_mapped,
with and without a plan from ocp_mapped_plan, with the handle's own cached
plan, and with a plan made from other maps) against the oracle's slot-map
assembly, bit for bit: under the node-grouped
fill-reducing ordering (every tile staged), under a random ordering (every
tile falls back to direct stores) and under the natural ordering (where it
must equal ocp_assemble_kkt); for both models, both schemes and every
boundary option, with and without reg; and at the quadrotor's N = 1e6 and
the synthetic family's N = 1e5 sizes."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(1, 1, 0, 0, 0), (2, 2, 1, 1, 2), (7, 3, 1, 0, 1), (257, 4, 2, 0, 0), (300, 5, 3, 1, 2),
          (1000, 16, 8, 0, 1), (65, 32, 32, 0, 0)]


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


def _dev(*arrays):
    dev = torch.device("cuda", 0)
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrays]


def _check_orders(ocp, prob, rp, ci, pj, ph, jv, hv, stage, seed):
    dim = len(rp) - 1
    reg = np.random.default_rng(seed).normal(size=dim)
    orders = {"stage": stage, "random": np.random.default_rng(seed).permutation(dim).astype(np.int32),
              "natural": np.arange(dim, dtype=np.int32)}
    gj, gh = _dev(jv, hv)
    for name, order in orders.items():
        rp2, ci2, pj2, ph2, dg2 = ocp.kkt_permute(rp, ci, pj, ph, order)
        maps = _dev(pj2, ph2, dg2)
        plan = prob.mapped_plan(*maps)
        pl = plan.cpu().numpy().reshape(-1, 2)
        assert pl[:, 1].sum() == rp2[-1]  # the tiles' slots partition the KKT
        if name == "stage":
            assert np.all(pl[:, 0] >= 0)  # every tile is one contiguous CSR range
        for r in (None, reg):
            rt = None if r is None else _dev(r)[0]
            want = oracle.assemble_mapped(rp2[-1], dg2, pj2, jv, ph2, hv, r)
            for use_plan in (False, True):
                got = prob.assemble_kkt_mapped(*maps, gj, gh, rt, plan=plan if use_plan else None).cpu().numpy()
                assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (name, r is None, use_plan)
        if name == "natural":
            nat = prob.assemble_kkt(*_dev(pj, ph, rp), gj, gh, _dev(reg)[0]).cpu().numpy()
            got = prob.assemble_kkt_mapped(*_dev(pj2, ph2, dg2), gj, gh, _dev(reg)[0]).cpu().numpy()
            assert np.array_equal(got.view(np.uint64), nat.view(np.uint64))


@pytest.mark.parametrize("N,n,m,scheme,bnd", SHAPES)
def test_mapped_assembly_synthetic(ocp, N, n, m, scheme, bnd):
    _say(f"[mapped] N={N} n={n} m={m} scheme={scheme} bnd={bnd}")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=31, scheme=scheme, bnd=bnd)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y = _dev(inst.z, inst.y)
    jv, hv = prob.jac(z).cpu().numpy(), prob.hess(z, y, 1.0).cpu().numpy()
    rp, ci, pj, ph = ocp.kkt_pattern(N, n, m, scheme=scheme, boundary=bnd)
    _check_orders(ocp, prob, rp, ci, pj, ph, jv, hv, ocp.stage_order(N, n, m, scheme, bnd), N)
    prob.close()


@pytest.mark.parametrize("N,bnd", [(1, 1), (2, 0), (255, 2), (1000, 1)])
def test_mapped_assembly_quadrotor(ocp, N, bnd):
    _say(f"[mapped quad] N={N} bnd={bnd}")
    dev = torch.device("cuda", 0)
    q = synth.make_quadrotor(N, seed=32, bnd=bnd)
    prob = ocp.QuadrotorProblem.from_instance(q, dev)
    z, y = _dev(q.z, q.y)
    jv, hv = prob.jac(z).cpu().numpy(), prob.hess(z, y, 1.0).cpu().numpy()
    rp, ci, pj, ph = ocp.quad_kkt_pattern(N, bnd)
    _check_orders(ocp, prob, rp, ci, pj, ph, jv, hv, ocp.quad_stage_order(N, bnd), N)
    prob.close()


def test_mapped_assembly_overwrites_output(ocp):
    dev = torch.device("cuda", 0)
    N, n, m = 300, 4, 2
    inst = synth.make_instance(N, n, m, seed=33)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y = _dev(inst.z, inst.y)
    jv, hv = prob.jac(z), prob.hess(z, y, 1.0)
    rp, ci, pj, ph = ocp.kkt_pattern(N, n, m)
    rp2, ci2, pj2, ph2, dg2 = ocp.kkt_permute(rp, ci, pj, ph, ocp.stage_order(N, n, m))
    out = torch.full((prob.sizes["nnzk"],), float("nan"), dtype=torch.float64, device=dev)
    prob.assemble_kkt_mapped(*_dev(pj2, ph2, dg2), jv, hv, out=out)
    want = oracle.assemble_mapped(rp2[-1], dg2, pj2, jv.cpu().numpy(), ph2, hv.cpu().numpy(), None)
    assert np.array_equal(out.cpu().numpy().view(np.uint64), want.view(np.uint64))
    prob.close()


def test_mapped_assembly_large(ocp):
    """Reordered KKT of the quadrotor at N = 1e6 and of the synthetic family at
    N = 1e5 (n = 8, m = 4), in the launch configuration the benchmark times."""
    dev = torch.device("cuda", 0)
    _say("[mapped] quadrotor N=1e6")
    N = synth.QUAD_LARGE
    q = synth.make_quadrotor(N, seed=0, bnd=1)
    prob = ocp.QuadrotorProblem.from_instance(q, dev)
    z, y = _dev(q.z, q.y)
    jv, hv = prob.jac(z), prob.hess(z, y, 1.0)
    rp, ci, pj, ph = ocp.quad_kkt_pattern(N, 1)
    rp2, ci2, pj2, ph2, dg2 = ocp.kkt_permute(rp, ci, pj, ph, ocp.quad_stage_order(N, 1))
    del ci, ci2
    reg = np.full(prob.sizes["dim"], 1e-8)
    maps = _dev(pj2, ph2, dg2)
    plan = prob.mapped_plan(*maps)
    want = oracle.assemble_mapped(rp2[-1], dg2, pj2, jv.cpu().numpy(), ph2, hv.cpu().numpy(), reg)
    for pl in (None, plan):
        got = prob.assemble_kkt_mapped(*maps, jv, hv, _dev(reg)[0], plan=pl).cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    prob.close()
    del got, want, jv, hv
    torch.cuda.empty_cache()
    _say("[mapped] synthetic N=1e5")
    N, n, m = synth.IPM_LOOP
    inst = synth.make_instance(N, n, m, seed=0)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y = _dev(inst.z, inst.y)
    jv, hv = prob.jac(z), prob.hess(z, y, 1.0)
    rp, ci, pj, ph = ocp.kkt_pattern(N, n, m)
    rp2, ci2, pj2, ph2, dg2 = ocp.kkt_permute(rp, ci, pj, ph, ocp.stage_order(N, n, m))
    got = prob.assemble_kkt_mapped(*_dev(pj2, ph2, dg2), jv, hv).cpu().numpy()
    want = oracle.assemble_mapped(rp2[-1], dg2, pj2, jv.cpu().numpy(), ph2, hv.cpu().numpy(), None)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    prob.close()


def test_stale_plan_gives_oracle_values(ocp):
    """A plan made from other slot maps (another ordering, or the handle's
    cached plan when new maps reuse the old addresses) is caught per tile:
    the values are still the oracle's, bit for bit."""
    dev = torch.device("cuda", 0)
    for N, n, m, scheme, bnd in [(300, 5, 3, 0, 2), (1000, 16, 8, 1, 1)]:
        _say(f"[mapped stale plan] N={N} n={n} m={m}")
        inst = synth.make_instance(N, n, m, seed=34, scheme=scheme, bnd=bnd)
        prob = ocp.Problem.from_instance(inst, dev)
        z, y = _dev(inst.z, inst.y)
        jv, hv = prob.jac(z), prob.hess(z, y, 1.0)
        rp, ci, pj, ph = ocp.kkt_pattern(N, n, m, scheme=scheme, boundary=bnd)
        dim = len(rp) - 1
        reg = np.random.default_rng(5).normal(size=dim)
        stage = ocp.stage_order(N, n, m, scheme, bnd)
        rng = np.random.default_rng(6)
        # the stage order with its node runs shuffled: still node-grouped, but
        # every tile's range moves, so a plan of the stage order is stale
        shuffled = stage.copy()
        swap = rng.choice(dim, size=dim // 50, replace=False)
        shuffled[np.sort(swap)] = shuffled[swap]
        mapsA = ocp.kkt_permute(rp, ci, pj, ph, stage)
        mapsB = ocp.kkt_permute(rp, ci, pj, ph, shuffled)
        dA = _dev(*mapsA[2:5])
        planA = prob.mapped_plan(*dA)
        dB = _dev(*mapsB[2:5])
        want = oracle.assemble_mapped(mapsB[0][-1], mapsB[4], mapsB[2], jv.cpu().numpy(), mapsB[3],
                                      hv.cpu().numpy(), reg)
        got = prob.assemble_kkt_mapped(*dB, jv, hv, _dev(reg)[0], plan=planA).cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), "explicit stale plan"
        # the handle's cached plan: first keyed to A's maps, then B's maps are
        # written into A's arrays (same addresses, stale plan)
        prob.assemble_kkt_mapped(*dA, jv, hv, _dev(reg)[0])
        for a, b in zip(dA, dB):
            a.copy_(b)
        got = prob.assemble_kkt_mapped(*dA, jv, hv, _dev(reg)[0]).cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), "stale cached plan"
        # and the cached plan of the right maps
        got = prob.assemble_kkt_mapped(*dB, jv, hv, _dev(reg)[0]).cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), "cached plan"
        got = prob.assemble_kkt_mapped(*dB, jv, hv, _dev(reg)[0]).cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), "cached plan, reused"
        prob.close()
