"""Batched evaluation of a whole interior-point step on the GPU: objective,
gradient, defects (with boundary rows), Jacobian, Hessian of the Lagrangian
and the fused KKT values of many instances with uneven N, under both
schemes and the boundary options, in one persistent launch.  Every
instance's outputs must match the CPU oracle (1e-12 * mu; the KKT values
against the oracle's own assembly of its Jacobian and Hessian) and be
bitwise those of the per-instance launches, for every tile shape and every
subset of the evaluations; graph replays repeat the eager result bit for bit."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import check_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SMALL_NS = [1, 2, 3, 17, 256, 257, 511, 513, 1000, 1001]
OUTS = ("obj", "grad", "cons", "jac", "hess", "kkt")


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


def _setup(ocp, insts, scheme, bnd, seed=9):
    dev = torch.device("cuda", 0)
    batch = ocp.Batch.from_instances(insts, dev, scheme=scheme, boundary=bnd)
    zp, yp = synth.pack(insts)
    reg = np.random.default_rng(seed).normal(size=int(batch.offsets["dim"][-1]))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return batch, t(zp), t(yp), t(reg), reg


def _bits(t):
    return t.contiguous().view(torch.int64)


def _slices(batch, b):
    off = batch.offsets
    key = {"grad": "z", "cons": "c", "jac": "jac", "hess": "hess", "kkt": "kkt"}
    out = {"obj": slice(b, b + 1)}
    for name, k in key.items():
        out[name] = slice(int(off[k][b]), int(off[k][b + 1]))
    return out


def _check_against_oracle(ocp, batch, insts, got, reg, sigma, scheme, bnd, tag):
    dim = batch.offsets["dim"]
    for b, inst in enumerate(insts):
        sl = _slices(batch, b)
        g = {k: got[k][sl[k]].cpu().numpy() for k in OUTS}
        f, fmu = oracle.obj_ex(inst, scheme, bnd)
        check_close(g["obj"], np.array([f]), np.array([fmu]), what=f"obj {tag} b={b}")
        for name, fn in (("grad", oracle.grad_ex), ("cons", oracle.cons_ex), ("jac", oracle.jac_ex)):
            want, mu = fn(inst, scheme, bnd)
            check_close(g[name], want, mu, what=f"{name} {tag} b={b}")
        oh, mh = oracle.hess_ex(inst, scheme, bnd, sigma=sigma)
        check_close(g["hess"], oh, mh, what=f"hess {tag} b={b}")
        oj, mj = oracle.jac_ex(inst, scheme, bnd)
        rp, _, pj, ph = ocp.kkt_pattern(inst.N, inst.n, inst.m, colind=False, scheme=scheme, boundary=bnd)
        rb = reg[int(dim[b]):int(dim[b + 1])]
        want = oracle.assemble(rp, pj, oj, ph, oh, rb)
        mu = oracle.assemble(rp, pj, mj, ph, mh, np.abs(rb))
        check_close(g["kkt"], want, mu, what=f"kkt {tag} b={b}")


@pytest.mark.parametrize("n,m,scheme,bnd", [(6, 3, 0, 0), (6, 3, 0, 2), (6, 3, 1, 1), (2, 1, 1, 0),
                                            (1, 0, 0, 1), (16, 8, 0, 0), (16, 8, 1, 2), (3, 2, 0, 2)])
def test_whole_step_matches_oracle_and_per_instance(ocp, n, m, scheme, bnd):
    _say(f"[batch step] n={n} m={m} scheme={scheme} bnd={bnd}")
    insts = synth.make_batch(len(SMALL_NS), n, m, seed=5, Ns=SMALL_NS, scheme=scheme, bnd=bnd)
    batch, z, y, regt, reg = _setup(ocp, insts, scheme, bnd)
    sigma = 0.7
    got = batch.step(z, y, sigma, regt, what=ocp.EVAL_ALL, mode="persistent")
    ref = batch.step(z, y, sigma, regt, what=ocp.EVAL_ALL, mode="per_instance")
    torch.cuda.synchronize()
    for k in OUTS:
        assert torch.equal(_bits(got[k]), _bits(ref[k])), f"{k}: persistent differs from per-instance"
    _check_against_oracle(ocp, batch, insts, got, reg, sigma, scheme, bnd, f"n={n} m={m} s={scheme} b={bnd}")
    batch.close()


SHAPES = [dict(block=128, pair=0, wgs_per_cu=0, order=0), dict(block=128, pair=1, wgs_per_cu=2, order=1),
          dict(block=256, pair=0, wgs_per_cu=1, order=1), dict(block=256, pair=1, wgs_per_cu=32, order=0)]


@pytest.mark.parametrize("scheme,bnd", [(0, 2), (1, 1)])
def test_every_tile_shape_and_subset_is_bitwise_identical(ocp, scheme, bnd):
    _say(f"[batch step shapes] scheme={scheme} bnd={bnd}")
    Ns = SMALL_NS + [100_000, 4097]  # 100000: 391 objective tiles, two partials per virtual lane
    insts = synth.make_batch(len(Ns), 6, 3, seed=6, Ns=Ns, scheme=scheme, bnd=bnd)
    batch, z, y, regt, _ = _setup(ocp, insts, scheme, bnd)
    ref = batch.step(z, y, 1.3, regt, what=ocp.EVAL_ALL, mode="per_instance")
    subsets = [ocp.EVAL_ALL, ocp.EVAL_OBJ, ocp.EVAL_CONS | ocp.EVAL_GRAD, ocp.EVAL_KKT,
               ocp.EVAL_JAC | ocp.EVAL_CONS | ocp.EVAL_OBJ]
    for shape in SHAPES:
        batch.config = shape
        for what in subsets:
            got = batch.step(z, y, 1.3, regt, what=what, mode="persistent")
            torch.cuda.synchronize()
            for k, bit in zip(OUTS, (ocp.EVAL_OBJ, ocp.EVAL_GRAD, ocp.EVAL_CONS, ocp.EVAL_JAC,
                                     ocp.EVAL_HESS, ocp.EVAL_KKT)):
                if what & bit:
                    assert torch.equal(_bits(got[k]), _bits(ref[k])), f"{k}: shape {shape} what {what}"
                else:
                    assert got[k] is None
    batch.close()


def test_graph_replays_repeat_the_eager_step(ocp):
    _say("[batch step graph]")
    insts = synth.make_batch(len(SMALL_NS), 6, 3, seed=7, Ns=SMALL_NS, scheme=0, bnd=1)
    batch, z, y, regt, _ = _setup(ocp, insts, 0, 1)
    eager = batch.step(z, y, 1.0, regt, what=ocp.EVAL_ALL)
    eager = {k: v.clone() for k, v in eager.items()}
    outs = {k: torch.full_like(v, float("nan")) for k, v in eager.items()}
    for mode in ("persistent", "per_instance"):
        g = batch.step_graph(z, y, 1.0, regt, what=ocp.EVAL_ALL, mode=mode, out=outs)
        for rep in range(3):
            for v in outs.values():
                v.fill_(float("nan"))
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            # eager work between replays
            batch.step(z, y, 1.0, regt, what=ocp.EVAL_OBJ)
            torch.cuda.synchronize()
            for k in OUTS:
                assert torch.equal(_bits(outs[k]), _bits(eager[k])), f"{mode} replay {rep}: {k}"
        g.close()
    batch.close()


def test_bad_arguments_are_refused(ocp):
    insts = synth.make_batch(3, 4, 2, seed=8, Ns=[5, 6, 7])
    batch, z, y, regt, _ = _setup(ocp, insts, 0, 0)
    with pytest.raises(ocp.OcpError):
        batch.step(z, None, 1.0, None, what=ocp.EVAL_HESS)  # y missing
    with pytest.raises(ocp.OcpError):
        batch.step(z, y, float("nan"), None, what=ocp.EVAL_KKT)
    with pytest.raises(ocp.OcpError):
        batch.step(z, y, 1.0, None, what=64)
    batch.close()
