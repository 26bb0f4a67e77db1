"""Batched evaluation on the GPU: many instances with uneven N in one
persistent launch, the per-instance launches it replaces, HIP-graph replay,
and the autotuner.  Every instance's values must match the CPU oracle
(1e-12 * mu) and be bitwise those of the single-instance path, for every mode
and tile shape."""
from __future__ import annotations

import itertools
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import check_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SMALL_NS = [1, 2, 3, 17, 256, 257, 511, 513, 1000, 1001]


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


def _bits(t):
    return t.view(torch.int64)


def _setup(ocp, insts):
    dev = torch.device("cuda", 0)
    batch = ocp.Batch.from_instances(insts, dev)
    zp, yp = synth.pack(insts)
    return batch, torch.from_numpy(zp).to(dev), torch.from_numpy(yp).to(dev)


@pytest.mark.parametrize("n,m", [(6, 3), (1, 0), (2, 1), (16, 8), (32, 32)])
def test_batch_matches_oracle_and_single_path(ocp, n, m):
    _say(f"[batch] n={n} m={m}")
    insts = synth.make_batch(len(SMALL_NS), n, m, seed=3, Ns=SMALL_NS)
    batch, z, y = _setup(ocp, insts)
    jac, hess = batch.eval(z, y, 1.0)
    torch.cuda.synchronize()
    off = batch.offsets
    dev = z.device
    for b, inst in enumerate(insts):
        jb = jac[off["jac"][b]:off["jac"][b + 1]]
        hb = hess[off["hess"][b]:off["hess"][b + 1]]
        want, mu = oracle.jac(inst)
        check_close(jb.cpu().numpy(), want, mu, what=f"jac b={b}")
        want, mu = oracle.hess(inst)
        check_close(hb.cpu().numpy(), want, mu, what=f"hess b={b}")
        prob = ocp.Problem.from_instance(inst, dev)
        zs = torch.from_numpy(inst.z).to(dev)
        ys = torch.from_numpy(inst.y).to(dev)
        assert torch.equal(_bits(prob.jac(zs)), _bits(jb))
        assert torch.equal(_bits(prob.hess(zs, ys, 1.0)), _bits(hb))
        prob.close()
    batch.close()


def test_batch_modes_shapes_and_alignment_bitwise(ocp):
    """Persistent launch under every tile shape the autotuner tries, the
    per-instance launches, and a misaligned Jacobian output all agree bitwise."""
    insts = synth.make_batch(len(SMALL_NS), 6, 3, seed=4, Ns=SMALL_NS)
    batch, z, y = _setup(ocp, insts)
    ref_j, ref_h = batch.eval(z, y, 0.7, mode="per_instance")
    for block, pair, wpc, order in itertools.product((128, 256), (0, 1), (0, 1, 2, 4, 8, 16, 32),
                                                     (0, 1)):
        batch.config = {"block": block, "pair": pair, "wgs_per_cu": wpc, "order": order}
        j, h = batch.eval(z, y, 0.7)
        assert torch.equal(_bits(j), _bits(ref_j)), (block, pair, wpc, order)
        assert torch.equal(_bits(h), _bits(ref_h)), (block, pair, wpc, order)
    batch.config = {"block": 256, "pair": 1, "wgs_per_cu": 8, "order": 0}
    tot = int(batch.offsets["jac"][-1])
    buf = torch.empty(tot + 1, dtype=torch.float64, device=z.device)
    j, _ = batch.eval(z, y, 0.7, jac=buf[1:], what=1)
    assert j.data_ptr() % 16 == 8
    assert torch.equal(_bits(j), _bits(ref_j))
    j, _ = batch.eval(z, y, 0.7, jac=buf[1:], what=1, mode="per_instance")
    assert torch.equal(_bits(j), _bits(ref_j))
    _, h = batch.eval(z, y, 0.7, what=2)
    assert torch.equal(_bits(h), _bits(ref_h))
    batch.close()


@pytest.mark.parametrize("mode", ["persistent", "per_instance"])
def test_batch_graph_replays(ocp, mode):
    """A captured graph replays correctly several times, with eager work and
    synchronizations between replays and new values written into its bound
    input between them."""
    insts = synth.make_batch(len(SMALL_NS), 6, 3, seed=5, Ns=SMALL_NS)
    batch, z, y = _setup(ocp, insts)
    g, gj, gh = batch.graph(z, y, 1.0, mode=mode)
    for rep in range(4):
        if rep:
            z.mul_(0.9).add_(0.05)   # eager work that changes the bound input
            y.neg_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        ej, eh = batch.eval(z, y, 1.0)
        torch.cuda.synchronize()
        assert torch.equal(_bits(gj), _bits(ej)), rep
        assert torch.equal(_bits(gh), _bits(eh)), rep
    batch.close()
    # the graph reads the batch's coefficients: once the batch is closed the
    # binding refuses to replay it (on the host, before any GPU work)
    with pytest.raises(ocp.OcpError) as e:
        g.launch()
    assert e.value.code == ocp.OCP_ERR_ARG
    g.close()


def test_batch_autotune_and_cache(ocp, tmp_path):
    insts = synth.make_batch(len(SMALL_NS), 6, 3, seed=6, Ns=SMALL_NS)
    batch, z, y = _setup(ocp, insts)
    ref_j, ref_h = batch.eval(z, y, 1.0)
    path = str(tmp_path / "tune.json")
    cfg, ms = batch.autotune(z, y, 1.0, reps=2, cache=path)
    assert cfg["block"] in (128, 256) and cfg["pair"] in (0, 1)
    assert cfg["wgs_per_cu"] in (0, 1, 2, 4, 8, 16, 32) and cfg["order"] in (0, 1)
    assert ms > 0
    assert batch.config == cfg
    batch.config = {"block": 128, "pair": 0, "wgs_per_cu": 1, "order": 0}
    cfg2, ms2 = batch.autotune(z, y, 1.0, reps=2, cache=path)   # served from the cache
    assert cfg2 == cfg and ms2 == ms and batch.config == cfg
    j, h = batch.eval(z, y, 1.0)
    assert torch.equal(_bits(j), _bits(ref_j)) and torch.equal(_bits(h), _bits(ref_h))
    batch.close()


def test_batched_workload_512_instances(ocp):
    """512 instances, N_b ~ U{200..20000}, n = 6, m = 3: the persistent launch
    equals the per-instance launches bitwise; sampled instances match the oracle."""
    _say("[batch] 512-instance workload")
    insts = synth.make_batch(512, 6, 3, seed=0)
    batch, z, y = _setup(ocp, insts)
    pj, ph = batch.eval(z, y, 1.0)
    qj, qh = batch.eval(z, y, 1.0, mode="per_instance")
    assert torch.equal(_bits(pj), _bits(qj)) and torch.equal(_bits(ph), _bits(qh))
    off = batch.offsets
    for b in (0, 1, 255, 511, int(np.argmax([i.N for i in insts])), int(np.argmin([i.N for i in insts]))):
        want, mu = oracle.jac(insts[b])
        check_close(pj[off["jac"][b]:off["jac"][b + 1]].cpu().numpy(), want, mu, what=f"jac b={b}")
        want, mu = oracle.hess(insts[b])
        check_close(ph[off["hess"][b]:off["hess"][b + 1]].cpu().numpy(), want, mu, what=f"hess b={b}")
    batch.close()
