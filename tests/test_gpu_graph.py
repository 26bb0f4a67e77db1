"""The evaluation calls captured in a HIP graph (torch.cuda.CUDAGraph on the
current stream, which the binding passes to the library): none of them
allocates or clears memory with a memset, so a whole step can be captured
once and replayed.  Each replay runs at a new point copied into the captured
input tensors, with eager evaluations of the same point between the replays,
and every output of every replay must equal the eager one bit for bit (the
kernels and their reduction orders are the same)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import synth

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
    ocp.lib()
    return ocp


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def _outputs(prob, fused):
    s = prob.sizes
    f64 = dict(dtype=torch.float64, device=torch.device("cuda", 0))
    names = {"obj": 1, "grad": s["nvar"], "cons": s["ncon"], "jac": s["nnzj"], "hess": s["nnzh"],
             "kkt": s["nnzk"]}
    if fused:
        names["kkt_fused"] = s["nnzk"]
    return {k: torch.full((v,), float("nan"), **f64) for k, v in names.items()}


def _step(prob, maps, z, y, reg, o, fused):
    pj, ph, rp = maps
    prob.obj(z, out=o["obj"])
    prob.grad(z, out=o["grad"])
    prob.cons(z, out=o["cons"])
    prob.jac(z, out=o["jac"])
    prob.hess(z, y, 0.8, out=o["hess"])
    prob.assemble_kkt(pj, ph, rp, o["jac"], o["hess"], reg, out=o["kkt"])
    if fused:
        prob.eval_kkt(z, y, 0.8, reg, out=o["kkt_fused"])


def _points(make, count):
    return [make(seed) for seed in range(100, 100 + count)]


def _run(ocp, prob, pattern, points, fused):
    dev = torch.device("cuda", 0)
    rowptr, _, perm_j, perm_h = pattern
    maps = tuple(_t(a) for a in (perm_j, perm_h, rowptr))
    reg = torch.linspace(1e-6, 2e-6, prob.sizes["dim"], dtype=torch.float64, device=dev)
    zs, ys = _t(points[0][0]).clone(), _t(points[0][1]).clone()
    outs = _outputs(prob, fused)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        _step(prob, maps, zs, ys, reg, outs, fused)
    torch.cuda.synchronize()
    for r, (z, y) in enumerate(points):
        ref = _outputs(prob, fused)
        _step(prob, maps, _t(z), _t(y), reg, ref, fused)  # eager, same point
        torch.cuda.synchronize()
        zs.copy_(_t(z))
        ys.copy_(_t(y))
        g.replay()
        torch.cuda.synchronize()
        for k in outs:
            assert torch.equal(outs[k].view(torch.int64), ref[k].view(torch.int64)), (r, k)
        assert not torch.isnan(outs["kkt"]).any()
    del g


def test_calls_go_to_the_current_stream(ocp):
    """The binding hands every call torch's current stream: its stream query
    gives the same handle as torch's public one on the default stream and
    inside a side stream's context, and a call issued there is ordered on that
    stream (its result is complete after the stream alone synchronizes)."""
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(5000, 6, 3, seed=3)
    prob = ocp.Problem.from_instance(inst, dev)
    handle = lambda: prob._stream().value or 0  # the null stream's handle is 0 (None as a c_void_p)
    assert handle() == torch.cuda.current_stream(dev).cuda_stream
    z = _t(inst.z)
    want = prob.cons(z)
    torch.cuda.synchronize()
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        assert handle() == side.cuda_stream != torch.cuda.default_stream(dev).cuda_stream
        got = prob.cons(z)
    side.synchronize()
    assert torch.equal(got.view(torch.int64), want.view(torch.int64))
    prob.close()


def test_evaluations_on_one_handle_overlap(ocp):
    """Evaluations that use no handle workspace may run concurrently on
    different streams: the Jacobian and the defects on one stream,
    overlapping the Hessian, grad_z L, H v and J v on another, give the bits
    of the same calls run one after another."""
    _say("[streams] overlapping evaluations on one handle")
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(50_000, 8, 4, seed=21, scheme=0, bnd=1)
    prob = ocp.Problem.from_instance(inst, dev)
    z, y = _t(inst.z), _t(inst.y)
    v = _t(np.random.default_rng(2).normal(size=prob.sizes["nvar"]))
    first = lambda: (prob.jac(z), prob.cons(z))
    second = lambda: (prob.hess(z, y, 0.6), prob.lag_grad(z, y, 0.6), prob.hvp(z, y, v, 0.6), prob.jvp(z, v))
    want = first() + second()
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(dev), torch.cuda.Stream(dev)  # default priority
    got = []
    for _ in range(5):
        with torch.cuda.stream(s1):
            a = first()
        with torch.cuda.stream(s2):
            b = second()
        got.append(a + b)
    torch.cuda.synchronize()
    for outs in got:
        for g, w in zip(outs, want):
            assert torch.equal(g.view(torch.int64), w.view(torch.int64))
    prob.close()


@pytest.mark.parametrize("N,n,m,scheme,bnd", [(3000, 6, 3, 0, 0), (1001, 16, 8, 0, 1), (777, 5, 2, 1, 2)])
def test_graph_replays_equal_eager_synthetic(ocp, N, n, m, scheme, bnd):
    _say(f"[graph] synthetic N={N} n={n} m={m} scheme={scheme} bnd={bnd}")
    base = synth.make_instance(N, n, m, seed=61, scheme=scheme, bnd=bnd)
    prob = ocp.Problem.from_instance(base, torch.device("cuda", 0))

    def point(seed):
        other = synth.make_instance(N, n, m, seed=seed, scheme=scheme, bnd=bnd)
        return other.z, other.y

    pattern = ocp.kkt_pattern(N, n, m, scheme=scheme, boundary=bnd, colind=False)
    _run(ocp, prob, pattern, _points(point, 3), fused=True)
    prob.close()


@pytest.mark.parametrize("N,bnd", [(2000, 1), (333, 0)])
def test_graph_replays_equal_eager_quadrotor(ocp, N, bnd):
    _say(f"[graph] quadrotor N={N} bnd={bnd}")
    prob = ocp.QuadrotorProblem.from_instance(synth.make_quadrotor(N, seed=62, bnd=bnd),
                                              torch.device("cuda", 0))

    def point(seed):
        q = synth.make_quadrotor(N, seed=seed, bnd=bnd)
        return q.z, q.y

    pattern = ocp.quad_kkt_pattern(N, bnd, colind=False)
    _run(ocp, prob, pattern, _points(point, 3), fused=True)
    prob.close()


def _diff_outputs(prob, coef):
    s = prob.sizes
    f64 = dict(dtype=torch.float64, device=torch.device("cuda", 0))
    o = {"L": torch.full((1,), float("nan"), **f64)}
    for k in ("g", "hv"):
        o[k] = torch.full((s["nvar"],), float("nan"), **f64)
    o["jv"] = torch.full((s["ncon"],), float("nan"), **f64)
    if coef:
        n, m = prob.n, prob.m
        for tag in ("cg", "cm", "cn"):
            o[tag] = (torch.full((n, n), float("nan"), **f64), torch.full((n, m), float("nan"), **f64),
                      torch.full((n,), float("nan"), **f64))
        o["az"] = torch.full((s["nvar"],), float("nan"), **f64)
        o["ay"] = torch.full((s["ncon"],), float("nan"), **f64)
    return o


def _diff_calls(prob, z, y, v, o, coef):
    prob.lagrangian(z, y, 0.7, out=o["L"])
    prob.lag_grad(z, y, 0.7, out=o["g"])
    prob.hvp(z, y, v, 0.7, out=o["hv"])
    prob.jvp(z, v, out=o["jv"])
    if coef:
        prob.coef_grad(z, y, out=o["cg"])
        prob.coef_mixed(z, y, v, out=o["cm"])
        prob.coef_grad(z, y, noalloc=True, out=o["cn"])
        # the adjoint, with the coefficient gradient just computed as cotangents
        prob.coef_adjoint(z, y, *o["cg"], out_z=o["az"], out_y=o["ay"])


def _flat(o):
    out = {}
    for k, t in o.items():
        if isinstance(t, tuple):
            for i, u in enumerate(t):
                out[f"{k}{i}"] = u
        else:
            out[k] = t
    return out


@pytest.mark.parametrize("model,scheme,bnd", [("synthetic", 0, 0), ("synthetic", 1, 2), ("quadrotor", 0, 1)])
def test_graph_replays_equal_eager_differentiation(ocp, model, scheme, bnd):
    """The Lagrangian entry points (L, grad_z L, H v, J v and, for the
    synthetic family, the coefficient gradient, its mixed derivative, the
    allocation-free coefficient gradient and the adjoint fed by the first)
    captured in one graph: each replay at a new point equals the eager calls
    bit for bit."""
    _say(f"[graph] differentiation {model} scheme={scheme} bnd={bnd}")
    dev = torch.device("cuda", 0)
    coef = model == "synthetic"
    if coef:
        make = lambda seed: synth.make_instance(900, 6, 3, seed=seed, scheme=scheme, bnd=bnd)
        prob = ocp.Problem.from_instance(make(70), dev)
    else:
        make = lambda seed: synth.make_quadrotor(700, seed=seed, bnd=bnd)
        prob = ocp.QuadrotorProblem.from_instance(make(70), dev)
    rng = np.random.default_rng(5)
    first = make(100)
    zs, ys = _t(first.z).clone(), _t(first.y).clone()
    vs = _t(rng.normal(size=prob.sizes["nvar"])).clone()
    outs = _diff_outputs(prob, coef)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        _diff_calls(prob, zs, ys, vs, outs, coef)
    torch.cuda.synchronize()
    for r, seed in enumerate((100, 101, 102)):
        p = make(seed)
        v = _t(rng.normal(size=prob.sizes["nvar"]))
        ref = _diff_outputs(prob, coef)
        _diff_calls(prob, _t(p.z), _t(p.y), v, ref, coef)  # eager, same point
        torch.cuda.synchronize()
        zs.copy_(_t(p.z))
        ys.copy_(_t(p.y))
        vs.copy_(v)
        g.replay()
        torch.cuda.synchronize()
        fo, fr = _flat(outs), _flat(ref)
        for k in fo:
            assert torch.equal(fo[k].view(torch.int64), fr[k].view(torch.int64)), (r, k)
    del g
    prob.close()
