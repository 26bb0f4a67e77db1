"""Benchmark of the evaluation path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-ipm-loop] [--no-batched] [--no-diff] [--no-euler] [--no-quad] [--only-quad] [--no-reorder] [--only-reorder] [--no-fused]

Workload: the large single instance -- N = 1e6 intervals, n = 16 states, m = 8
controls, dense 16 x 16 A, FP64, synthetic seeded inputs (numpy PCG64, seed 0)
already resident in HBM.  One step is one pass of the whole device path:
eval_obj, eval_grad, eval_cons, eval_jac, eval_hess(sigma = 1) and
assemble_kkt (with a regularization diagonal).  The KKT structure and slot maps
are built once on the host before timing (the one-time symbolic step).

Prints ONE JSON line.  `value` is the headline metric, FP64 Jacobian + Hessian
nonzeros per second: (nnzj + nnzh) / (eval_jac + eval_hess time), measured
with HIP events on the stream the kernels run on, over the K timed steps.
`ms_per_step` is the wall time of one whole step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
CSRC = os.path.join(ROOT, "paper_2510_03932_amd", "csrc")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_large.json")


def sources_sha256() -> str:
    """SHA-256 over every source file of the library (sorted by name): the
    committed traffic counters apply only while it is unchanged."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(s, N, n, m):
    """Bytes each call must move (reads + writes), counting only the parts of
    z each call reads."""
    nx = n * (N + 1)
    return {
        "eval_obj": 8 * s["nvar"],
        "eval_grad": 16 * s["nvar"],
        "eval_cons": 8 * s["nvar"] + 8 * s["ncon"],
        "eval_jac": 8 * s["nnzj"] + 8 * nx,
        "eval_hess": 8 * s["nnzh"] + 8 * nx + 8 * s["ncon"],
        # perm (4 B) + value (8 B) per COO entry, the KKT values, the reg
        # diagonal, and rowptr at the constraint rows
        "assemble_kkt": 12 * (s["nnzj"] + s["nnzh"]) + 8 * s["nnzk"] + 8 * s["dim"] + 4 * s["ncon"],
    }


def cpu_model() -> str:
    """The host CPU's model name, from lscpu (falling back to /proc/cpuinfo)."""
    import subprocess
    names = []
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        names += [ln.split(":", 1)[1].strip() for ln in out.splitlines() if ln.startswith("Model name")]
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            names += [ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")][:1]
    except OSError:
        pass
    return max(names, key=len) if names else "unknown"


def cpu_baseline(inst, synth, target_s=4.0):
    """The oracle's Jacobian + Hessian timed on the host cores (wall time,
    median of repetitions):
      - the large workload (N = 1e6, n = 16, m = 8) on a bounded slice,
        intervals [0, K) for the Jacobian and nodes [0, K) for the Hessian,
        K chosen so one repetition takes about target_s; median of 3, on all
        OpenMP threads and on one thread;
      - the 1000-interval parity workload and the 1e5-interval
        interior-point-loop workload in full, median of 10, all threads."""
    import oracle
    oracle.build(force=False)
    threads = oracle.get_threads()
    N = inst.N
    T = 2 * inst.n + 2 * inst.m
    S = oracle.sizes(inst.N, inst.n, inst.m)["S"]

    def run(K, reps):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.jac(inst, 0, K)
            oracle.hess(inst, 0, K)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    K = 2000
    dt = run(K, 1)
    K = int(min(N, max(K, K * target_s / max(dt, 1e-6))))
    dt = run(K, 3)
    nnz = K * inst.n * T + K * S
    # the same on one thread, over a slice sized for about a tenth of target_s
    K1 = max(1000, min(N, int(K * (target_s / 10) / max(dt * threads, 1e-6))))
    oracle.set_threads(1)
    try:
        dt1 = run(K1, 3)
    finally:
        oracle.set_threads(threads)
    nnz1 = K1 * inst.n * T + K1 * S
    small = {}
    for name, (Ns, ns, ms) in (("parity_N1e3_n4_m2", synth.PARITY), ("ipm_loop_N1e5_n8_m4", synth.IPM_LOOP)):
        si = synth.make_instance(Ns, ns, ms, seed=0)
        ts = []
        for _ in range(10):
            t0 = time.perf_counter()
            oracle.jac(si)
            oracle.hess(si)
            ts.append(time.perf_counter() - t0)
        sz = oracle.sizes(Ns, ns, ms)
        small[name] = {"median_s": round(float(np.median(ts)), 6),
                       "nnz_per_s": (sz["nnzj"] + sz["nnzh"]) / float(np.median(ts)), "reps": 10}
    return {"value": nnz / dt, "unit": "nonzeros/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle jac on intervals [0,{K}) + hess on nodes [0,{K}) of the "
                      f"N={N} n={inst.n} m={inst.m} workload ({nnz} nonzeros), median of 3 "
                      f"repetitions ({dt:.2f} s each), OpenMP threads={threads}",
            "single_thread_value": nnz1 / dt1,
            "single_thread_sample": f"intervals/nodes [0,{K1}), {nnz1} nonzeros, median of 3 "
                                    f"repetitions ({dt1:.2f} s each)",
            "full_workloads": small,
            "cpu_model": cpu_model(),
            "seconds": dt}


def ipm_loop(torch, ocp, synth, iters=50):
    """The interior-point-loop workload: N = 1e5, n = 8, m = 4, coefficients
    from seed 0; each iteration evaluates cons + jac + hess + assemble_kkt at a
    fresh point drawn on the device (seed 1000 + it) outside the timed region.
    Its Jacobian + Hessian values (169 MB) fit in the 256 MiB Infinity Cache,
    so the figure may be cache-assisted."""
    N, n, m = synth.IPM_LOOP
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=0)
    prob = ocp.Problem.from_instance(inst, dev)
    s = prob.sizes
    rowptr, _, perm_j, perm_h = ocp.kkt_pattern(N, n, m, colind=False)
    pj, ph, rp = (torch.from_numpy(a).to(dev) for a in (perm_j, perm_h, rowptr))
    reg = torch.full((s["dim"],), 1e-8, dtype=torch.float64, device=dev)
    f64 = dict(dtype=torch.float64, device=dev)
    c = torch.empty(s["ncon"], **f64)
    jv = torch.empty(s["nnzj"], **f64)
    hv = torch.empty(s["nnzh"], **f64)
    kkt = torch.empty(s["nnzk"], **f64)
    times = []
    for it in range(iters + 3):
        z, y = synth.device_point(torch, dev, N, n, m, 1000 + (it % iters))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        prob.cons(z, out=c)
        prob.jac(z, out=jv)
        prob.hess(z, y, 1.0, out=hv)
        prob.assemble_kkt(pj, ph, rp, jv, hv, reg, out=kkt)
        e1.record()
        torch.cuda.synchronize()
        if it >= 3:  # the first three are warm-up
            times.append(e0.elapsed_time(e1))
    # the same four calls captured once in a HIP graph and replayed, each
    # iteration's point copied into the captured inputs outside the timing
    zs, ys = synth.device_point(torch, dev, N, n, m, 1000)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        prob.cons(zs, out=c)
        prob.jac(zs, out=jv)
        prob.hess(zs, ys, 1.0, out=hv)
        prob.assemble_kkt(pj, ph, rp, jv, hv, reg, out=kkt)
    gtimes = []
    for it in range(iters + 3):
        z, y = synth.device_point(torch, dev, N, n, m, 1000 + (it % iters))
        zs.copy_(z)
        ys.copy_(y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        if it >= 3:
            gtimes.append(e0.elapsed_time(e1))
    del graph
    prob.close()
    ms = float(np.median(times))
    gms = float(np.median(gtimes))
    return {"workload": f"N={N} n={n} m={m}, {iters} iterations of cons+jac+hess+assemble_kkt "
                        "at fresh device-drawn points",
            "ms_per_iteration": round(ms, 4),
            "mean_ms": round(float(np.mean(times)), 4),
            "p10_ms": round(float(np.percentile(times, 10)), 4),
            "p90_ms": round(float(np.percentile(times, 90)), 4),
            "jac_hess_nnz_per_s_in_loop": (s["nnzj"] + s["nnzh"]) / (ms * 1e-3),
            "graph_ms_per_iteration": round(gms, 4),
            "graph_p10_ms": round(float(np.percentile(gtimes, 10)), 4),
            "graph_p90_ms": round(float(np.percentile(gtimes, 90)), 4),
            "note": "J+H values fit in the 256 MiB Infinity Cache"}


def batched(torch, ocp, synth, reps=10):
    """The batched workload: 512 instances, N_b ~ U{200..20000}, n = 6, m = 3.

    Jacobian + Hessian values of all of them, four ways: one single-instance
    launch per instance and evaluation (1024 launches), the same captured in a
    HIP graph, the batched launch over the tile list (after autotuning its tile
    shape), and that launch replayed from a graph.  Then the whole
    interior-point step (objective, gradient, defects and the fused KKT
    values of every instance) batched against per-instance launches, and the
    same with the COO Jacobian and Hessian values added."""
    import tempfile
    insts = synth.make_batch(512, 6, 3, seed=0)
    dev = torch.device("cuda", 0)
    batch = ocp.Batch.from_instances(insts, dev)
    zp, yp = synth.pack(insts)
    z = torch.from_numpy(zp).to(dev)
    y = torch.from_numpy(yp).to(dev)
    tot = {k: int(v[-1]) for k, v in batch.offsets.items()}
    jac = torch.empty(tot["jac"], dtype=torch.float64, device=dev)
    hess = torch.empty(tot["hess"], dtype=torch.float64, device=dev)
    nnz = tot["jac"] + tot["hess"]
    nx = sum(i.n * (i.N + 1) for i in insts)
    nbytes = 8 * nnz + 8 * nx * 2 + 8 * tot["c"]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    res = {}
    res["per_instance_ms"] = timed(lambda: batch.eval(z, y, 1.0, jac, hess, mode="per_instance"))
    g1, _, _ = batch.graph(z, y, 1.0, jac, hess, mode="per_instance")
    res["per_instance_graph_ms"] = timed(g1.launch)
    g1.close()
    with tempfile.TemporaryDirectory() as td:
        cfg, tune_ms = batch.autotune(z, y, 1.0, jac, hess, reps=3, cache=os.path.join(td, "t.json"))
    table = batch.tuning
    looped = min((t for t in table if t["wgs_per_cu"] > 0), key=lambda t: t["ms"])
    res["batched_ms"] = timed(lambda: batch.eval(z, y, 1.0, jac, hess))
    g2, _, _ = batch.graph(z, y, 1.0, jac, hess)
    res["batched_graph_ms"] = timed(g2.launch)
    g2.close()
    out = {"workload": "512 instances, N_b ~ U{200..20000} (sum %d), n=6, m=3, jac+hess" % sum(
               i.N for i in insts),
           "nnz": nnz, "autotuned_config": cfg,
           "autotuned_grid": ("one workgroup per tile (the tile loop runs once)" if cfg["wgs_per_cu"] == 0
                              else "persistent: %d workgroups per CU loop over the tiles" % cfg["wgs_per_cu"]),
           "best_persistent_looping_shape": looped,
           "autotune_table_ms": {"%d/%d/%d/%d" % (t["block"], t["pair"], t["wgs_per_cu"], t["order"]):
                                 round(t["ms"], 4) for t in table}}
    for k, v in res.items():
        out[k] = round(v, 4)
        out[k.replace("_ms", "_nnz_per_s")] = nnz / (v * 1e-3)
    out["batched_graph_hbm_frac"] = round(nbytes / (res["batched_graph_ms"] * 1e-3) / HBM_PEAK, 4)
    out["speedup_batched_graph_vs_per_instance"] = round(res["per_instance_ms"] / res["batched_graph_ms"], 3)
    out["speedup_batched_graph_vs_per_instance_graph"] = round(
        res["per_instance_graph_ms"] / res["batched_graph_ms"], 3)
    del jac, hess

    # the whole interior-point step: objective, gradient, defects and the
    # fused KKT values (the matrix a step factorizes), and the same plus the
    # COO Jacobian and Hessian values
    nvar, ncon, dim = tot["z"], tot["c"], tot["dim"]
    reg = torch.full((dim,), 1e-8, dtype=torch.float64, device=dev)
    step_bytes = {  # algorithmic bytes of each part, summed over the instances
        ocp.EVAL_OBJ: 8 * nvar, ocp.EVAL_GRAD: 16 * nvar, ocp.EVAL_CONS: 8 * (nvar + ncon),
        ocp.EVAL_KKT: 8 * (nx + ncon + dim + tot["kkt"]),
        ocp.EVAL_JAC: 8 * (tot["jac"] + nx), ocp.EVAL_HESS: 8 * (tot["hess"] + nx + ncon)}
    masks = {"step_fused_kkt": ocp.EVAL_OBJ | ocp.EVAL_GRAD | ocp.EVAL_CONS | ocp.EVAL_KKT,
             "step_all": ocp.EVAL_ALL}
    for name, what in masks.items():
        outs = batch.step(z, y, 1.0, reg, what=what)  # allocates the outputs once
        sb = sum(v for bit, v in step_bytes.items() if what & bit)
        per = timed(lambda: batch.step(z, y, 1.0, reg, what=what, mode="per_instance", out=outs))
        gp = batch.step_graph(z, y, 1.0, reg, what=what, mode="per_instance", out=outs)
        per_g = timed(gp.launch)
        gp.close()
        cfg_s, _, tab = batch.autotune_step(z, y, 1.0, reg, what=what, reps=3, out=outs)
        bat = timed(lambda: batch.step(z, y, 1.0, reg, what=what, out=outs))
        gb = batch.step_graph(z, y, 1.0, reg, what=what, out=outs)
        bat_g = timed(gb.launch)
        gb.close()
        loop = min((t for t in tab if t["wgs_per_cu"] > 0), key=lambda t: t["ms"])
        # the parts of the step on their own, at the step's tuned shape
        parts = {}
        for pname, pw in (("obj_grad_cons", ocp.EVAL_OBJ | ocp.EVAL_GRAD | ocp.EVAL_CONS),
                          ("kkt", ocp.EVAL_KKT), ("jac_hess", ocp.EVAL_JAC | ocp.EVAL_HESS)):
            if what & pw == pw:
                pb = sum(v for bit, v in step_bytes.items() if pw & bit)
                pms = timed(lambda: batch.step(z, y, 1.0, reg, what=pw, out=outs))
                parts[pname] = {"ms": round(pms, 4), "bytes": pb,
                                "hbm_frac": round(pb / (pms * 1e-3) / HBM_PEAK, 4)}
        out[name] = {"what": what, "bytes": sb, "parts": parts,
                     "per_instance_ms": round(per, 4), "per_instance_graph_ms": round(per_g, 4),
                     "autotuned_config": cfg_s, "batched_ms": round(bat, 4),
                     "batched_graph_ms": round(bat_g, 4),
                     "best_persistent_looping_shape": loop,
                     "batched_graph_hbm_frac": round(sb / (bat_g * 1e-3) / HBM_PEAK, 4),
                     "speedup_batched_graph_vs_per_instance": round(per / bat_g, 3),
                     "speedup_batched_graph_vs_per_instance_graph": round(per_g / bat_g, 3)}
        del outs
    batch.close()
    return out


def _call_times(torch, fn, reps):
    """(eager ms, graph ms) per call: `reps` calls issued from Python between
    two HIP events, then the same `reps` calls captured in one HIP graph and
    replayed (median of 5 timed replays).  At small sizes the eager figure is bounded by Python's
    per-call dispatch (ctypes, argument checks); the graph figure is the
    device's time per call."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    eager = e0.elapsed_time(e1) / reps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(5):
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / reps)
    del g
    return eager, float(np.median(times))


def differentiation(torch, ocp, synth, reps=20):
    """The differentiation workload: N = 2e5, n = 8, m = 4.  Each Lagrangian
    entry point timed on its own (HIP events, mean of `reps`; eager calls and
    a replayed graph of the same calls, hbm_frac from the latter), then one
    autograd forward + backward of L(z, y) with gradients for z, y, A, B and
    gamma, and one Hessian-vector product."""
    from paper_2510_03932_amd.autograd import lagrangian
    N, n, m = synth.DIFF
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=0)
    prob = ocp.Problem.from_instance(inst, dev)
    s = prob.sizes
    z = torch.from_numpy(inst.z).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    v = torch.from_numpy(np.random.default_rng(1).normal(size=s["nvar"])).to(dev)
    f64 = dict(dtype=torch.float64, device=dev)
    L, g, hv = torch.empty(1, **f64), torch.empty(s["nvar"], **f64), torch.empty(s["nvar"], **f64)
    jv = torch.empty(s["ncon"], **f64)
    cg = (torch.empty(n, n, **f64), torch.empty(n, m, **f64), torch.empty(n, **f64))
    nx, nv, nc = n * (N + 1), s["nvar"], s["ncon"]
    calls = {
        "lagrangian": (lambda: prob.lagrangian(z, y, 1.0, out=L), 8 * (nv + nc)),
        "lag_grad": (lambda: prob.lag_grad(z, y, 1.0, out=g), 8 * (2 * nv + nc)),
        "hvp": (lambda: prob.hvp(z, y, v, 1.0, out=hv), 8 * (nx + nc + 2 * nv)),
        "jvp": (lambda: prob.jvp(z, v, out=jv), 8 * (nx + nv + nc)),
        "coef_grad": (lambda: prob.coef_grad(z, y, out=cg), 8 * (nv + nc)),
        "coef_mixed": (lambda: prob.coef_mixed(z, y, v, out=cg), 8 * (nx + nv + nc)),
        # cotangents: the coefficient-shaped outputs the calls above leave in cg
        "coef_adjoint": (lambda: prob.coef_adjoint(z, y, *cg, out_z=hv, out_y=jv), 8 * (2 * nv + 2 * nc)),
    }
    out = {"workload": f"N={N} n={n} m={m}, seed 0"}
    # the autograd pass first: it is timed on the host clock, and HIP graph
    # captures made before it slowed its Python-side dispatch
    leaf = lambda a: torch.from_numpy(np.array(a)).to(dev).requires_grad_(True)
    zt, yt, At, Bt, gt = (leaf(a) for a in (inst.z, inst.y, inst.A, inst.B, inst.gamma))

    def fwd_bwd():
        for t in (zt, yt, At, Bt, gt):
            t.grad = None
        lagrangian(prob, zt, yt, At, Bt, gt, 1.0).backward()

    fwd_bwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fwd_bwd()
    torch.cuda.synchronize()
    out["autograd_forward_backward_ms"] = round(1e3 * (time.perf_counter() - t0) / reps, 4)
    for name, (fn, nbytes) in calls.items():
        ms, gms = _call_times(torch, fn, reps)
        out[name] = {"ms": round(ms, 4), "graph_ms": round(gms, 4), "bytes": nbytes,
                     "hbm_frac": round(nbytes / (gms * 1e-3) / HBM_PEAK, 4),
                     "eager_hbm_frac": round(nbytes / (ms * 1e-3) / HBM_PEAK, 4)}
    prob.close()

    # the same entry points on the quadrotor model at the paper's largest
    # grid (no coefficient gradient: the model has no coefficient arrays)
    q = synth.make_quadrotor(synth.QUAD_PAPER, seed=0, bnd=1)
    qp = ocp.QuadrotorProblem.from_instance(q, dev)
    qs = qp.sizes
    qz, qy = torch.from_numpy(q.z).to(dev), torch.from_numpy(q.y).to(dev)
    qv = torch.from_numpy(np.random.default_rng(2).normal(size=qs["nvar"])).to(dev)
    qL, qg, qhv = torch.empty(1, **f64), torch.empty(qs["nvar"], **f64), torch.empty(qs["nvar"], **f64)
    qjv = torch.empty(qs["ncon"], **f64)
    qv_, qc = qs["nvar"], qs["ncon"]
    qcalls = {
        "lagrangian": (lambda: qp.lagrangian(qz, qy, 1.0, out=qL), 8 * (qv_ + qc)),
        "lag_grad": (lambda: qp.lag_grad(qz, qy, 1.0, out=qg), 8 * (2 * qv_ + qc)),
        "hvp": (lambda: qp.hvp(qz, qy, qv, 1.0, out=qhv), 8 * (qv_ + qc + 2 * qv_)),
        "jvp": (lambda: qp.jvp(qz, qv, out=qjv), 8 * (2 * qv_ + qc)),
    }
    qout = {"workload": f"quadrotor, x(0) rows, N={q.N}, seed 0"}
    for name, (fn, nbytes) in qcalls.items():
        ms, gms = _call_times(torch, fn, reps)
        qout[name] = {"ms": round(ms, 4), "graph_ms": round(gms, 4), "bytes": nbytes,
                      "hbm_frac": round(nbytes / (gms * 1e-3) / HBM_PEAK, 4),
                      "eager_hbm_frac": round(nbytes / (ms * 1e-3) / HBM_PEAK, 4)}
    qp.close()
    out["quadrotor"] = qout
    return out


def euler(torch, ocp, synth, reps=10):
    """Forward-Euler transcription with initial- and final-state rows, at the
    large shape (N = 1e6, n = 16, m = 8): cons, jac, hess and assemble_kkt
    timed with HIP events, against their algorithmic bytes, each repeated
    back to back and all four in sequence as a step (`in_step`)."""
    N, n, m = synth.LARGE
    dev = torch.device("cuda", 0)
    inst = synth.make_instance(N, n, m, seed=0, scheme=1, bnd=2)
    prob = ocp.Problem.from_instance(inst, dev)
    s = prob.sizes
    z = torch.from_numpy(inst.z).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    rowptr, _, perm_j, perm_h = ocp.kkt_pattern(N, n, m, colind=False, scheme=1, boundary=2)
    pj = torch.from_numpy(perm_j).to(dev)
    del perm_j
    ph, rp = torch.from_numpy(perm_h).to(dev), torch.from_numpy(rowptr).to(dev)
    f64 = dict(dtype=torch.float64, device=dev)
    c, jv, hv = torch.empty(s["ncon"], **f64), torch.empty(s["nnzj"], **f64), torch.empty(s["nnzh"], **f64)
    kkt = torch.empty(s["nnzk"], **f64)
    nx = n * (N + 1)
    calls = {
        "eval_cons": (lambda: prob.cons(z, out=c), 8 * s["nvar"] + 8 * s["ncon"]),
        "eval_jac": (lambda: prob.jac(z, out=jv), 8 * s["nnzj"] + 8 * nx),
        "eval_hess": (lambda: prob.hess(z, y, 1.0, out=hv), 8 * s["nnzh"] + 8 * nx + 8 * n * N),
        "assemble_kkt": (lambda: prob.assemble_kkt(pj, ph, rp, jv, hv, None, out=kkt),
                         12 * (s["nnzj"] + s["nnzh"]) + 8 * s["nnzk"] + 4 * s["ncon"]),
    }
    out = {"workload": f"forward Euler, initial+final state rows, N={N} n={n} m={m}, seed 0",
           "nnzj": s["nnzj"], "nnzh": s["nnzh"]}
    for name, (fn, nbytes) in calls.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": round(ms, 4), "bytes": nbytes,
                     "hbm_frac": round(nbytes / (ms * 1e-3) / HBM_PEAK, 4)}
    t = (out["eval_jac"]["ms"] + out["eval_hess"]["ms"]) * 1e-3
    out["jac_hess_nnz_per_s"] = (s["nnzj"] + s["nnzh"]) / t
    # the four calls in sequence as one step (HIP events between them), as
    # the headline times its step; the figures above are each call repeated
    # back to back
    names = list(calls)
    for _ in range(2):
        for nm in names:
            calls[nm][0]()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(reps)]
    for ev in evs:
        ev[0].record()
        for i, nm in enumerate(names):
            calls[nm][0]()
            ev[i + 1].record()
    torch.cuda.synchronize()
    in_step = {}
    for i, nm in enumerate(names):
        ms = float(np.mean([ev[i].elapsed_time(ev[i + 1]) for ev in evs]))
        in_step[nm] = {"ms": round(ms, 4), "hbm_frac": round(calls[nm][1] / (ms * 1e-3) / HBM_PEAK, 4)}
    in_step["step_ms"] = round(float(np.mean([ev[0].elapsed_time(ev[-1]) for ev in evs])), 4)
    t = (in_step["eval_jac"]["ms"] + in_step["eval_hess"]["ms"]) * 1e-3
    in_step["jac_hess_nnz_per_s"] = (s["nnzj"] + s["nnzh"]) / t
    out["in_step"] = in_step
    # the fused evaluation into the KKT values (no reg), against the separate
    # eval_jac + eval_hess + assemble_kkt above
    fn = lambda: prob.eval_kkt(z, y, 1.0, None, out=kkt)
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 8 * (nx + n * N + s["nnzk"])  # states and y in, the KKT values out
    sep = out["eval_jac"]["ms"] + out["eval_hess"]["ms"] + out["assemble_kkt"]["ms"]
    out["eval_kkt"] = {"ms": round(ms, 4), "bytes": nbytes, "hbm_frac": round(nbytes / (ms * 1e-3) / HBM_PEAK, 4),
                       "speedup_vs_separate": round(sep / ms, 3)}
    prob.close()
    return out


def quadrotor(torch, ocp, synth, reps=10):
    """The quadrotor model (68 Jacobian and 23 Hessian entries per node) with
    the initial-state rows: a full step (obj, grad, cons, jac, hess,
    assemble_kkt) at N = 1e6, and the same at the paper's largest grid
    N = 2e5, each call timed with HIP events against its algorithmic bytes."""
    out = {}
    for tag, N in (("N1e6", synth.QUAD_LARGE), ("N2e5", synth.QUAD_PAPER)):
        dev = torch.device("cuda", 0)
        q = synth.make_quadrotor(N, seed=0, bnd=1)
        prob = ocp.QuadrotorProblem.from_instance(q, dev)
        s = prob.sizes
        z = torch.from_numpy(q.z).to(dev)
        y = torch.from_numpy(q.y).to(dev)
        rowptr, _, perm_j, perm_h = ocp.quad_kkt_pattern(N, 1, colind=False)
        pj, ph, rp = (torch.from_numpy(a).to(dev) for a in (perm_j, perm_h, rowptr))
        f64 = dict(dtype=torch.float64, device=dev)
        o = torch.empty(1, **f64)
        g = torch.empty(s["nvar"], **f64)
        c, jv, hv = torch.empty(s["ncon"], **f64), torch.empty(s["nnzj"], **f64), torch.empty(s["nnzh"], **f64)
        kkt = torch.empty(s["nnzk"], **f64)
        N1 = N + 1
        # algorithmic bytes: the attitude and controls (7 per node) feed the
        # derivatives; the Hessian also reads the six nonlinear rows' y
        calls = {
            "eval_obj": (lambda: prob.obj(z, out=o), 8 * 10 * N1),
            "eval_grad": (lambda: prob.grad(z, out=g), 8 * 10 * N1 + 8 * s["nvar"]),
            "eval_cons": (lambda: prob.cons(z, out=c), 8 * s["nvar"] + 8 * s["ncon"]),
            "eval_jac": (lambda: prob.jac(z, out=jv), 8 * s["nnzj"] + 8 * 7 * N1),
            "eval_hess": (lambda: prob.hess(z, y, 1.0, out=hv), 8 * s["nnzh"] + 8 * 7 * N1 + 8 * 6 * N),
            "assemble_kkt": (lambda: prob.assemble_kkt(pj, ph, rp, jv, hv, None, out=kkt),
                             12 * (s["nnzj"] + s["nnzh"]) + 8 * s["nnzk"] + 4 * s["ncon"]),
        }
        r = {"workload": f"quadrotor (paper Appendix A), trapezoidal, x(0) rows, N={N}, seed 0",
             "nnzj": s["nnzj"], "nnzh": s["nnzh"], "nnzk": s["nnzk"]}
        for name, (fn, nbytes) in calls.items():
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            r[name] = {"ms": round(ms, 4), "bytes": nbytes,
                       "hbm_frac": round(nbytes / (ms * 1e-3) / HBM_PEAK, 4)}
        r["step_ms"] = round(sum(r[k]["ms"] for k in calls), 4)
        t = (r["eval_jac"]["ms"] + r["eval_hess"]["ms"]) * 1e-3
        r["jac_hess_nnz_per_s"] = (s["nnzj"] + s["nnzh"]) / t

        # the six calls back to back as one step, eagerly and replayed from a
        # HIP graph captured once
        def step():
            for fn, _ in calls.values():
                fn()

        def timed_steps(run):
            run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                run()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        # the fused evaluation into the KKT values, against jac + hess + assemble
        r["eval_kkt"] = {"ms": round(timed_steps(lambda: prob.eval_kkt(z, y, 1.0, None, out=kkt)), 4)}
        nb_fused = 8 * (7 * N1 + 6 * N + s["nnzk"])  # attitude, controls, y in; KKT values out
        r["eval_kkt"]["bytes"] = nb_fused
        r["eval_kkt"]["hbm_frac"] = round(nb_fused / (r["eval_kkt"]["ms"] * 1e-3) / HBM_PEAK, 4)
        sep = r["eval_jac"]["ms"] + r["eval_hess"]["ms"] + r["assemble_kkt"]["ms"]
        r["eval_kkt"]["speedup_vs_separate"] = round(sep / r["eval_kkt"]["ms"], 3)
        r["eager_step_ms"] = round(timed_steps(step), 4)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        r["graph_step_ms"] = round(timed_steps(graph.replay), 4)
        del graph
        prob.close()
        del pj, ph, rp, jv, hv, kkt
        torch.cuda.empty_cache()
        out[tag] = r
    return out


def reordered(torch, ocp, synth, reps=10):
    """Assembly into the fill-reducingly reordered KKT matrix P K P^T, the
    ordering folded into the slot maps (ocp_assemble_kkt_mapped), against the
    natural-order assembly and against natural assembly followed by a device
    gather into the reordered layout (what a solver does without the fold).
    Quadrotor at N = 1e6 and the synthetic family at N = 1e5 (n = 8, m = 4)."""
    out = {}
    dev = torch.device("cuda", 0)
    cases = (("quadrotor_N1e6", lambda: synth.make_quadrotor(synth.QUAD_LARGE, seed=0, bnd=1)),
             ("synthetic_N1e5_n8_m4", lambda: synth.make_instance(*synth.IPM_LOOP, seed=0)))
    for tag, make in cases:
        inst = make()
        if tag.startswith("quadrotor"):
            prob = ocp.QuadrotorProblem.from_instance(inst, dev)
            rp, ci, pj, ph = ocp.quad_kkt_pattern(inst.N, 1)
            order = ocp.quad_stage_order(inst.N, 1)
        else:
            prob = ocp.Problem.from_instance(inst, dev)
            rp, ci, pj, ph = ocp.kkt_pattern(inst.N, inst.n, inst.m)
            order = ocp.stage_order(inst.N, inst.n, inst.m)
        s = prob.sizes
        t0 = time.perf_counter()
        rp2, ci2, pj2, ph2, dg2 = ocp.kkt_permute(rp, ci, pj, ph, order)
        t_perm = time.perf_counter() - t0
        # old slot -> new slot, then new slot -> old slot for the gather
        smap = np.empty(s["nnzk"], np.int64)
        smap[pj], smap[ph], smap[rp[1:] - 1] = pj2, ph2, dg2
        inv = np.empty(s["nnzk"], np.int64)
        inv[smap] = np.arange(s["nnzk"])
        del ci, ci2, smap
        z, y = (torch.from_numpy(a).to(dev) for a in (inst.z, inst.y))
        jv, hv = prob.jac(z), prob.hess(z, y, 1.0)
        t_pj, t_ph, t_rp, t_pj2, t_ph2, t_dg2 = (torch.from_numpy(a).to(dev) for a in (pj, ph, rp, pj2, ph2, dg2))
        t_inv = torch.from_numpy(inv).to(dev)
        del inv
        f64 = dict(dtype=torch.float64, device=dev)
        kkt, kkt2 = torch.empty(s["nnzk"], **f64), torch.empty(s["nnzk"], **f64)
        plan = prob.mapped_plan(t_pj2, t_ph2, t_dg2)  # once per set of slot maps
        nbytes = 12 * (s["nnzj"] + s["nnzh"]) + 8 * s["nnzk"] + 4 * s["ncon"]
        calls = {
            "natural_assemble_kkt": lambda: prob.assemble_kkt(t_pj, t_ph, t_rp, jv, hv, None, out=kkt),
            "reordered_assemble_kkt_mapped": lambda: prob.assemble_kkt_mapped(t_pj2, t_ph2, t_dg2, jv, hv,
                                                                              None, out=kkt2),
            "reordered_assemble_kkt_mapped_planned": lambda: prob.assemble_kkt_mapped(
                t_pj2, t_ph2, t_dg2, jv, hv, None, out=kkt2, plan=plan),
            "natural_then_gather": lambda: (prob.assemble_kkt(t_pj, t_ph, t_rp, jv, hv, None, out=kkt),
                                            torch.index_select(kkt, 0, t_inv, out=kkt2)),
        }
        r = {"nnzk": s["nnzk"], "host_permute_s": round(t_perm, 2), "bytes": nbytes,
             "note": "reordered_assemble_kkt_mapped passes no plan: the handle builds one for the maps on "
                     "its first call and reuses it"}
        for name, fn in calls.items():
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            r[name] = {"ms": round(ms, 4), "hbm_frac": round(nbytes / (ms * 1e-3) / HBM_PEAK, 4)}
        r["speedup_fold_vs_gather"] = round(r["natural_then_gather"]["ms"] /
                                            r["reordered_assemble_kkt_mapped_planned"]["ms"], 3)
        prob.close()
        del jv, hv, kkt, kkt2, t_pj, t_ph, t_rp, t_pj2, t_ph2, t_dg2, t_inv, plan
        torch.cuda.empty_cache()
        out[tag] = r
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the 512-instance batched measurement (profiling runs)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 512-instance batched measurement (profiling runs)")
    ap.add_argument("--no-euler", action="store_true",
                    help="skip the forward-Euler measurement (profiling runs)")
    ap.add_argument("--no-fused", action="store_true",
                    help="skip the fused KKT evaluation measurement (profiling runs)")
    ap.add_argument("--no-reorder", action="store_true",
                    help="skip the reordered-KKT assembly measurement (profiling runs)")
    ap.add_argument("--only-reorder", action="store_true",
                    help="run only the reordered-KKT assembly measurement (profiling runs)")
    ap.add_argument("--no-quad", action="store_true",
                    help="skip the quadrotor measurement (profiling runs)")
    ap.add_argument("--only-quad", action="store_true",
                    help="run only the quadrotor measurement (profiling runs)")
    ap.add_argument("--no-diff", action="store_true",
                    help="skip the N=2e5 differentiation measurement (profiling runs)")
    ap.add_argument("--no-ipm-loop", action="store_true",
                    help="skip the N=1e5 interior-point-loop measurement (profiling runs)")
    ap.add_argument("--N", type=int, default=None, help="override the interval count")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); the evaluation "
              "path would shard by node range across GPUs, but no multi-GPU run is provided",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2510_03932_amd as ocp
    import synth

    if args.only_batched:
        torch.cuda.set_device(0)
        log("[bench] batched workload only")
        print(json.dumps({"batched": batched(torch, ocp, synth)}), flush=True)
        return
    if args.only_reorder:
        log("[bench] reordered KKT assembly only")
        print(json.dumps({"reordered": reordered(torch, ocp, synth)}), flush=True)
        return
    if args.only_quad:
        log("[bench] quadrotor workload only")
        print(json.dumps({"quadrotor": quadrotor(torch, ocp, synth)}), flush=True)
        return

    N, n, m = synth.LARGE
    if args.N:
        N = args.N
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"[bench] generating inputs N={N} n={n} m={m}")
    inst = synth.make_instance(N, n, m, seed=0)
    prob = ocp.Problem.from_instance(inst, dev)
    s = prob.sizes
    log("[bench] building KKT structure on the host")
    t0 = time.perf_counter()
    rowptr, _, perm_j, perm_h = ocp.kkt_pattern(N, n, m, colind=False)
    t_kkt_build = time.perf_counter() - t0
    z = torch.from_numpy(inst.z).to(dev)
    y = torch.from_numpy(inst.y).to(dev)
    pj = torch.from_numpy(perm_j).to(dev)
    del perm_j
    ph = torch.from_numpy(perm_h).to(dev)
    rp = torch.from_numpy(rowptr).to(dev)
    reg = torch.full((s["dim"],), 1e-8, dtype=torch.float64, device=dev)
    f64 = dict(dtype=torch.float64, device=dev)
    obj = torch.empty(1, **f64)
    g = torch.empty(s["nvar"], **f64)
    c = torch.empty(s["ncon"], **f64)
    jv = torch.empty(s["nnzj"], **f64)
    hv = torch.empty(s["nnzh"], **f64)
    kkt = torch.empty(s["nnzk"], **f64)
    names = ["eval_obj", "eval_grad", "eval_cons", "eval_jac", "eval_hess", "assemble_kkt"]

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        prob.obj(z, out=obj)
        if ev is not None:
            ev[1].record()
        prob.grad(z, out=g)
        if ev is not None:
            ev[2].record()
        prob.cons(z, out=c)
        if ev is not None:
            ev[3].record()
        prob.jac(z, out=jv)
        if ev is not None:
            ev[4].record()
        prob.hess(z, y, 1.0, out=hv)
        if ev is not None:
            ev[5].record()
        prob.assemble_kkt(pj, ph, rp, jv, hv, reg, out=kkt)
        if ev is not None:
            ev[6].record()

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # exactly K timed steps; HIP events on the launch stream split each step
    # into its kernels (recording an event costs no device time)
    log(f"[bench] timing {args.steps} steps")
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    per = {nm: [] for nm in names}
    for ev in events:
        for i, nm in enumerate(names):
            per[nm].append(ev[i].elapsed_time(ev[i + 1]))
    avg = {nm: float(np.mean(v)) for nm, v in per.items()}
    med = {nm: float(np.median(v)) for nm, v in per.items()}

    byt = algorithmic_bytes(s, N, n, m)
    kern = {}
    for nm in names:
        bw = byt[nm] / (avg[nm] * 1e-3)
        kern[nm] = {"avg_ms": round(avg[nm], 4), "median_ms": round(med[nm], 4),
                    "p10_ms": round(float(np.percentile(per[nm], 10)), 4),
                    "p90_ms": round(float(np.percentile(per[nm], 90)), 4),
                    "bytes": int(byt[nm]), "GB_per_s": round(bw / 1e9, 1),
                    "hbm_frac": round(bw / HBM_PEAK, 4)}
    t_jh = (avg["eval_jac"] + avg["eval_hess"]) * 1e-3
    nnz_jh = s["nnzj"] + s["nnzh"]
    value = nnz_jh / t_jh
    jh_frac = (byt["eval_jac"] + byt["eval_hess"]) / t_jh / HBM_PEAK

    dom = max(names, key=lambda nm: avg[nm])
    traffic = None
    if os.path.exists(TRAFFIC):
        tr = json.load(open(TRAFFIC))
        sha = sources_sha256()
        ent = tr.get("kernels", {}).get(dom)
        if ent and tr.get("source_sha256") == sha:
            traffic = int(ent["bytes_per_launch"])
    roof = {"bound": "hbm", "kernel": dom,
            "achieved": round(byt[dom] / (avg[dom] * 1e-3) / 1e9, 1),
            "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": round(byt[dom] / (avg[dom] * 1e-3) / HBM_PEAK, 4),
            "traffic": traffic}

    # each call on its own, its inputs evicted from the caches by a 1 GiB read
    # just before it: the in-step figures above also carry the write-back of
    # the previous call's output (up to the 256 MiB Infinity Cache of dirty
    # lines), which lands on whichever kernel runs next
    log("[bench] isolated call timings")
    flush = torch.ones(2 ** 27, **f64)
    calls = {"eval_obj": lambda: prob.obj(z, out=obj), "eval_grad": lambda: prob.grad(z, out=g),
             "eval_cons": lambda: prob.cons(z, out=c), "eval_jac": lambda: prob.jac(z, out=jv),
             "eval_hess": lambda: prob.hess(z, y, 1.0, out=hv),
             "assemble_kkt": lambda: prob.assemble_kkt(pj, ph, rp, jv, hv, reg, out=kkt)}
    iso = {}
    for nm, fn in calls.items():
        ts = []
        for _ in range(max(args.steps // 2, 5)):
            flush.sum()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        iso[nm] = {"median_ms": round(ms, 4), "GB_per_s": round(byt[nm] / (ms * 1e-3) / 1e9, 1),
                   "hbm_frac": round(byt[nm] / (ms * 1e-3) / HBM_PEAK, 4)}
    del flush
    t_jh_iso = (iso["eval_jac"]["median_ms"] + iso["eval_hess"]["median_ms"]) * 1e-3

    # achievable-bandwidth context: plain device streams over 2 GiB buffers
    # (torch's fill kernel = a pure write stream, copy_ = a read + write stream)
    def stream_rate(fn, nbytes, reps=10):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return reps * nbytes / (e0.elapsed_time(e1) * 1e-3)

    a = torch.empty(2 ** 28, **f64)
    b = torch.empty_like(a)
    a.fill_(0.5)
    copy_bw = stream_rate(lambda: b.copy_(a), 2 * a.numel() * 8)
    write_bw = stream_rate(lambda: b.fill_(1.0), a.numel() * 8)
    del a, b

    out = {
        "metric": "FP64 Jac+Hess nonzeros/s at N=1e6 (% HBM peak)",
        "value": value,
        "unit": "nonzeros/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"single trapezoidal OCP instance N={N} n={n} m={m}, dense A, seed 0",
                   "N": N, "n": n, "m": m, "nnzj": s["nnzj"], "nnzh": s["nnzh"],
                   "nnzk": s["nnzk"], "step": "+".join(names)},
        "jac_hess_ms_per_step": round(t_jh * 1e3, 4),
        "jac_hess_hbm_frac": round(jh_frac, 4),
        "step_nnz_per_s": nnz_jh / (ms_per_step * 1e-3),
        "roofline": roof,
        "kernels": kern,
        "kernels_isolated": iso,
        "jac_hess_isolated_hbm_frac": round((byt["eval_jac"] + byt["eval_hess"]) / t_jh_iso / HBM_PEAK, 4),
        "copy_GB_per_s": round(copy_bw / 1e9, 1),
        "write_stream_GB_per_s": round(write_bw / 1e9, 1),
        "jac_frac_of_write_stream": round(kern["eval_jac"]["GB_per_s"] * 1e9 / write_bw, 4),
        "kkt_host_build_s": round(t_kkt_build, 2),
    }
    # the fused path: the same KKT values written straight from (z, y) by
    # ocp_eval_kkt, against eval_jac + eval_hess + assemble_kkt above
    if not args.no_fused:
        log("[bench] fused evaluation into the KKT matrix")
        prob.eval_kkt(z, y, 1.0, reg, out=kkt)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(args.steps, 5)
        e0.record()
        for _ in range(reps):
            prob.eval_kkt(z, y, 1.0, reg, out=kkt)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        fbytes = 8 * n * (N + 1) + 8 * n * N + 8 * s["dim"] + 8 * s["nnzk"]
        sep_ms = avg["eval_jac"] + avg["eval_hess"] + avg["assemble_kkt"]
        out["fused_kkt"] = {
            "call": "ocp_eval_kkt (Jacobian + Hessian + reg into the CSR KKT values)",
            "ms": round(ms, 4), "bytes": fbytes, "hbm_frac": round(fbytes / (ms * 1e-3) / HBM_PEAK, 4),
            "separate_jac_hess_assemble_ms": round(sep_ms, 4), "speedup_vs_separate": round(sep_ms / ms, 3),
            "jac_hess_nnz_per_s": nnz_jh / (ms * 1e-3),
            "step_ms_with_fused": round(avg["eval_obj"] + avg["eval_grad"] + avg["eval_cons"] + ms, 4)}
    del jv, hv, kkt, pj, ph, rp, z, y, g, c, reg
    torch.cuda.empty_cache()
    if not args.no_ipm_loop:
        log("[bench] interior-point loop workload")
        out["ipm_loop"] = ipm_loop(torch, ocp, synth)
    if not args.no_euler:
        log("[bench] forward-Euler workload")
        out["euler"] = euler(torch, ocp, synth)
    if not args.no_quad:
        log("[bench] quadrotor workload")
        out["quadrotor"] = quadrotor(torch, ocp, synth)
    if not args.no_reorder:
        log("[bench] reordered KKT assembly")
        out["reordered"] = reordered(torch, ocp, synth)
    if not args.no_diff:
        log("[bench] differentiation workload")
        out["differentiation"] = differentiation(torch, ocp, synth)
    if not args.no_batched:
        log("[bench] batched workload")
        out["batched"] = batched(torch, ocp, synth)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        cb = cpu_baseline(inst, synth)
        cb.pop("seconds")
        out["cpu_baseline"] = cb
    prob.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
