"""Benchmark of the shift-and-invert low-rank path on one MI355X.

A step is one whole lowrank_solve (sampling table, estimate phase, shift
tuning, shift-and-invert subspace iteration with SVRG inner solves, final
Rayleigh-Ritz) on one resident synthetic matrix: the planted-spectrum
2048 x 200000 FP32 workload (sigma_1..10 geometric 10 -> 5, sigma_11 = 4.95,
sigma_i = 4 (i - 10)^-0.8 beyond, N(0, 1e-4^2) noise; k = 10, p = 20,
eps = 1e-4).  Prints one JSON line; unless --no-serve, the line also carries
the serving legs described below under "serve".

--mode serve runs the serving form instead: a trace of independent requests
(d in {256..4096}, n in [4096, 131072] log-uniform, k in 1..16, p = k + 4..16,
FP32 or BF16 storage, eps = 1e-4, Poisson arrivals at 50/s) through the
library's request server, once as plain FP32 requests one at a time and once
continuously batched with each request's own storage type; it reports
solves/s, p50/p99 latency and whether every FP32 request's result is bitwise
the same in the batch as alone.

Modes for profiler runs: --mode solve (default), --mode pass (only the
X (X^T W) pass, --steps times), --mode epoch (--steps inner-solver epochs of
the solve's own schedule, each one warm-start pass, m inner steps and a
residual pass), --mode copy (a device copy of the same bytes as X, used to
calibrate HBM byte counters).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
WORKLOAD = "planted-2048x200000-f32"
SPARSE_WORKLOAD = "zipf-50000x1000000-csc-f32"
METRIC = "solves/s + HBM GB/s at ε=1e-4 (plain FP32 vs BF16 batched); p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="solve",
                    choices=["solve", "pass", "epoch", "copy", "serve", "sparse", "sparse-solve",
                             "steps"])
    ap.add_argument("--sparse-workload", default=SPARSE_WORKLOAD)
    ap.add_argument("--sparse-steps", type=int, default=200,
                    help="sparse/steps: inner steps timed (one epoch of this length)")
    ap.add_argument("--precision", type=int, default=4,
                    help="0: FP64 arithmetic; 1: BF16 matrix-core inner steps (BF16 X); "
                         "2: FP32 matrix-core inner steps (FP32 or BF16 X); 3: matrix-core "
                         "passes; 4 (default): matrix-core passes and inner steps")
    ap.add_argument("--batch", type=int, default=0, help="steps: minibatch size (0: 4096)")
    ap.add_argument("--adaptive", type=int, default=0,
                    help="solve: 1 = adaptive partitioning of Algorithm main")
    ap.add_argument("--accel", type=int, default=0,
                    help="solve: 1 = accelerated inner solver")
    ap.add_argument("--no-variants", action="store_true",
                    help="solve: skip the adaptive / accelerated legs")
    ap.add_argument("--requests", type=int, default=512, help="serve: trace length")
    ap.add_argument("--slots", type=int, default=8, help="serve: concurrent worker slots")
    ap.add_argument("--budget-gb", type=float, default=4.0, help="serve: HBM budget (GB)")
    ap.add_argument("--rate", type=float, default=50.0, help="serve: arrivals per second")
    ap.add_argument("--forms", default="seq,closed,open,mc",
                    help="serve: comma list of seq (FP32 one at a time), seq_mc (one at a "
                         "time, matrix-core form), closed, open, mc (closed and open loops in "
                         "the matrix-core form)")
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true",
                    help="solve mode: skip the serving legs of the report")
    ap.add_argument("--no-legs", action="store_true",
                    help="solve mode: skip the 4096 x 500000 BF16 and compressed-column legs")
    return ap.parse_args()


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    pos = (len(xs) - 1) * q
    lo, hi = int(math.floor(pos)), int(math.ceil(pos))
    return xs[lo] + (xs[hi] - xs[lo]) * (pos - lo)


# kernel -> the source file whose SHA-256 a committed counter summary must match
KERNEL_SOURCES = {
    "k_step_update": "kernels.hip", "k_xtm_gathered": "kernels.hip",
    "k_xtm_pass": "kernels.hip", "k_xt_part": "kernels.hip",
    "k_supd_f32": "f32steps.hip", "k_sdot_f32": "f32steps.hip",
    "k_supd_bf16": "bf16.hip", "k_sdot_bf16": "bf16.hip",
    "k_mc_xtw": "mcpass.hip", "k_mc_xt": "mcpass.hip",
}


def measured_traffic(kernel, workload):
    """Calibrated HBM bytes per launch of `kernel` from the committed rocprofv3
    counter summary, or None when the kernel's source has changed since it was
    taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s.md" % workload)
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    src = os.path.join(ROOT, "paper_1607_02925_amd", "csrc", KERNEL_SOURCES[kernel])
    text = open(path).read()
    if "```json" not in text:
        return None
    t = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if t.get("sources_sha256", {}).get(KERNEL_SOURCES[kernel]) != sha:
        return None
    k = t["per_launch_kib"].get(kernel)
    if k is None:
        return None
    c = t["calibration"]
    return (k["fetch"] * c["fetch_scale"] + k["write"] * c["write_scale"]) * 1024.0


def cpu_baseline(Xt_dev, w, sched, rep):
    """Time the oracle (NumPy FP64) on a bounded sample of the same workload:
    the sampling table, one X(X^T S) pass and one inner-solver epoch at full
    size, then scale to a whole solve with the pass and epoch counts of the
    GPU run."""
    import numpy as np
    import oracle
    from threadpoolctl import threadpool_info
    t0 = time.time()
    xt = Xt_dev.cpu().numpy()
    X = oracle.decode(xt, w["storage"])
    t_prep0 = time.time()
    wn = oracle.column_sq_norms(X)
    _, qc = oracle.build_table(wn)
    t_prep = time.time() - t_prep0
    d, p = X.shape[0], w["p"]
    S = oracle.cholqr2(oracle.gaussian_block(w["solver_seed"], 2, 0, d, p))[0]
    t1 = time.time()
    oracle.apply_A(X, S)
    t_pass = time.time() - t1
    t2 = time.time()
    oracle.svrg_solve(X, qc, S, sched.lam, sched.eta, sched.m, sched.b, 0.0, w["solver_seed"],
                      sched.first_solve, 60, fixed_epochs=1)
    t_epoch_incl = time.time() - t2   # warm-start pass + one epoch (steps + residual pass)
    t_steps = max(t_epoch_incl - 2 * t_pass, 0.0)
    est = t_prep + rep["passes"] * t_pass + rep["total_epochs"] * t_steps
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    log("cpu baseline: prep %.2fs pass %.2fs epoch-steps %.2fs -> est %.1fs per solve "
        "(sample wall %.1fs)" % (t_prep, t_pass, t_steps, est, time.time() - t0))
    return {"value": 1.0 / est, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": "oracle (NumPy FP64) on the full-size workload: sampling table, one "
                      "X(X^T S) pass and one inner-solver epoch (m=%d steps, b=%d) timed, "
                      "scaled by the GPU run's %d passes and %d epochs per solve"
                      % (sched.m, sched.b, rep["passes"], rep["total_epochs"])}


def variant_leg(Xt, w, U_qk, args, name, **kw):
    """The same workload through a variant of the method (kw: adaptive = 1 for
    the adaptive partitioning of Algorithm main, accel = 1 for the accelerated
    inner solver, precision = 2 for FP32 matrix-core inner steps): solves/s,
    what it did, and the principal-angle sine between its U_k and the plain
    q = k branch's."""
    import torch
    from paper_1607_02925_amd import lowrank
    plan = lowrank.Plan(Xt, w["k"], w["p"], w["eps"], seed=w["solver_seed"], **kw)
    plan.solve()
    torch.cuda.synchronize()
    lat = []
    for _ in range(max(1, args.steps)):
        t = time.time()
        st, U, theta, rep = plan.solve()
        torch.cuda.synchronize()
        lat.append(time.time() - t)
    Uq = U_qk.contiguous()
    Ua = U.contiguous()
    sin = float(torch.linalg.matrix_norm(Ua - Uq @ (Uq.T @ Ua), ord=2))
    sc = plan.schedule()
    out = {"solves_per_s": len(lat) / sum(lat), "ms_per_solve": sum(lat) / len(lat) * 1e3,
           "status": st, "passes": rep["passes"], "inner_steps": rep["steps"],
           "epochs": rep["total_epochs"], "sin_vs_q_eq_k": sin}
    if kw.get("adaptive"):
        out["intervals"] = rep["intervals"]
    else:
        out.update(outer=rep["outer"], b=sc.b, m=sc.m)
    if kw.get("accel"):
        out.update(kappa=rep["accel_kappa"], beta=rep["accel_beta"])
    log("%s: %s" % (name, json.dumps(out)))
    return out


def serve_run(reqs, X, slots, budget, open_loop=False, matrix_core=False):
    """Push every request of `reqs` (device matrices X[i]) through a server with
    `slots` worker slots and an HBM budget; closed loop submits all at t = 0,
    open loop at each request's arrival time.  matrix_core: passes and inner
    steps on matrix cores (LR_PREC_MC: BF16-part passes with refined residuals,
    BF16 steps for BF16 X, FP32 steps for FP32 X) instead of FP64.
    Returns per-request results."""
    import torch
    from paper_1607_02925_amd import lowrank
    srv = lowrank.Server(budget, slots=slots)
    torch.cuda.synchronize()
    tickets = []
    t0 = time.time()
    for r, x in zip(reqs, X):
        if open_loop:
            delay = r["arrival"] - (time.time() - t0)
            if delay > 0:
                time.sleep(delay)
        prec = 4 if matrix_core else 0
        tickets.append(srv.submit(x, r["k"], r["p"], r["eps"], sync=False,
                                  seed=r["solver_seed"], precision=prec))
    outs = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    t_first = min(o[4]["t_submit"] for o in outs)
    t_last = max(o[4]["t_done"] for o in outs)
    lat = [o[4]["t_done"] - o[4]["t_submit"] for o in outs]
    svc = [o[4]["t_done"] - o[4]["t_admit"] for o in outs]
    bad = [(r["id"], o[0]) for r, o in zip(reqs, outs) if o[0] != 0]
    pass_bytes = sum(o[3]["passes"] * x.numel() * x.element_size() for o, x in zip(outs, X))
    res = {"requests": len(reqs), "slots": slots, "budget_bytes": int(budget),
           "makespan_s": t_last - t_first, "solves_per_s": len(reqs) / (t_last - t_first),
           "latency_ms": {"p50": percentile(lat, 0.5) * 1e3, "p99": percentile(lat, 0.99) * 1e3,
                          "max": max(lat) * 1e3},
           "service_ms": {"p50": percentile(svc, 0.5) * 1e3, "p99": percentile(svc, 0.99) * 1e3},
           "pass_GBps_alg": pass_bytes / (t_last - t_first) / 1e9,
           "inner_steps_total": int(sum(o[3]["steps"] for o in outs)),
           "passes_total": int(sum(o[3]["passes"] for o in outs)),
           "peak_running": stats["peak_running"], "peak_bytes": stats["peak_bytes"],
           "failed": bad}
    return res, outs


def sparse_bench(args, dev):
    """Compressed-column workload: plan creation (row-ordered copy), the pass
    X (X^T W) and inner steps at the minibatch size the method picks for it
    (b = 8192), timed on the device.  A whole solve of this workload takes
    hundreds of outer iterations of ~10^4 inner steps each, so it is measured
    per pass and per step."""
    import torch
    import workloads
    from paper_1607_02925_amd import lowrank
    w = workloads.workload(args.sparse_workload)
    X = lowrank.CscMatrix.from_arrays(w["d"], w["n"], w["col_ptr"], w["row_idx"], w["values"],
                                      device=dev)
    torch.cuda.synchronize()
    d, p = w["d"], w["p"]
    t0 = time.time()
    plan = lowrank.Plan(X, w["k"], p, w["eps"], seed=w["solver_seed"])
    torch.cuda.synchronize()
    t_plan = time.time() - t0
    _, _, fro2 = plan.prepare()
    S = torch.linalg.qr(torch.randn((d, p), dtype=torch.float64, device=dev))[0]
    for _ in range(6):                      # top Ritz value for a realistic shift
        S = torch.linalg.qr(plan.apply_A(S))[0]
    theta1 = float(torch.linalg.eigvalsh(S.T @ plan.apply_A(S))[-1])
    Wm = torch.randn((d, p), dtype=torch.float64, device=dev)
    plan.apply_A(Wm)
    torch.cuda.synchronize()
    reps = max(3, args.steps)
    t = time.time()
    for _ in range(reps):
        plan.apply_A(Wm)
    torch.cuda.synchronize()
    ms_pass = (time.time() - t) / reps * 1e3
    lam, mu, b = 1.05 * theta1, 0.05 * theta1, 8192
    eta = min(1.0 / lam, mu * b / (4.0 * fro2 * theta1))
    m = args.sparse_steps
    plan.svrg_solve(S, lam, eta, 8, b, 1, 1)
    torch.cuda.synchronize()
    t = time.time()
    plan.svrg_solve(S, lam, eta, m, b, 2, 1)
    torch.cuda.synchronize()
    ms_epoch = (time.time() - t) * 1e3
    us_step = (ms_epoch - 2 * ms_pass) / m * 1e3
    elt = w["values"].dtype.itemsize
    csc_bytes = w["nnz"] * (elt + 4) + (w["n"] + 1) * 4
    out = {"workload": args.sparse_workload, "d": d, "n": w["n"], "nnz": w["nnz"], "p": p,
           "plan_s": t_plan, "pass_ms": ms_pass,
           "pass_GBps_alg": (csc_bytes + 3 * d * p * 8) / (ms_pass * 1e-3) / 1e9,
           "pass_gather_GBps": 2 * w["nnz"] * lowrank_pad16(p) * 8 / (ms_pass * 1e-3) / 1e9,
           "theta1": theta1, "b": b, "epoch_steps": m, "epoch_ms": ms_epoch,
           "step_us": us_step}
    log("sparse: %s" % json.dumps(out))
    return out


def sparse_solve(args, dev):
    """One whole solve (q = k branch, FP64) of the compressed-column workload;
    a few minutes, so not part of the default run."""
    import torch
    import workloads
    from paper_1607_02925_amd import lowrank
    w = workloads.workload(args.sparse_workload)
    X = lowrank.CscMatrix.from_arrays(w["d"], w["n"], w["col_ptr"], w["row_idx"], w["values"],
                                      device=dev)
    log("generated %s" % args.sparse_workload)
    plan = lowrank.Plan(X, w["k"], w["p"], w["eps"], seed=w["solver_seed"], timing=1)
    torch.cuda.synchronize()
    t = time.time()
    st, U, theta, rep = plan.solve()
    torch.cuda.synchronize()
    sc = plan.schedule()
    return {"workload": args.sparse_workload, "status": st, "seconds": time.time() - t,
            "outer": rep["outer"], "epochs": rep["total_epochs"], "passes": rep["passes"],
            "inner_steps": rep["steps"], "shift_rounds": rep["shift_rounds"], "lambda": sc.lam,
            "b": sc.b, "m": sc.m, "theta": [float(x) for x in theta],
            "ms_pass": rep["ms_pass_total"] / max(rep["timed_passes"], 1),
            "us_step": rep["ms_steps_total"] * 1e3 / max(rep["timed_steps"], 1)}


def steps_bench(args, dev):
    """Dense workload: one pass and one epoch of --sparse-steps inner steps at
    minibatch b (default 4096) in the chosen precision, with a shift 5% above
    the top Ritz value of six power steps."""
    import torch
    import workloads
    from paper_1607_02925_amd import lowrank
    w = dict(workloads.WORKLOADS[args.workload])
    data = workloads.workload(args.workload, device=dev)
    Xt = data["Xt"]
    torch.cuda.synchronize()
    d, p = w["d"], w["p"]
    plan = lowrank.Plan(Xt, w["k"], p, w["eps"], seed=w["solver_seed"], precision=args.precision)
    _, _, fro2 = plan.prepare()
    S = torch.linalg.qr(torch.randn((d, p), dtype=torch.float64, device=dev))[0]
    for _ in range(6):
        S = torch.linalg.qr(plan.apply_A(S))[0]
    theta1 = float(torch.linalg.eigvalsh(S.T @ plan.apply_A(S))[-1])
    torch.cuda.synchronize()
    reps = max(3, args.steps)
    t = time.time()
    for _ in range(reps):
        plan.apply_A(S)
    torch.cuda.synchronize()
    ms_pass = (time.time() - t) / reps * 1e3
    lam, mu, b = 1.05 * theta1, 0.05 * theta1, args.batch or 4096
    eta = min(1.0 / lam, mu * b / (4.0 * fro2 * theta1))
    m = args.sparse_steps
    plan.svrg_solve(S, lam, eta, 8, b, 1, 1)
    torch.cuda.synchronize()
    t = time.time()
    plan.svrg_solve(S, lam, eta, m, b, 2, 1)
    torch.cuda.synchronize()
    ms_epoch = (time.time() - t) * 1e3
    out = {"workload": args.workload, "precision": args.precision, "d": d, "n": w["n"], "p": p,
           "b": b, "pass_ms": ms_pass, "epoch_steps": m, "epoch_ms": ms_epoch,
           "step_us": (ms_epoch - 2 * ms_pass) / m * 1e3}
    log("steps: %s" % json.dumps(out))
    return out


def big_dense_leg(args, dev, name):
    """A dense workload too large for a whole solve per bench step: its pass in
    FP64 and on matrix cores (roofline on |X| + 3 d p 4 bytes) and an epoch of
    matrix-core inner steps at the minibatch the method picks for it (b = 4096),
    with a shift 5% above the top Ritz value of six power steps."""
    import torch
    import workloads
    from paper_1607_02925_amd import lowrank
    w = dict(workloads.WORKLOADS[name])
    data = workloads.workload(name, device=dev)
    Xt = data["Xt"]
    torch.cuda.synchronize()
    d, n, p = w["d"], w["n"], w["p"]
    x_bytes = Xt.numel() * Xt.element_size()
    out = {"workload": name, "d": d, "n": n, "p": p}
    W = torch.randn((p, d), dtype=torch.float64, device=dev).T
    for prec, key in ((0, "pass_f64"), (3, "pass_mc")):
        plan = lowrank.Plan(Xt, w["k"], p, w["eps"], seed=w["solver_seed"], precision=prec)
        plan.apply_A(W)
        torch.cuda.synchronize()
        reps = max(3, args.steps)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            plan.apply_A(W)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        gbs = (x_bytes + 3 * d * p * 4) / (ms * 1e-3) / 1e9
        out[key] = {"ms": ms, "hbm_GBps_alg": gbs, "frac_hbm": gbs / PEAK_HBM_GBS}
        del plan
    plan = lowrank.Plan(Xt, w["k"], p, w["eps"], seed=w["solver_seed"], precision=4)
    _, _, fro2 = plan.prepare()
    S = torch.linalg.qr(torch.randn((d, p), dtype=torch.float64, device=dev))[0]
    for _ in range(6):
        S = torch.linalg.qr(plan.apply_A(S))[0]
    theta1 = float(torch.linalg.eigvalsh(S.T @ plan.apply_A(S))[-1])
    lam, mu, b = 1.05 * theta1, 0.05 * theta1, 4096
    eta = min(1.0 / lam, mu * b / (4.0 * fro2 * theta1))
    m = 200
    plan.svrg_solve(S, lam, eta, 8, b, 1, 1)
    torch.cuda.synchronize()
    t = time.time()
    plan.svrg_solve(S, lam, eta, m, b, 2, 1)
    torch.cuda.synchronize()
    ms_epoch = (time.time() - t) * 1e3
    out["epoch_mc"] = {"b": b, "steps": m, "epoch_ms": ms_epoch,
                       "step_us": (ms_epoch - out["pass_f64"]["ms"] - out["pass_mc"]["ms"])
                       / m * 1e3}
    log("%s: %s" % (name, json.dumps(out)))
    return out


def accel_leg(args, dev):
    """The accelerated inner solver where it pays: a 600 x 5000 Zipf(1.1)
    compressed-column X (16 nonzeros per column, k = 1, p = 4, eps = 1e-4), on
    which kappa > 0 (a plain epoch samples far more columns than a pass reads).
    Plain and accelerated solves timed back to back; the principal-angle sine
    between their U_k."""
    import torch
    from workloads import sparse
    from paper_1607_02925_amd import lowrank
    sp = sparse.zipf_csc(600, 5000, 16, seed=11)
    X = lowrank.CscMatrix.from_arrays(sp["d"], sp["n"], sp["col_ptr"], sp["row_idx"],
                                      sp["values"], device=dev)
    out = {"workload": "zipf-600x5000-csc-f32", "k": 1, "p": 4, "eps": 1e-4}
    Us = {}
    for name, acc in (("plain", 0), ("accel", 1)):
        plan = lowrank.Plan(X, 1, 4, 1e-4, seed=7, accel=acc)
        t = time.time()
        st, U, theta, rep = plan.solve()
        torch.cuda.synchronize()
        Us[name] = U.contiguous()
        out[name] = {"s_per_solve": time.time() - t, "status": st, "epochs": rep["total_epochs"],
                     "inner_steps": rep["steps"], "passes": rep["passes"],
                     "kappa": rep["accel_kappa"], "beta": rep["accel_beta"]}
    Ua, Ub = Us["plain"], Us["accel"]
    out["sin_accel_vs_plain"] = float(torch.linalg.matrix_norm(Ub - Ua @ (Ua.T @ Ub), ord=2))
    out["speedup"] = out["plain"]["s_per_solve"] / out["accel"]["s_per_solve"]
    log("accel leg: %s" % json.dumps(out))
    return out


def lowrank_pad16(p):
    return (p + 15) // 16 * 16


def serve_bench(args, dev):
    import torch
    import workloads
    reqs = workloads.serving.trace(args.requests, rate=args.rate)
    t0 = time.time()
    X32, Xown = [], []
    for r in reqs:
        x = workloads.serving.request_data(r, device=dev, storage="f32")
        X32.append(x)
        Xown.append(x if r["storage"] == "f32" else x.to(torch.bfloat16))
    torch.cuda.synchronize()
    log("serve: generated %d requests (%.1f GB FP32) in %.1fs" %
        (len(reqs), sum(x.numel() * 4 for x in X32) / 1e9, time.time() - t0))
    budget = int(args.budget_gb * 1e9)
    forms = set(args.forms.split(","))
    out = {"trace": {"requests": len(reqs), "rate_per_s": args.rate,
                     "f32": sum(r["storage"] == "f32" for r in reqs),
                     "bf16": sum(r["storage"] == "bf16" for r in reqs)}}
    seq_outs = closed_outs = None
    if "seq" in forms:
        out["fp32_per_request"], seq_outs = serve_run(reqs, X32, 1, budget)
        log("serve fp32 per-request: %s" % json.dumps(out["fp32_per_request"]))
    if "seq_mc" in forms:   # one request at a time, each in the matrix-core form
        out["matrix_core_per_request"], _ = serve_run(reqs, Xown, 1, budget, matrix_core=True)
        log("serve matrix-core per-request: %s" % json.dumps(out["matrix_core_per_request"]))
    if "closed" in forms:
        out["batched_closed"], closed_outs = serve_run(reqs, Xown, args.slots, budget)
        log("serve batched closed loop: %s" % json.dumps(out["batched_closed"]))
    if "open" in forms:
        out["batched_open"], _ = serve_run(reqs, Xown, args.slots, budget, open_loop=True)
        log("serve batched open loop: %s" % json.dumps(out["batched_open"]))
    if "mc" in forms:
        out["batched_closed_matrix_core"], mc_outs = serve_run(reqs, Xown, args.slots, budget,
                                                               matrix_core=True)
        if closed_outs is not None:
            # principal-angle sine of each U_k against the FP64-step batched run
            sins = {"f32": [], "bf16": []}
            for r, a, b in zip(reqs, closed_outs, mc_outs):
                Ua, Ub = a[1].contiguous(), b[1].contiguous()
                sins[r["storage"]].append(
                    float(torch.linalg.matrix_norm(Ub - Ua @ (Ua.T @ Ub), ord=2)))
            out["batched_closed_matrix_core"]["max_sin_vs_fp64_steps"] = {
                k: max(v) if v else None for k, v in sins.items()}
            out["matrix_core_agrees"] = all(
                v is None or v <= (1e-6 if kk == "f32" else 1e-3) for kk, v in
                out["batched_closed_matrix_core"]["max_sin_vs_fp64_steps"].items())
        log("serve batched closed loop, matrix-core steps: %s" %
            json.dumps(out["batched_closed_matrix_core"]))
        # the same form against the arrival process: served as requests arrive
        out["batched_open_matrix_core"], mco_outs = serve_run(reqs, Xown, args.slots, budget,
                                                              open_loop=True, matrix_core=True)
        # every result is bitwise the same whichever requests shared the device with it
        same_mc = [torch.equal(a[1], b[1]) for a, b in zip(mc_outs, mco_outs)]
        out["matrix_core_closed_equals_open"] = "%d/%d" % (sum(same_mc), len(same_mc))
        out["matrix_core_mix_invariant"] = all(same_mc)
        log("serve batched open loop, matrix-core: %s" %
            json.dumps(out["batched_open_matrix_core"]))
    if seq_outs is not None and closed_outs is not None:
        same = [torch.equal(a[1], b[1]) for r, a, b in zip(reqs, seq_outs, closed_outs)
                if r["storage"] == "f32"]
        out["f32_bitwise_alone_vs_mix"] = "%d/%d" % (sum(same), len(same))
        out["alone_equals_mix"] = all(same)
        out["speedup_batched_vs_fp32_per_request"] = \
            out["batched_closed"]["solves_per_s"] / out["fp32_per_request"]["solves_per_s"]
        if "batched_closed_matrix_core" in out:
            out["speedup_matrix_core_batched_vs_fp32_per_request"] = \
                out["batched_closed_matrix_core"]["solves_per_s"] / \
                out["fp32_per_request"]["solves_per_s"]
    failed = [name for name in ("fp32_per_request", "matrix_core_per_request", "batched_closed",
                                "batched_open", "batched_closed_matrix_core",
                                "batched_open_matrix_core")
              if name in out and out[name]["failed"]]
    out["consistent"] = (not failed and out.get("alone_equals_mix", True) and
                         out.get("matrix_core_agrees", True) and
                         out.get("matrix_core_mix_invariant", True))
    return out


def serve_consistency_exit(serve):
    """Non-zero exit when the serving legs disagree with themselves: a request
    that failed, an FP32 request whose U_k is not bitwise the same alone and in
    the mix, or a matrix-core result off the FP64-step one."""
    if serve is not None and not serve.get("consistent", True):
        log("serving results are inconsistent (failed requests, alone != mix, or "
            "matrix-core != FP64 steps); see the serve object")
        sys.exit(3)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads
    from paper_1607_02925_amd import lowrank

    lowrank.load_library()
    dev = "cuda:0"
    if args.mode == "serve":
        out = serve_bench(args, dev)
        print(json.dumps({"mode": "serve", **out}), flush=True)
        serve_consistency_exit(out)
        return
    if args.mode == "sparse":
        out = sparse_bench(args, dev)
        print(json.dumps({"mode": "sparse", **out}), flush=True)
        return
    if args.mode == "sparse-solve":
        out = sparse_solve(args, dev)
        print(json.dumps({"mode": "sparse-solve", **out}), flush=True)
        return
    if args.mode == "steps":
        out = steps_bench(args, dev)
        print(json.dumps({"mode": "steps", **out}), flush=True)
        return
    w = dict(workloads.WORKLOADS[args.workload])
    t0 = time.time()
    data = workloads.workload(args.workload, device=dev)
    Xt = data["Xt"]
    torch.cuda.synchronize()
    log("generated %s on the GPU in %.1fs" % (args.workload, time.time() - t0))
    x_bytes = Xt.numel() * Xt.element_size()
    d, n, k, p = w["d"], w["n"], w["k"], w["p"]

    if args.mode == "copy":
        dst = torch.empty_like(Xt)
        for _ in range(args.warmup):
            dst.copy_(Xt)
        torch.cuda.synchronize()
        t = time.time()
        for _ in range(args.steps):
            dst.copy_(Xt)
        torch.cuda.synchronize()
        dt = (time.time() - t) / args.steps
        print(json.dumps({"mode": "copy", "bytes_read": x_bytes, "bytes_written": x_bytes,
                          "ms": dt * 1e3, "GBps": 2 * x_bytes / dt / 1e9}), flush=True)
        return

    plan = lowrank.Plan(Xt, k, p, w["eps"], seed=w["solver_seed"], timing=1,
                        adaptive=args.adaptive, accel=args.accel, precision=args.precision)

    if args.mode == "pass":
        Wm = torch.randn((p, d), dtype=torch.float64, device=dev).T
        for _ in range(args.warmup):
            plan.apply_A(Wm)
        torch.cuda.synchronize()
        t = time.time()
        for _ in range(args.steps):
            plan.apply_A(Wm)
        torch.cuda.synchronize()
        dt = (time.time() - t) / args.steps
        print(json.dumps({"mode": "pass", "ms": dt * 1e3, "x_bytes": x_bytes,
                          "GBps_alg": x_bytes / dt / 1e9}), flush=True)
        return

    if args.mode == "epoch":
        # schedule of the same workload (shift 101.647, b 2048, m 124 for this seed)
        lam, eta, m, b = 101.64710238615051, 0.009837925024862453, 124, 2048
        plan.prepare()
        S = torch.linalg.qr(torch.randn((d, p), dtype=torch.float64, device=dev))[0]
        plan.svrg_solve(S, lam, eta, m, b, 1, 1)
        torch.cuda.synchronize()
        t = time.time()
        for i in range(args.steps):
            plan.svrg_solve(S, lam, eta, m, b, 2 + i, 1)
        torch.cuda.synchronize()
        dt = (time.time() - t) / args.steps
        print(json.dumps({"mode": "epoch", "ms": dt * 1e3, "m": m, "b": b,
                          "ms_per_step_incl_passes": dt * 1e3 / m}), flush=True)
        return

    for i in range(args.warmup):
        st, U, theta, rep = plan.solve()
        log("warmup %d: status %d outer %d epochs %d" % (i, st, rep["outer"],
                                                         rep["total_epochs"]))
    torch.cuda.synchronize()
    lat = []
    reps = []
    t_start = time.time()
    for i in range(args.steps):
        ts = time.time()
        st, U, theta, rep = plan.solve()
        torch.cuda.synchronize()
        lat.append(time.time() - ts)
        reps.append(rep)
        log("step %d: %.3fs status %d outer %d epochs %d passes %d steps %d" %
            (i, lat[-1], st, rep["outer"], rep["total_epochs"], rep["passes"], rep["steps"]))
    torch.cuda.synchronize()
    total = time.time() - t_start
    sched = plan.schedule()
    rep = reps[-1]

    # dominant kernel among the inner-step pair (each gathers b columns of X)
    sx = Xt.element_size()
    b = sched.b
    PCw = lowrank_pad16(p)
    if args.precision in (0, 3):
        names = ("k_step_update", "k_xtm_gathered")
        bytes_update = b * d * sx + b * PCw * 8 + 3 * d * p * 8
        bytes_sdot = b * d * sx + d * PCw * 8 + b * PCw * 8 + b * 12
    else:
        form = "bf16" if (args.precision == 1 or (args.precision == 4 and sx == 2)) else "f32"
        names = ("k_supd_" + form, "k_sdot_" + form)
        cb = 4 if form == "f32" else 4          # C as FP32 (or two BF16 parts)
        bytes_update = b * d * sx + b * PCw * cb + 3 * d * p * 8 + d * PCw * cb
        bytes_sdot = b * d * sx + d * PCw * cb + b * PCw * cb + b * 12
    probes = sum(r["probes"] for r in reps)
    ms_upd = sum(r["ms_update_probe"] for r in reps) / max(probes, 1)
    ms_sdot = sum(r["ms_sample_dot_probe"] for r in reps) / max(probes, 1)
    ms_pass = sum(r["ms_pass_total"] for r in reps) / max(sum(r["timed_passes"] for r in reps), 1)
    t_upd_total = ms_upd * rep["steps"]
    t_sdot_total = ms_sdot * rep["steps"]
    t_pass_total = ms_pass * rep["passes"]
    kernels = {
        names[0]: (t_upd_total, bytes_update, ms_upd),
        names[1]: (t_sdot_total, bytes_sdot, ms_sdot),
    }
    dom = max(kernels, key=lambda kk: kernels[kk][0])
    _, dbytes, dms = kernels[dom]
    achieved = dbytes / (dms * 1e-3) / 1e9 if dms > 0 else None
    # the pass: |X| + 3 d p 4 algorithmic bytes (X once, W~ and S in, G~ out)
    pass_bytes = x_bytes + 3 * d * p * 4
    pass_gbs = pass_bytes / (ms_pass * 1e-3) / 1e9 if ms_pass > 0 else None
    mc = args.precision in (3, 4)
    dtype = {0: "f64", 1: "f64+bf16-steps", 2: "f64+f32-steps",
             3: "bf16x3-passes(f32-acc)+f64",
             4: "bf16x3-passes(f32-acc)+%s-steps+f64" % ("bf16" if sx == 2 else "f32")}
    out = {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype.get(args.precision, "f64"),
        "data": "synthetic planted-spectrum matrix generated on the GPU from fixed seeds",
        "config": {"workload": args.workload, "d": d, "n": n, "k": k, "p": p, "eps": w["eps"],
                   "storage": w["storage"], "form": "per-request", "precision": args.precision,
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": percentile(lat, 0.5) * 1e3, "p99": percentile(lat, 0.99) * 1e3},
        "pass": {"kernels": "k_mc_split_w + k_mc_xtw + k_mc_xt + k_mc_reduce" if mc
                 else "k_cm_to_tile + k_xtm + k_xt_part + k_reduce_y",
                 "ms": ms_pass, "bytes_alg": pass_bytes, "hbm_GBps_alg": pass_gbs,
                 "frac_hbm": pass_gbs / PEAK_HBM_GBS if pass_gbs else None,
                 "x_reads_per_pass": 2},
        "solve": {"status": st, "outer": rep["outer"], "epochs": rep["total_epochs"],
                  "passes": rep["passes"], "mc_passes": rep["mc_passes"],
                  "inner_steps": rep["steps"],
                  "shift_rounds": rep["shift_rounds"], "lambda": sched.lam, "m": sched.m,
                  "b": sched.b, "share_update": t_upd_total / (total / args.steps * 1e3),
                  "share_sample_dot": t_sdot_total / (total / args.steps * 1e3),
                  "share_pass": t_pass_total / (total / args.steps * 1e3)},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS if achieved else None,
                     "traffic": measured_traffic(dom, args.workload),
                     "bytes_per_launch": dbytes, "avg_launch_ms": dms},
        "cpu_baseline": None,
    }
    if args.adaptive or args.accel:
        out["config"]["variant"] = {"adaptive": args.adaptive, "accel": args.accel}
    elif not args.no_variants:
        if args.precision != 0:
            out["f64"] = variant_leg(Xt, w, U, args, "f64", precision=0)
        if args.precision != 2 and Xt.dtype != torch.float64:
            out["f32_steps"] = variant_leg(Xt, w, U, args, "f32-steps", precision=2)
        out["adaptive"] = variant_leg(Xt, w, U, args, "adaptive", adaptive=1)
        out["accel"] = variant_leg(Xt, w, U, args, "accel", accel=1)
        out["adaptive_accel"] = variant_leg(Xt, w, U, args, "adaptive+accel", adaptive=1,
                                            accel=1)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(Xt, dict(w, **data), sched, rep)
    if not args.no_legs or not args.no_serve:
        del Xt, data, plan
        torch.cuda.empty_cache()
    if not args.no_legs:
        out["bf16_4096x500000"] = big_dense_leg(args, dev, "planted-4096x500000-bf16")
        torch.cuda.empty_cache()
        out["csc_50000x1000000"] = sparse_bench(args, dev)
        torch.cuda.empty_cache()
        out["accel_csc_600x5000"] = accel_leg(args, dev)
    if not args.no_serve:
        out["serve"] = serve_bench(args, dev)
    print(json.dumps(out), flush=True)
    serve_consistency_exit(out.get("serve"))


if __name__ == "__main__":
    main()
