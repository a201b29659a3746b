"""Benchmark: MLMC gradient estimates/s of the entropic-risk MLSGD hot path on
one MI355X.

A step is one complete MLMC gradient estimate (draws, batched state solves on
every level, misfits, batched adjoint solves, max-shifted weights, level
means, telescoping, gradient) with fresh samples, inputs resident in HBM.
Headline workload: levels 9^3..129^3 with M = 4096/1024/256/64/16, FP64
MG-PCG to rtol 1e-12, theta = 1, alpha = 1e-3, u = 0.1 xyz,
y_d = sin(pi x) sin(pi y) sin(pi z) (synthetic, seed 0).  The mixed-precision
form (FP32 V-cycles inside the FP64 Krylov iteration, sigma^2 = 2,
theta = 10, same grids and counts) is reported beside it.

Prints one JSON line.  --gpus N > 1 is not supported (one GPU per run).
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLMC gradient estimates/s + state/adjoint solves/s, mixed vs FP64, % HBM peak"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILES = {  # committed counter summaries of the timed kernel, by timing kind
    2: os.path.join(ROOT, "profiles", "traffic_post_smoothing_129.json"),
}
# Bytes per interior point of the timed kernels by timing kind and element
# size: the algorithmic bytes (coefficient regenerated, so 0 bytes) and the
# per-call coefficient cache the kernels read on top of them.
#   kind 2, fused post-smoothing pass: x and b read, x'' written, coarse
#     correction read once (1/8 point);
#   kind 1, plain smoothing step: x and b read, x' written.
#   kind 3, fused pre-smoothing pass: b read, x2 written, the x-restricted
#     residual written on every second plane;
#   kind 4, Krylov matvec: z read, p_old read, p_new and q written, x read
#     and written by the deferred step (z in FP32 under FP32 V-cycles).
ALG_BYTES_PER_POINT = {2: lambda e: 3.0 * e + e / 8.0, 1: lambda e: 3.0 * e,
                       3: lambda e: 2.5 * e}
# (kind 1 also has launches from a zero start, 2e, and with a folded
# correction, 3e + e/8; kind 4's first iteration of a solve applies no x
# step, 32 instead of 48 B; the library reports each launch's own bytes)
CACHE_BYTES_PER_POINT = {"fp64": 8.0, "mixed": 4.0, "mixed_bf16": 2.0}
ELEM_BYTES = {"fp64": 8.0, "mixed": 4.0, "mixed_bf16": 4.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mlmc_129")
    ap.add_argument("--mixed-workload", default="mlmc_129_mixed")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-per-sample", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="run the main workload as one replayed HIP graph per estimate")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the single-level SGD and 257^3 batched legs")
    ap.add_argument("--mlsgd", action="store_true",
                    help="run the adaptive MLSGD optimisation on the 257^3 workload instead")
    ap.add_argument("--mlsgd-steps", type=int, default=50)
    ap.add_argument("--rates", action="store_true",
                    help="level rates (alpha, beta, gamma) of the 129^3 hierarchy per theta")
    ap.add_argument("--thetas", default="1,5,10")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    ap.add_argument("--odd-size", action="store_true",
                    help="only run the batch of 300 independent odd-size solves")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def problem_counts(grid, M):
    """Solves per estimate (state and adjoint counted separately) and the
    interior unknowns they cover."""
    solves, unknowns = 0, 0
    for i, n in enumerate(grid):
        solves += 2 * M[i]
        unknowns += 2 * M[i] * (n - 2) ** 3
        if i > 0:
            solves += 2 * M[i]
            unknowns += 2 * M[i] * (grid[i - 1] - 2) ** 3
    return solves, unknowns


def make_ctx(m, w, dev):
    prec = {"fp64": m.FP64, "mixed": m.MIXED_FP32, "mixed_bf16": m.MIXED_BF16}[w.precision]
    solver = m.SOLVER_CG if w.solver == "cg" else m.SOLVER_MGPCG
    pb = m.Problem(grid_n=w.grid_n, y_d=w.y_d(), f=w.f() if w.f_value else None, seed=w.seed,
                   K=w.K, sigma2=w.sigma2, theta=w.theta, alpha=w.alpha, precision=prec,
                   solver=solver, rtol=w.rtol, max_iters=200, law=w.law, rho=w.rho)
    return m.Context(pb, device=dev)


def run(args, m, w, dev, steps, warmup, timing_n=None, graph=False, timing_kind=2, u0=None):
    """Warm up, then time `steps` estimates with fresh samples each.  graph:
    the first warm-up call captures the batch shape as a HIP graph and every
    later call replays it (no event timing then).  timing_kind selects the
    kernel timed on grid timing_n: 2 the fused post-smoothing pass, 1 the
    plain smoothing step, 3 the fused pre-smoothing pass, 4 the Krylov
    matvec."""
    import torch
    ctx = make_ctx(m, w, dev)
    if graph:
        ctx.set_graph(True)
        timing_n = None
        warmup = max(warmup, 1)
    u = torch.as_tensor(w.u0() if u0 is None else u0, device=dev).contiguous()
    L = len(w.grid_n)
    off = [0] * L
    for k in range(warmup):
        g, st = ctx.mlmc_gradient(u, w.M, first=off)
        off = [o + mm for o, mm in zip(off, w.M)]
        log(args, f"  warmup {k}: {st['ms_total']:.2f} ms, iters "
                  f"{st['iters_state']}/{st['iters_adjoint']}")
    if timing_n:
        ctx.kernel_timing(timing_kind, timing_n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(steps):
        g, st = ctx.mlmc_gradient(u, w.M, first=off)
        off = [o + mm for o, mm in zip(off, w.M)]
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = ctx.kernel_timing(0, 0) if timing_n else None
    ctx.close()
    return {"dt": dt, "stats": stats, "timing": tm, "grad": g}


KERNEL_NAMES = {
    2: ("fused post-smoothing pass (k_post2: coarse-grid correction folded in, two Chebyshev "
        "steps, cached 1/a) on the {n}^3 rows"),
    1: "Chebyshev smoothing step (k_march OP_JAC, damped Jacobi, cached 1/a) on the {n}^3 rows",
    3: ("fused pre-smoothing pass (k_pre2r: two Chebyshev steps from zero, residual restricted "
        "along x, cached 1/a and 1/D) on the {n}^3 rows"),
    4: ("Krylov matvec (k_march OP_MATVEC: p = z + beta p, q = A p, deferred x step, cached 1/a) "
        "on the {n}^3 rows"),
}


def other_kernel_rooflines(args, m, w, dev, nfin):
    """Live roofline records of the fused pre-smoothing pass and the Krylov
    matvec on the finest grid, each from its own short host-driven run of the
    same workload after the timed region (one kernel is timed per run)."""
    recs = []
    for kind in (3, 4):
        tm = run(args, m, w, dev, 2, 1, timing_n=nfin, timing_kind=kind)["timing"]
        rec = roofline(tm, kind, nfin, w.precision)
        rec.pop("traffic", None)
        recs.append(rec)
    return recs


def dominant_timing(args, m, w, dev, tm, nfin):
    """Event totals of the dominant smoothing kernel on the finest grid: the
    fused post-smoothing pass where the run used it, else the plain smoothing
    step (timed in a short host-driven pass, as are graph runs, whose replays
    carry no per-launch events).  Returns (totals, kind)."""
    if tm is None:
        log(args, "host-driven pass for the kernel timing")
        tm = run(args, m, w, dev, 2, 1, timing_n=nfin, timing_kind=2)["timing"]
    if tm["launches"]:
        return tm, 2
    log(args, "no fused post-smoothing pass on the finest grid: timing the plain step")
    return run(args, m, w, dev, 2, 1, timing_n=nfin, timing_kind=1)["timing"], 1


def same_samples_error(m, w_fast, w_ref, dev):
    """Relative L2 difference of one estimate of w_fast against the FP64 GPU
    path on identical samples and problem data (the FP64 path itself matches
    the oracle in the parity tests)."""
    import dataclasses
    import torch
    w64 = dataclasses.replace(w_ref, precision="fp64")
    u = torch.as_tensor(w_fast.u0(), device=dev).contiguous()
    c1 = make_ctx(m, w_fast, dev)
    g1, _ = c1.mlmc_gradient(u, w_fast.M)
    c1.close()
    c2 = make_ctx(m, w64, dev)
    g2, _ = c2.mlmc_gradient(u, w64.M)
    c2.close()
    return float(torch.linalg.norm(g1 - g2) / torch.linalg.norm(g2))


def per_sample_fp64(m, w, dev, reps=2):
    """The plain FP64 GPU solver without batching: state and adjoint solves of
    one sample per call (same kernels, one problem per launch sequence), timed
    per grid and extrapolated to the workload's sample counts."""
    import dataclasses
    import torch
    w64 = dataclasses.replace(w, precision="fp64")
    ctx = make_ctx(m, w64, dev)
    u = torch.as_tensor(w64.u0(), device=dev).contiguous()
    per = []
    for i in range(len(w64.grid_n)):
        t_level = 0.0
        for coarse in ([0, 1] if i > 0 else [0]):
            ctx.solve_state_adjoint(i, coarse, 0, 1, u, want_y=False)   # warm the plan
            torch.cuda.synchronize()
            t = time.perf_counter()
            for r in range(reps):
                ctx.solve_state_adjoint(i, coarse, 1 + r, 1, u, want_y=False)
            torch.cuda.synchronize()
            t_level += (time.perf_counter() - t) / reps
        per.append(t_level)
    ctx.close()
    est = sum(mm * tp for mm, tp in zip(w64.M, per))
    return {"value": 1.0 / est, "unit": "gradient estimates/s",
            "seconds_per_sample_by_level": per,
            "sample": f"{reps} samples per grid after one warm-up call, extrapolated to M={list(w64.M)}"}


def single_level_sgd(m, dev, steps=5):
    """The single-level workload: 17^3, 64 fresh samples per step, CG to 1e-12,
    theta = 1, alpha = 1e-3, u_0 = 0, five projected steps with tau = 10."""
    import torch
    from paper_2606_09291_amd import inputs
    w = inputs.WORKLOADS["single_level_17"]
    ctx = make_ctx(m, w, dev)
    u = torch.zeros((w.grid_n[0],) * 3, dtype=torch.float64, device=dev)
    ctx.set_batch(w.M)
    ctx.step(u, w.tau)        # warm-up step (plan build)
    u.zero_()
    ctx.set_batch(w.M)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for j in range(steps):
        st = ctx.step(u, w.tau)
        recs.append({"J": st["grad"]["J"], "grad_norm": st["grad"]["grad_norm"],
                     "iters": st["grad"]["iters_state"]})
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return {"workload": w.name, "steps_per_s": steps / dt, "ms_per_step": 1e3 * dt / steps,
            "records": recs}


def odd_size_solves(m, dev, reps=3):
    """The batch of 300 independent state solves on grids of random size in
    {33, 41, 49, 57, 65} (f = 1, u = 0) that accompanies the 257^3 MLMC
    workload, in its precision (mixed) and tolerance."""
    import torch
    from paper_2606_09291_amd import inputs
    cfg = inputs.ODD_SOLVES
    w = inputs.WORKLOADS["mlmc_257_batched"]
    sizes = inputs.odd_sizes(cfg["count"], seed=cfg["seed"], level=cfg["level"],
                             first=cfg["first"])
    ctx = make_ctx(m, w, dev)
    ctx.solve_sizes(sizes, level=cfg["level"], first=cfg["first"], f_value=cfg["f_value"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        _, st = ctx.solve_sizes(sizes, level=cfg["level"], first=cfg["first"] + r * cfg["count"],
                                f_value=cfg["f_value"])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ctx.close()
    unknowns = sum((n - 2) ** 3 for n in sizes)
    return {"workload": f"{len(sizes)} state solves, grids of random size in {list(inputs.ODD_SIZES)}, "
                        f"f = 1, {w.precision}",
            "solves_per_s": len(sizes) / dt, "ms_per_batch": 1e3 * dt,
            "unknown_solves_per_s": unknowns / dt, "iterations": st["iterations"],
            "max_relres": st["max_relres"]}


def run_rates(args):
    """Level rates of the 9^3..129^3 hierarchy (FP64) for each theta: per
    level |E dX|, Var dX, |E dY| averaged over a few estimates with fresh
    samples, the cost per sample from level-by-level batched solves (measured
    time and the work model interior unknowns x iterations), and the fitted
    alpha, beta, gamma and constants (rates.py)."""
    import dataclasses
    import torch
    import paper_2606_09291_amd as m
    from paper_2606_09291_amd import inputs, rates
    dev = torch.device("cuda:0")
    base = inputs.WORKLOADS["mlmc_129"]
    E = max(2, args.steps)
    out = {"mode": "rates", "workload": base.name, "estimates_per_theta": E, "runs": []}
    for th in [float(t) for t in args.thetas.split(",")]:
        w = dataclasses.replace(base, theta=th)
        ctx = make_ctx(m, w, dev)
        u = torch.as_tensor(w.u0(), device=dev).contiguous()
        L = len(w.grid_n)
        acc = None
        off = [0] * L
        for k in range(E):
            _, st = ctx.mlmc_gradient(u, w.M, first=off)
            off = [o + mm for o, mm in zip(off, w.M)]
            e, V, wy = rates.level_statistics(st, w.M, th)
            cur = [e, V, wy]
            acc = cur if acc is None else [[a + b for a, b in zip(x, y)] for x, y in zip(acc, cur)]
        e, V, wy = [[x / E for x in row] for row in acc]
        t_meas, work = [], []
        for lv in range(L):
            cnt = int(w.M[lv])
            tot_t, tot_w = 0.0, 0.0
            for coarse in ((0, 1) if lv > 0 else (0,)):
                n = w.grid_n[lv - coarse]
                ctx.solve_state_adjoint(lv, coarse, off[lv], cnt, u, want_y=False)  # warm
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, _, sst = ctx.solve_state_adjoint(lv, coarse, off[lv], cnt, u, want_y=False)
                torch.cuda.synchronize()
                tot_t += (time.perf_counter() - t0) / cnt
                tot_w += (n - 2) ** 3 * sst["iterations"]
            t_meas.append(tot_t)
            work.append(tot_w)
        ctx.close()
        fit_t = rates.fit_rates(w.grid_n, e, V, wy, t_meas)
        fit_w = rates.fit_rates(w.grid_n, e, V, wy, work)
        rec = {"theta": th, "grid": w.grid_n, "M": w.M, "norm_mean_dX": e, "var_dX": V,
               "abs_mean_dY": wy, "seconds_per_sample": t_meas, "work_per_sample": work,
               "fit": {k: fit_w[k] for k in ("alpha", "beta", "alpha_Y", "C_X", "C_V", "C_Y")},
               "gamma_work": fit_w["gamma"], "gamma_measured": fit_t["gamma"]}
        out["runs"].append(rec)
        log(args, f"theta {th}: alpha {fit_w['alpha']:.3f} beta {fit_w['beta']:.3f} "
                  f"gamma(work) {fit_w['gamma']:.3f} gamma(time) {fit_t['gamma']:.3f}")
    print(json.dumps(out))


def mlsgd_run(args, m, w, dev, theta, steps):
    """Adaptive MLSGD (Algorithm 1) on workload w at theta: projected steps
    with step size 1/(1+j), batch sizes chosen by the controller after every
    step.  Returns the wall time and the per-step records."""
    import dataclasses
    import torch
    wt = dataclasses.replace(w, theta=theta)
    ctx = make_ctx(m, wt, dev)
    u = torch.as_tensor(wt.u0(), device=dev).contiguous()
    ctx.set_batch(wt.M)
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(steps):
        st = ctx.step(u, 1.0 / (1.0 + j), adapt=True)
        g = st["grad"]
        recs.append({"step": j, "J": g["J"], "grad_norm": g["grad_norm"], "M": st["M_next"],
                     "err_sam": st["err_sam"], "err_num": st["err_num"], "eps": st["eps"],
                     "iters": [g["iters_state"], g["iters_adjoint"]], "ms": g["ms_total"]})
        log(args, f"theta {theta} step {j}: J {g['J']:.6e} |g| {g['grad_norm']:.4e} "
                  f"M_next {st['M_next']} {g['ms_total']:.1f} ms")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return dt, recs


def run_mlsgd(args):
    """Adaptive MLSGD for every theta of --thetas, with every step's record."""
    import torch
    import paper_2606_09291_amd as m
    from paper_2606_09291_amd import inputs
    w = inputs.WORKLOADS["adaptive_257"]
    dev = torch.device("cuda:0")
    out = {"workload": w.name, "runs": []}
    for th in [float(x) for x in args.thetas.split(",")]:
        dt, recs = mlsgd_run(args, m, w, dev, th, args.mlsgd_steps)
        out["runs"].append({"theta": th, "seconds": dt, "steps": args.mlsgd_steps,
                            "final_J": recs[-1]["J"], "final_grad_norm": recs[-1]["grad_norm"],
                            "records": recs})
    print(json.dumps(out), flush=True)


def autograd_leg(m, dev, reps=3):
    """The autograd objective J(u) at 65^3 with 256 samples (single level,
    FP64, rtol 1e-12) and its backward pass, timed separately after one
    warm-up pass."""
    import torch
    from paper_2606_09291_amd import inputs
    from paper_2606_09291_amd.autograd import objective
    yd = inputs.target_sin(65)
    ctx = m.Context(m.Problem(grid_n=[65], y_d=yd, theta=1.0, alpha=1e-3, rtol=1e-12))
    u0 = torch.as_tensor(inputs.control_xyz(65), device=dev).contiguous()
    fwd = bwd = 0.0
    for r in range(reps + 1):
        u = u0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = objective(u, ctx, [256], [256 * r])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r > 0:
            fwd += t1 - t0
            bwd += t2 - t1
    ctx.close()
    return {"workload": "autograd J(u) and dJ/du, 65^3, 256 samples, FP64 MG-PCG, rtol 1e-12",
            "forward_ms": 1e3 * fwd / reps, "backward_ms": 1e3 * bwd / reps,
            "value": reps / (fwd + bwd), "unit": "forward+backward passes/s"}


def adaptive_leg(args, m, dev):
    """The adaptive MLSGD run at theta = 1 in the default bench line: its
    50 steps' wall time and outcome (the controller's batches per step are
    in bench.py --mlsgd)."""
    from paper_2606_09291_amd import inputs
    w = inputs.WORKLOADS["adaptive_257"]
    dt, recs = mlsgd_run(args, m, w, dev, 1.0, w.steps)
    return {"workload": w.name + ", theta=1, mixed, rtol 1e-10", "steps": w.steps,
            "seconds": dt, "steps_per_s": w.steps / dt,
            "ms_per_step_after_first": sum(r["ms"] for r in recs[1:]) / max(1, len(recs) - 1),
            "J_first": recs[0]["J"], "J_final": recs[-1]["J"],
            "grad_norm_first": recs[0]["grad_norm"], "grad_norm_final": recs[-1]["grad_norm"],
            "M_final": recs[-1]["M"], "iters_final": recs[-1]["iters"]}


def level_rates(w, stats):
    """Level rates of the headline hierarchy from the timed estimates
    (fresh samples each): per-level |E dX_l|, Var dX_l and |E dY_l| averaged
    over the estimates, then the least-squares exponents alpha (weak error),
    beta (variance) and alpha_Y over the levels l >= 1 (rates.py).  gamma is
    the exponent of the work per sample: interior unknowns of the fine and
    coarse grid times the estimate's state plus adjoint iterations."""
    from paper_2606_09291_amd import rates
    acc = None
    for st in stats:
        cur = rates.level_statistics(st, w.M, w.theta)
        acc = cur if acc is None else [[a + b for a, b in zip(x, y)] for x, y in zip(acc, cur)]
    e, V, wy = [[x / len(stats) for x in row] for row in acc]
    it = max(s["iters_state"] for s in stats) + max(s["iters_adjoint"] for s in stats)
    work = []
    for i, n in enumerate(w.grid_n):
        u = (n - 2) ** 3 + ((w.grid_n[i - 1] - 2) ** 3 if i else 0)
        work.append(float(u * it))
    fit = rates.fit_rates(w.grid_n, e, V, wy, work)
    return {"estimates": len(stats), "alpha": fit["alpha"], "beta": fit["beta"],
            "alpha_Y": fit["alpha_Y"], "gamma_work": fit["gamma"], "C_X": fit["C_X"],
            "C_V": fit["C_V"], "norm_mean_dX": e, "var_dX": V, "abs_mean_dY": wy}


def host_threads():
    """Host threads the oracle may use: the CPUs this process may run on,
    bounded by OMP_NUM_THREADS where the environment sets it (the share of
    the host that comes with one GPU)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def first_estimate(m, w, dev):
    """One estimate of workload w at sample offsets 0 (the draws the oracle
    reproduces for the accuracy figures), as a host array."""
    import torch
    ctx = make_ctx(m, w, dev)
    u = torch.as_tensor(w.u0(), device=dev).contiguous()
    g, _ = ctx.mlmc_gradient(u, w.M, first=[0] * len(w.M))
    ctx.close()
    return g.cpu().numpy()


def cpu_baseline(w, threads, acc_grads):
    """The oracle on the host cores.  Baseline: one complete estimate of the
    headline workload w (every pair of every level, offsets 0) on `threads`
    OpenMP threads, timed.  Accuracy: the relative L2 error of each GPU
    estimate in acc_grads (same workload data and draws) against the oracle's
    estimate of it; workloads sharing problem data share one oracle run."""
    import numpy as np
    import oracle
    pb = oracle.make_problem(w.grid_n, K=w.K, sigma2=w.sigma2, theta=w.theta, alpha=w.alpha,
                             rtol=w.rtol, nthreads=threads)
    t = time.perf_counter()
    g_ref, st = oracle.mlmc_gradient(pb, w.f() if w.f_value else None, w.u0(), w.y_d(), w.M,
                                     first=[0] * len(w.M))
    sec = time.perf_counter() - t
    base = {"value": 1.0 / sec, "unit": "gradient estimates/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"one complete estimate of the headline workload (M={list(w.M)}, "
                       f"{sum(w.M)} level pairs, state and adjoint solves), FP64 MG-PCG to "
                       f"rtol {w.rtol}, OpenMP over the pairs"),
            "seconds_per_estimate": sec, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
            else None,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS"),
            "cpu_model": cpu_model(), "oracle_max_iters": st["max_iters"]}
    refs = {}

    def key_of(wk):
        return (tuple(wk.grid_n), tuple(wk.M), wk.K, wk.sigma2, wk.theta, wk.alpha, wk.f_value,
                wk.law, wk.rho, wk.seed)

    refs[key_of(w)] = g_ref
    errs = {}
    for name, (wk, g) in acc_grads.items():
        k = key_of(wk)
        if k not in refs:
            pbk = oracle.make_problem(wk.grid_n, K=wk.K, sigma2=wk.sigma2, theta=wk.theta,
                                      alpha=wk.alpha, rtol=1e-12, nthreads=threads)
            refs[k], _ = oracle.mlmc_gradient(pbk, wk.f() if wk.f_value else None, wk.u0(),
                                              wk.y_d(), wk.M, first=[0] * len(wk.M))
        r = refs[k]
        errs[name] = float(np.linalg.norm(g - r) / np.linalg.norm(r))
    return base, errs


def roofline(tm, kind, n, precision):
    """Roofline record of the timed kernel: algorithmic bytes per launch (the
    interior points times ALG_BYTES_PER_POINT) over its average launch time
    from live HIP events, against 8 TB/s.  The coefficient-cache bytes the
    kernel also reads are reported beside, not counted."""
    launches = tm["launches"]
    if not launches:
        return {"kernel": KERNEL_NAMES[kind].format(n=n), "bound": "hbm", "achieved": None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None, "traffic": None}
    avg_ms = tm["ms"] / launches
    alg = tm["bytes"] / launches
    e = ELEM_BYTES[precision]
    achieved = alg / (avg_ms * 1e-3) / 1e9
    # kind 2 and 3 launches all move the same bytes per point; kinds 1 and 4
    # mix launches of different bytes, so their point count is not derived
    points = alg / ALG_BYTES_PER_POINT[kind](e) if kind in (2, 3) else None
    cache = points * CACHE_BYTES_PER_POINT[precision] if points else None
    return {
        "kernel": KERNEL_NAMES[kind].format(n=n),
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic_for(alg, kind),
        "avg_launch_ms": avg_ms,
        "launches": launches,
        "algorithmic_bytes_per_launch": alg,
        "algorithmic_bytes_per_point": (ALG_BYTES_PER_POINT[kind](e) if kind in ALG_BYTES_PER_POINT
                                        else None),
        "interior_points_per_launch": points,
        "coefficient_cache_bytes_per_launch": cache,
        "frac_with_cache_bytes": ((alg + cache) / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                  if cache else None),
    }


def source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "runtime.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_2606_09291_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(launch_bytes, kind):
    """HBM bytes per launch of the timed kernel: the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factors) gives traffic
    over algorithmic bytes for these launches; None when there is none for
    this kernel or the kernels changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILES[kind]) as fh:
            t = json.load(fh)
    except (KeyError, OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash():
        return None
    return t["traffic_over_algorithmic"] * launch_bytes


def copy_calibration(args):
    import torch
    n = 1 << 27  # 128 Mi doubles = 1 GiB each way
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 5}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args)
        return
    if args.odd_size:
        import torch
        import paper_2606_09291_amd as m
        print(json.dumps(odd_size_solves(m, torch.device("cuda:0"))), flush=True)
        return
    if args.rates:
        run_rates(args)
        return
    if args.mlsgd:
        run_mlsgd(args)
        return
    import torch
    import paper_2606_09291_amd as m
    from paper_2606_09291_amd import inputs

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    w = inputs.WORKLOADS[args.workload]
    nfin = w.grid_n[-1]
    log(args, f"workload {args.workload}: grids {w.grid_n} M {w.M} ({w.precision})")
    r = run(args, m, w, dev, args.steps, args.warmup, timing_n=nfin, graph=args.graph)
    dt = r["dt"]
    stats = r["stats"]
    log(args, f"timed {args.steps} steps in {dt:.3f} s")
    solves, unknowns = problem_counts(w.grid_n, w.M)
    value = args.steps / dt
    acc_grads = {"fp64": (w, first_estimate(m, w, dev))}
    tm, kind = dominant_timing(args, m, w, dev, r["timing"], nfin)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "gradient estimates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grids": w.grid_n, "M": w.M, "K": w.K,
                   "sigma2": w.sigma2, "theta": w.theta, "alpha": w.alpha, "rtol": w.rtol,
                   "solver": w.solver, "precision": w.precision},
        "solves_per_s": solves * value,
        "unknown_solves_per_s": unknowns * value,
        "iters_state": max(s["iters_state"] for s in stats),
        "iters_adjoint": max(s["iters_adjoint"] for s in stats),
        "max_relres": max(s["max_relres"] for s in stats),
        "roofline": roofline(tm, kind, nfin, w.precision),
    }
    out["rates"] = level_rates(w, stats)
    out["other_kernels"] = other_kernel_rooflines(args, m, w, dev, nfin)
    if not args.no_mixed:
        wm = inputs.WORKLOADS[args.mixed_workload]
        log(args, f"mixed workload {args.mixed_workload} ({wm.precision})")
        rm = run(args, m, wm, dev, args.steps, args.warmup, timing_n=wm.grid_n[-1])
        vm = args.steps / rm["dt"]
        tmm, kind_m = dominant_timing(args, m, wm, dev, rm["timing"], wm.grid_n[-1])
        rf_m = roofline(tmm, kind_m, wm.grid_n[-1], wm.precision)
        sm, um = problem_counts(wm.grid_n, wm.M)
        err = same_samples_error(m, wm, wm, dev)
        # the FP64 path on the mixed workload's data (sigma^2 = 2, theta = 10):
        # the like-for-like comparison for the mixed speed-up
        wf = dataclasses.replace(wm, precision="fp64",
                                 name=wm.name.replace("FP32 V-cycles in FP64 refinement",
                                                      "FP64 MG-PCG"))
        log(args, "FP64 on the mixed workload's data")
        rf = run(args, m, wf, dev, args.steps, args.warmup)
        vf = args.steps / rf["dt"]
        out["fp64_on_mixed_data"] = {
            "workload": wf.name, "value": vf, "unit": "gradient estimates/s",
            "ms_per_step": 1e3 * rf["dt"] / args.steps,
            "iters_state": max(s["iters_state"] for s in rf["stats"]),
            "iters_adjoint": max(s["iters_adjoint"] for s in rf["stats"]),
        }
        acc_grads["fp64_on_mixed_data"] = (wf, first_estimate(m, wf, dev))
        acc_grads["mixed"] = (wm, first_estimate(m, wm, dev))
        out["mixed"] = {
            "workload": wm.name,
            "value": vm,
            "unit": "gradient estimates/s",
            "ms_per_step": 1e3 * rm["dt"] / args.steps,
            "solves_per_s": sm * vm,
            "unknown_solves_per_s": um * vm,
            "iters_state": max(s["iters_state"] for s in rm["stats"]),
            "iters_adjoint": max(s["iters_adjoint"] for s in rm["stats"]),
            "grad_rel_err_vs_fp64_gpu_same_samples": err,
            "smoothing_pass": rf_m,
            "speedup_vs_fp64_batched_same_data": vm / vf,
        }
        wb = inputs.WORKLOADS["mlmc_129_bf16"]
        log(args, "bfloat16-smoother workload")
        rb = run(args, m, wb, dev, args.steps, args.warmup)
        vb = args.steps / rb["dt"]
        out["mixed_bf16"] = {
            "workload": wb.name, "value": vb, "unit": "gradient estimates/s",
            "ms_per_step": 1e3 * rb["dt"] / args.steps,
            "iters_state": max(s["iters_state"] for s in rb["stats"]),
            "iters_adjoint": max(s["iters_adjoint"] for s in rb["stats"]),
            "grad_rel_err_vs_fp64_gpu_same_samples": same_samples_error(m, wb, wb, dev),
            "speedup_vs_fp64_batched_same_data": vb / vf,
        }
        acc_grads["mixed_bf16"] = (wb, first_estimate(m, wb, dev))
    if not args.no_extra:
        log(args, "single-level SGD workload")
        out["single_level_sgd"] = single_level_sgd(m, dev)
        wb257 = inputs.WORKLOADS["mlmc_257_batched"]
        log(args, "batched 9^3..257^3 workload")
        r257 = run(args, m, wb257, dev, max(2, args.steps // 2), 1)
        s257, u257 = problem_counts(wb257.grid_n, wb257.M)
        v257 = max(2, args.steps // 2) / r257["dt"]
        out["batched_257"] = {"workload": wb257.name, "value": v257, "unit": "gradient estimates/s",
                              "ms_per_step": 1e3 / v257, "solves_per_s": s257 * v257,
                              "unknown_solves_per_s": u257 * v257,
                              "iters_state": max(x["iters_state"] for x in r257["stats"]),
                              "iters_adjoint": max(x["iters_adjoint"] for x in r257["stats"])}
        log(args, "batched 9^3..257^3 workload, one replayed HIP graph per estimate")
        k257 = max(2, args.steps // 2)
        g257 = run(args, m, wb257, dev, k257, 1, graph=True)
        vg = k257 / g257["dt"]
        out["batched_257"]["graph"] = {
            "value": vg, "ms_per_step": 1e3 / vg, "solves_per_s": s257 * vg}
        log(args, "adaptive MLSGD, 9^3..257^3, 50 steps")
        out["adaptive_257"] = adaptive_leg(args, m, dev)
        log(args, "autograd objective, 65^3, 256 samples")
        out["autograd_65"] = autograd_leg(m, dev)
        log(args, "odd-size solve batch")
        out["odd_size_solves"] = odd_size_solves(m, dev)
        wp = inputs.WORKLOADS["paper_law_65"]
        log(args, "Sec. 5 law workload")
        kp = max(2, args.steps)
        # at the initial control u = 0 every state solve is trivial; time the
        # estimate at a control away from it so both solves iterate
        up0 = inputs.control_xyz(wp.grid_n[-1]) + 3.0 * wp.y_d()
        rp = run(args, m, wp, dev, kp, 1, u0=up0)
        sp, up = problem_counts(wp.grid_n, wp.M)
        vp = kp / rp["dt"]
        out["paper_law"] = {"workload": wp.name + ", control 0.1xyz + 3 y_d",
                            "value": vp, "unit": "gradient estimates/s",
                            "ms_per_step": 1e3 / vp, "solves_per_s": sp * vp,
                            "iters_state": max(x["iters_state"] for x in rp["stats"]),
                            "iters_adjoint": max(x["iters_adjoint"] for x in rp["stats"])}
    if not args.no_per_sample:
        log(args, "per-sample FP64 comparator")
        ps = per_sample_fp64(m, inputs.WORKLOADS[args.mixed_workload], dev)
        out["fp64_per_sample"] = ps
        if "mixed" in out:
            out["mixed"]["speedup_vs_fp64_per_sample"] = out["mixed"]["value"] / ps["value"]
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or host_threads()
        log(args, f"cpu baseline with {threads} threads")
        cb, errs = cpu_baseline(w, threads, acc_grads)
        out["cpu_baseline"] = cb
        out["grad_rel_err_vs_oracle"] = errs
        for key in ("mixed", "mixed_bf16", "fp64_on_mixed_data"):
            if key in out and key in errs:
                out[key]["grad_rel_err_vs_oracle"] = errs[key]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
