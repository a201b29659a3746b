"""MLSGD outer loop (Algorithm 1, function MLSGD): projected SGD steps through
mlsgd_step with the adaptive batch controller (Sec. 4.1) and the adaptive step
size (Sec. 5), until the norm of the latest gradient estimate is at most
eps_tilde, the step limit is reached, or the wall-clock budget is spent (the
paper fixes eps_tilde through a time budget)."""
import time


def run(ctx, u, M0, tau, max_steps, eps_tilde=0.0, budget_s=None, adapt_batch=True,
        adapt_step=True, offsets=None, callback=None):
    """u: contiguous float64 device tensor on the finest grid, updated in place.
    M0: initial per-level batch; tau: step (with adapt_step: the first step and
    the fallback).  Returns {"steps", "stop", "seconds", "history"} with stop in
    {"eps", "budget", "steps"}."""
    ctx.set_batch(M0, offsets)
    hist = []
    stop = "steps"
    t0 = time.perf_counter()
    for k in range(max_steps):
        st = ctx.step(u, tau, adapt=adapt_batch, adapt_step=adapt_step)
        g = st["grad"]
        rec = {"step": k, "J": g["J"], "grad_norm": g["grad_norm"], "tau": st["tau"],
               "M": st["M_next"], "err_sam": st["err_sam"], "err_num": st["err_num"],
               "eps": st["eps"], "iters": [g["iters_state"], g["iters_adjoint"]]}
        hist.append(rec)
        if callback:
            callback(rec)
        if g["grad_norm"] <= eps_tilde:
            stop = "eps"
            break
        if budget_s is not None and time.perf_counter() - t0 >= budget_s:
            stop = "budget"
            break
    return {"steps": len(hist), "stop": stop, "seconds": time.perf_counter() - t0,
            "history": hist}
