"""Adaptive batch-size and level controller of the MLSGD method (Sec. 4.1),
written from the paper's formulas.  TEST INFRASTRUCTURE ONLY.

Readings where the printed formulas are ambiguous (listed with the others in
the design notes): the inner sum of the optimal batch size uses the previous
iteration's statistics; the factor is 2/eps^2, which makes the sampling
error of the unrounded batch exactly eps^2/2 (the stated target); the cost
per sample is the measured work passed in (interior unknowns x Krylov
iterations of the level's solves), or the interior-unknown count of the
fine and coarse grid;
the bias estimate extrapolates each level's correction to the finest level
with the fitted rate; eps = 0.9 |g| of the gradient just computed; every
level's batch, an added level's included, is capped at the number of samples
whose solver arrays fit a 32 GiB share of device memory (batch_cap).
"""
import math

import numpy as np


def level_costs(grid):
    """Deterministic cost per sample: interior unknowns of fine + coarse grid."""
    C = []
    for i, n in enumerate(grid):
        c = (n - 2) ** 3
        if i > 0:
            c += (grid[i - 1] - 2) ** 3
        C.append(float(c))
    return C


def batch_cap(n):
    """Largest batch of one level on an n^3 grid: the samples whose solver
    arrays (14 arrays of n^3 doubles each) fit 32 GiB.  The paper bounds the
    samples computed at once by memory (M^max in eq:optimal-parallelization)
    without giving a number; at least 2."""
    return max(2, math.floor(32.0 * 2 ** 30 / (14.0 * 8.0 * n ** 3)))


def power_sums(stats, theta, L):
    """v^2_l = sum |dX - mean dX|^2 + C_hat sum |dY - mean dY|^2 (unshifted),
    C_hat = |E^ML X|^2 / E^ML[Y]^2."""
    sc = math.exp(theta * stats["s"])
    chat = stats["norm2_EX"] / stats["EY_shifted"] ** 2
    v2 = [(stats["m2_dX"][i] + chat * stats["m2_dY"][i]) * sc * sc for i in range(L)]
    return v2, chat, sc


def optimal_batch(v2, M, C, eps, ceil=True, caps=None):
    """M_l = (2/eps^2) sqrt(V_l / C_l) sum_l' sqrt(V_l' C_l'), V = v^2/(M-1),
    rounded up, at least 2 and at most caps[l] when caps are given."""
    V = [v / max(m - 1, 1) for v, m in zip(v2, M)]
    tot = sum(math.sqrt(v * c) for v, c in zip(V, C))
    with np.errstate(all="ignore"):
        raw = [(2.0 / eps ** 2) * math.sqrt(v / c) * tot if eps > 0 else math.inf
               for v, c in zip(V, C)]
    if not ceil:
        return raw
    out = []
    for i, r in enumerate(raw):
        cap = caps[i] if caps is not None else math.inf
        out.append(max(2, cap if not math.isfinite(r) or r > cap else int(math.ceil(r))))
    return out


def sampling_error(v2, M):
    """err^sam = sum_l v^2_l / (M_l (M_l - 1))."""
    return sum(v / (m * max(m - 1, 1)) for v, m in zip(v2, M))


def fit_rate(level_norms):
    """alpha_hat: minus the least-squares slope of log2(e_l) over the levels
    l >= 1 (inputs: e_0, e_1, ...); 2 when fewer than two usable points or a
    slope flatter than 1/2."""
    pts = [(i, math.log2(e)) for i, e in enumerate(level_norms) if i >= 1 and e > 0]
    if len(pts) < 2:
        return 2.0
    x = np.array([p[0] for p in pts], dtype=float)
    y = np.array([p[1] for p in pts], dtype=float)
    slope = np.polyfit(x, y, 1)[0]
    return -slope if -slope > 0.5 else 2.0


def bias_estimate(level_norms2, alpha_hat, L):
    """max over levels 1..L-1 of e_l^2 / (2^a - 1)^2 * (h_L/h_l)^(2a)."""
    d = (2.0 ** alpha_hat - 1.0) ** 2
    out = 0.0
    for i in range(1, L):
        out = max(out, level_norms2[i] / d * 2.0 ** (-2.0 * alpha_hat * (L - 1 - i)))
    return out


def control(stats, M, grid, theta, grad_norm, n_levels_max=None, costs=None):
    """One controller update from the statistics of the estimate just made.
    costs: the measured cost per sample of each level (the paper uses the
    previous iteration's measured average cost); the interior-unknown count
    of level_costs when not given."""
    L = len(M)
    v2, chat, sc = power_sums(stats, theta, L)
    eps = 0.9 * grad_norm
    C = list(costs[:L]) if costs is not None else level_costs(grid[:L])
    Mn = optimal_batch(v2, M, C, eps, caps=[batch_cap(n) for n in grid[:L]])
    e2 = [(stats["norm2_mean_dX"][i] + chat * stats["mean_dY"][i] ** 2) * sc * sc
          for i in range(L)]
    ahat = fit_rate([math.sqrt(e) for e in e2])
    err_num = bias_estimate(e2, ahat, L)
    Lnew = L
    if n_levels_max is not None and err_num > 0.5 * eps ** 2 and L < n_levels_max:
        Mn = Mn + [max(2, min(batch_cap(grid[L]), Mn[-1] // 4))]
        Lnew = L + 1
    return {"M_next": Mn, "L": Lnew, "err_sam": sampling_error(v2, M), "err_num": err_num,
            "eps": eps, "alpha_hat": ahat, "v2": v2}


def adaptive_step(g_norm, err_sam, diff_norm, tau_prev, g_prev_norm):
    """Adaptive step size of Sec. 5 (eq. adaptive-step-size):
    Lhat = |g_k - g_{k-1}| / (tau_{k-1} |g_{k-1}|),
    tau_k = (|g_k|^2 - err_sam_k) / (Lhat |g_k|^2), clamped at 0 from below."""
    Lhat = diff_norm / (tau_prev * g_prev_norm)
    return max(0.0, (g_norm ** 2 - err_sam) / (Lhat * g_norm ** 2))
