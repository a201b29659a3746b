"""Level-rate verification of the MLMC hierarchy (Sec. 3, the assumptions on
the strong error, weak error and cost of the level corrections, and Sec. 5's
rate figures), from the per-level statistics that every gradient estimate
returns.

For level l >= 1 with mesh width h_l:
  e_l = |E[dX_l]|_h          expected  e_l <~ C_X h_l^alpha
  V_l = Var[dX_l] (h-norm)   expected  V_l <~ C_V h_l^beta
  w_l = |E[dY_l]|            expected  w_l <~ C_Y h_l^alpha
  C_l = cost per sample      expected  C_l ~  h_l^-gamma
The exponents are least-squares slopes of log2 of the quantity against
log2(1/h_l) over the levels l >= 1 (level 0 is plain Monte Carlo and carries
no correction), and the constants are the fitted intercepts 2^b.
"""
import math

import numpy as np


def loglog_fit(h, q):
    """Slope and constant of q ~ C h^s by least squares in log2 (levels with
    q > 0 only).  Returns (s, C); (nan, nan) with fewer than two points."""
    pts = [(math.log2(hh), math.log2(qq)) for hh, qq in zip(h, q) if qq > 0 and hh > 0]
    if len(pts) < 2:
        return float("nan"), float("nan")
    x = np.array([p[0] for p in pts])
    y = np.array([p[1] for p in pts])
    s, b = np.polyfit(x, y, 1)
    return float(s), float(2.0 ** b)


def level_statistics(stats, M, theta):
    """Per-level e_l, V_l, w_l in unshifted units from one estimate's
    statistics (mlmc_gradient's; its sums carry the weights exp(theta (Phi -
    s)), so e and w scale back by exp(theta s), V by its square)."""
    sc = math.exp(theta * stats["s"])
    L = len(M)
    e = [math.sqrt(max(stats["norm2_mean_dX"][i], 0.0)) * sc for i in range(L)]
    V = [stats["m2_dX"][i] / max(M[i] - 1, 1) * sc * sc for i in range(L)]
    w = [abs(stats["mean_dY"][i]) * sc for i in range(L)]
    return e, V, w


def fit_rates(grid, e, V, w, cost):
    """alpha, beta, gamma and C_X, C_V, C_Y over the levels l >= 1 of a grid
    hierarchy (grid = vertices per axis)."""
    h = [1.0 / (n - 1) for n in grid]
    a, cx = loglog_fit(h[1:], e[1:])
    b, cv = loglog_fit(h[1:], V[1:])
    ay, cy = loglog_fit(h[1:], w[1:])
    g, cc = loglog_fit(h[1:], cost[1:])
    return {"alpha": a, "beta": b, "alpha_Y": ay, "gamma": -g,
            "C_X": cx, "C_V": cv, "C_Y": cy, "C_cost": cc}
