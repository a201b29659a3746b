"""Pins of the oracle's adaptive controller (Sec. 4.1) against what the
formulas are designed to achieve, not against a retyped formula."""
import math

import numpy as np
import pytest

from oracle import controller as ctl


def test_optimal_batch_hits_target_and_minimises_cost():
    """Unrounded M_l meets sum V_l / M_l = eps^2/2 exactly, and any other batch
    meeting the same sampling error costs more (Lagrange optimum)."""
    rng = np.random.default_rng(0)
    for _ in range(20):
        L = rng.integers(2, 6)
        M = [int(x) for x in rng.integers(4, 200, size=L)]
        v2 = list(rng.uniform(0.1, 10.0, size=L))
        C = list(rng.uniform(1.0, 1e5, size=L))
        eps = rng.uniform(1e-3, 1.0)
        raw = ctl.optimal_batch(v2, M, C, eps, ceil=False)
        V = [v / (m - 1) for v, m in zip(v2, M)]
        assert sum(Vi / Mi for Vi, Mi in zip(V, raw)) == pytest.approx(eps ** 2 / 2, rel=1e-12)
        cost = sum(Mi * Ci for Mi, Ci in zip(raw, C))
        for _ in range(10):
            w = rng.uniform(0.5, 2.0, size=L)
            alt = [r * wi for r, wi in zip(raw, w)]
            s = sum(Vi / Mi for Vi, Mi in zip(V, alt)) / (eps ** 2 / 2)
            alt = [a * s for a in alt]   # rescale to the same sampling error
            assert sum(Mi * Ci for Mi, Ci in zip(alt, C)) >= cost * (1 - 1e-12)


def test_rounded_batch_meets_target():
    v2, M, C, eps = [4.0, 1.0, 0.25], [100, 50, 20], [1.0, 8.0, 64.0], 0.05
    Mo = ctl.optimal_batch(v2, M, C, eps)
    V = [v / (m - 1) for v, m in zip(v2, M)]
    assert sum(Vi / Mi for Vi, Mi in zip(V, Mo)) <= eps ** 2 / 2
    assert all(m >= 2 for m in Mo)


def test_rate_fit_and_bias_on_geometric_decay():
    """Level corrections e_l = c 2^{-a l}: alpha_hat = a exactly, and the bias
    estimate equals the remaining geometric tail bound of the finest level,
    e_{L-1}^2 / (2^a - 1)^2."""
    for a in (1.0, 1.5, 2.0, 3.0):
        L = 5
        e = [3.0 * 2.0 ** (-a * i) for i in range(L)]
        assert ctl.fit_rate(e) == pytest.approx(a, rel=1e-12)
        e2 = [x * x for x in e]
        b = ctl.bias_estimate(e2, a, L)
        assert b == pytest.approx(e2[-1] / (2 ** a - 1) ** 2, rel=1e-12)
    assert ctl.fit_rate([1.0, 0.0, 0.0]) == 2.0


def test_sampling_error_and_level_growth():
    stats = {"s": 0.1, "EY_shifted": 1.0, "norm2_EX": 0.5,
             "m2_dX": [3.0, 1.0, 0.2], "m2_dY": [0.3, 0.1, 0.02],
             "norm2_mean_dX": [1.0, 0.1, 0.05], "mean_dY": [1.0, 0.01, 0.005]}
    out = ctl.control(stats, [20, 10, 5], [9, 17, 33, 65], theta=0.0, grad_norm=0.01,
                      n_levels_max=4)
    v2 = out["v2"]
    assert out["err_sam"] == pytest.approx(sum(v / (m * (m - 1)) for v, m in zip(v2, [20, 10, 5])))
    # weak decay 0.05 -> bias far above eps^2/2 = 4e-5: one more level
    assert out["L"] == 4 and len(out["M_next"]) == 4
    out2 = ctl.control(stats, [20, 10, 5], [9, 17, 33], theta=0.0, grad_norm=0.01,
                       n_levels_max=3)
    assert out2["L"] == 3


def test_adaptive_step_is_exact_line_search_on_quadratics():
    """J(u) = 1/2 u^T H u - b^T u with exact gradients (err_sam = 0): along an
    eigenvector of H the estimate Lhat is the eigenvalue, so the step is 1/lam
    and lands on the minimiser in that direction; scaling J by c scales the
    step by 1/c; a gradient below the sampling error gives no step."""
    rng = np.random.default_rng(3)
    lam = rng.uniform(0.5, 20.0, size=6)
    H = np.diag(lam)
    b = rng.standard_normal(6)
    ustar = b / lam
    for j in range(6):
        e = np.zeros(6)
        e[j] = 1.0
        u0 = ustar + 3.0 * e
        g0 = H @ u0 - b
        tau0 = 0.05
        u1 = u0 - tau0 * g0
        g1 = H @ u1 - b
        tau1 = ctl.adaptive_step(np.linalg.norm(g1), 0.0, np.linalg.norm(g1 - g0), tau0,
                                 np.linalg.norm(g0))
        assert tau1 == pytest.approx(1.0 / lam[j], rel=1e-12)
        u2 = u1 - tau1 * g1
        assert np.linalg.norm(H @ u2 - b) <= 1e-12 * np.linalg.norm(g0)
        for c in (0.1, 7.0):
            gc0 = c * g0
            gc1 = c * (H @ (u0 - tau0 * gc0) - b)
            t = ctl.adaptive_step(np.linalg.norm(gc1), 0.0, np.linalg.norm(gc1 - gc0), tau0,
                                  np.linalg.norm(gc0))
            assert t == pytest.approx(1.0 / (c * lam[j]), rel=1e-12)
    assert ctl.adaptive_step(1.0, 2.0, 0.5, 0.1, 1.0) == 0.0


def test_batch_cap_bounds_every_level_including_an_added_one():
    """A vanishing eps asks for unbounded batches; each level, and the level
    the bias adds, stays within the samples whose 14 solver arrays of n^3
    doubles fit 32 GiB (257^3: 18 samples; 9^3: 420 827)."""
    assert ctl.batch_cap(257) == 18 and ctl.batch_cap(9) == 420827
    assert ctl.batch_cap(1025) == 2
    stats = {"s": 0.0, "EY_shifted": 1.0, "norm2_EX": 1.0,
             "m2_dX": [3.0, 1.0, 0.5], "m2_dY": [0.0, 0.0, 0.0],
             "norm2_mean_dX": [1.0, 0.5, 0.4], "mean_dY": [1.0, 0.0, 0.0]}
    grid = [65, 129, 257, 513]
    out = ctl.control(stats, [4, 4, 4], grid, theta=0.0, grad_norm=1e-9, n_levels_max=4)
    assert out["L"] == 4
    assert out["M_next"] == [ctl.batch_cap(n) for n in grid]


def test_costs_enter_only_through_their_ratios():
    """The optimal batch depends on the level costs only through their ratios
    (a common unit, seconds or unknowns x iterations, cancels), and the
    default costs are the interior-unknown counts."""
    stats = {"s": 0.1, "EY_shifted": 1.0, "norm2_EX": 0.5,
             "m2_dX": [3.0, 1.0, 0.2], "m2_dY": [0.3, 0.1, 0.02],
             "norm2_mean_dX": [1.0, 0.1, 0.05], "mean_dY": [1.0, 0.01, 0.005]}
    grid, M = [9, 17, 33], [40, 20, 10]
    base = ctl.control(stats, M, grid, theta=0.5, grad_norm=0.02)
    same = ctl.control(stats, M, grid, theta=0.5, grad_norm=0.02, costs=ctl.level_costs(grid))
    scaled = ctl.control(stats, M, grid, theta=0.5, grad_norm=0.02,
                         costs=[17.0 * c for c in ctl.level_costs(grid)])
    assert base["M_next"] == same["M_next"] == scaled["M_next"]
    # a level made twice as expensive gets fewer samples, by sqrt(2) before rounding
    C = ctl.level_costs(grid)
    C2 = [C[0], 2.0 * C[1], C[2]]
    v2, _, _ = ctl.power_sums(stats, 0.5, 3)
    r1 = ctl.optimal_batch(v2, M, C, 0.018, ceil=False)
    r2 = ctl.optimal_batch(v2, M, C2, 0.018, ceil=False)
    tot1 = sum(math.sqrt(v / max(m - 1, 1) * c) for v, m, c in zip(v2, M, C))
    tot2 = sum(math.sqrt(v / max(m - 1, 1) * c) for v, m, c in zip(v2, M, C2))
    assert r2[1] / r1[1] == pytest.approx(tot2 / tot1 / math.sqrt(2.0), rel=1e-12)
