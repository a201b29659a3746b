"""Host-side rate fits of the level hierarchy (rates.py) on exact power laws
and on a hand-built statistics record."""
import math

import pytest

from paper_2606_09291_amd import rates


def test_fit_recovers_exact_power_laws():
    grid = [9, 17, 33, 65, 129]
    h = [1.0 / (n - 1) for n in grid]
    for alpha, beta, gamma in [(2.0, 4.0, 3.0), (1.0, 2.0, 3.3), (1.5, 2.5, 2.0)]:
        e = [3.0 * x ** alpha for x in h]
        V = [0.5 * x ** beta for x in h]
        w = [7.0 * x ** alpha for x in h]
        C = [11.0 * x ** (-gamma) for x in h]
        r = rates.fit_rates(grid, e, V, w, C)
        assert r["alpha"] == pytest.approx(alpha, rel=1e-12)
        assert r["beta"] == pytest.approx(beta, rel=1e-12)
        assert r["alpha_Y"] == pytest.approx(alpha, rel=1e-12)
        assert r["gamma"] == pytest.approx(gamma, rel=1e-12)
        assert r["C_X"] == pytest.approx(3.0, rel=1e-10)
        assert r["C_V"] == pytest.approx(0.5, rel=1e-10)
        assert r["C_Y"] == pytest.approx(7.0, rel=1e-10)


def test_level_zero_is_excluded_and_nonpositive_skipped():
    grid = [9, 17, 33, 65]
    h = [1.0 / (n - 1) for n in grid]
    e = [1e6] + [x ** 2 for x in h[1:]]      # level 0 (plain MC) must not enter
    r = rates.fit_rates(grid, e, e, e, [1.0, 8.0, 64.0, 512.0])
    assert r["alpha"] == pytest.approx(2.0, rel=1e-12)
    assert r["gamma"] == pytest.approx(3.0, rel=1e-12)
    s, c = rates.loglog_fit([0.5], [1.0])
    assert math.isnan(s) and math.isnan(c)


def test_level_statistics_unshifts():
    """Sums are in units of exp(theta (Phi - s)): e and w scale by exp(theta s),
    the variance by exp(2 theta s), and M2 divides by M - 1."""
    st = {"s": 0.3, "norm2_mean_dX": [4.0, 1.0], "m2_dX": [9.0, 3.0], "mean_dY": [1.0, -0.25]}
    e, V, w = rates.level_statistics(st, [10, 4], theta=2.0)
    k = math.exp(0.6)
    assert e == pytest.approx([2.0 * k, 1.0 * k])
    assert V == pytest.approx([1.0 * k * k, 1.0 * k * k])
    assert w == pytest.approx([1.0 * k, 0.25 * k])
