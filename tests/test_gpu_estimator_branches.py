"""Rarely taken branches of the estimator and the controller, HIP path (through
the C ABI) against the oracle on identical inputs.

- The truncation max{1, E^ML[Y]} of eq:gradient_estimator (Sec. 2.2) where it
  fires (E^ML[Y] < 0 here): gradient <= 1e-9 relative L2 (FP64) or 1e-8
  (mixed), objective, the flag and every per-level statistic of
  eq:sec-order-sum.
- The level update of eq:optimal-level (Sec. 4.1) adding a level on the
  library path: the library's next batch and level count equal the oracle
  controller's on the same statistics.
"""
import math

import numpy as np
import pytest

from estimator_cases import LEVEL_GROWTH_CASE, TRUNCATION_CASE
from paper_2606_09291_amd import inputs

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def mm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_09291_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("precision,bar", [(0, 1e-9), (1, 1e-8)])
def test_truncated_estimate_matches_oracle(mm, orc, precision, bar):
    tc = TRUNCATION_CASE
    grid, M, first = tc["grid"], tc["M"], tc["first"]
    nL = grid[-1]
    print(f"truncation case, precision {precision}", flush=True)
    yd = tc["yd_scale"] * inputs.target_sin(nL)
    u = tc["u_over_yd"] * yd
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, seed=tc["seed"], theta=tc["theta"],
                                alpha=tc["alpha"], precision=precision, rtol=1e-12))
    g, st = ctx.mlmc_gradient(u, M, first=first)
    J, sto = ctx.mlmc_objective(u, M, first=first)
    ctx.close()
    pb = orc.make_problem(grid, seed=tc["seed"], theta=tc["theta"], alpha=tc["alpha"],
                          rtol=1e-14)
    go, so = orc.mlmc_gradient(pb, None, u, yd, M, first=first)
    assert so["truncated"] == 1
    assert st["truncated"] == 1 and sto["truncated"] == 1
    assert st["EY_shifted"] < 0
    assert _rel(g.cpu().numpy(), go) <= bar
    assert st["J"] == pytest.approx(so["J"], rel=1e-10)
    assert J == pytest.approx(so["J"], rel=1e-10)
    assert st["s"] == pytest.approx(so["s"], rel=1e-10)
    assert st["EY_shifted"] == pytest.approx(so["EY_shifted"], rel=bar)
    assert st["norm2_EX"] == pytest.approx(so["norm2_EX"], rel=bar)
    for key in ("mean_dY", "norm2_mean_dX", "m2_dX", "m2_dY", "mean_phi_f"):
        for i in range(len(grid)):
            assert st[key][i] == pytest.approx(so[key][i], rel=bar, abs=1e-300), (key, i)


def test_library_controller_adds_a_level(mm, orc):
    """Two of three levels, bias above eps^2/2: mlsgd_step(adapt) returns a third
    level, and its batch sizes and level count equal the oracle controller's on
    the library's own statistics; the step's gradient matches the oracle's
    two-level estimate prolonged to the finest grid."""
    import torch
    from oracle import controller as ctl
    lc = LEVEL_GROWTH_CASE
    grid, M = lc["grid"], lc["M"]
    nL = grid[-1]
    yd = inputs.target_sin(nL)
    u0 = lc["u_over_yd"] * yd
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, theta=lc["theta"], alpha=lc["alpha"],
                                sigma2=lc["sigma2"], rtol=1e-12))
    u = torch.as_tensor(u0, device="cuda:0").contiguous()
    ctx.set_batch(M)
    st = ctx.step(u, 0.0, adapt=True)
    ctx.close()
    gs = st["grad"]
    out = ctl.control(gs, M, grid, theta=lc["theta"], grad_norm=gs["grad_norm"],
                      n_levels_max=len(grid), costs=gs["work_per_sample"])
    assert out["L"] == 3 and out["err_num"] > 0.5 * out["eps"] ** 2
    assert st["M_next"] == out["M_next"]
    assert st["err_num"] == pytest.approx(out["err_num"], rel=1e-12)
    assert st["err_sam"] == pytest.approx(out["err_sam"], rel=1e-12)
    assert st["eps"] == pytest.approx(out["eps"], rel=1e-12)
    # the two-level estimate itself against the oracle on grids 9, 17 with
    # the control restricted by full weighting, then prolonged
    u17 = orc.restrict(nL, u0)
    pb = orc.make_problem(grid[:2], theta=lc["theta"], alpha=lc["alpha"], sigma2=lc["sigma2"],
                          rtol=1e-14)
    g17, so = orc.mlmc_gradient(pb, None, u17, inputs.target_sin(17), M)
    ex17 = g17 - lc["alpha"] * u17
    gref = orc.prolong(17, ex17) + lc["alpha"] * u0
    gref[0] = gref[-1] = 0
    gref[:, 0] = gref[:, -1] = 0
    gref[:, :, 0] = gref[:, :, -1] = 0
    h = 1.0 / (nL - 1)
    gn = math.sqrt(h ** 3 * float(np.sum(gref[1:-1, 1:-1, 1:-1] ** 2)))
    assert gs["grad_norm"] == pytest.approx(gn, rel=1e-9)
    for i in range(2):
        assert gs["m2_dX"][i] == pytest.approx(so["m2_dX"][i], rel=1e-8)
        assert gs["norm2_mean_dX"][i] == pytest.approx(so["norm2_mean_dX"][i], rel=1e-8)
