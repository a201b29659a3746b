"""Adaptive step size (mlsgd_step with ADAPT_STEP) and the MLSGD outer loop.

sigma = 0 pins the step exactly: every sample then gives the same field
(a = 1), the MLMC estimate is the exact finest-grid gradient, and along
u = c y_d (an eigenfunction of the 7-point Laplacian, eigenvalue lam1) the
objective is the quadratic with curvature H = 1/lam1^2 + alpha.  The adaptive
step after any first step is then 1/H, which lands on c* = lam1/(1 + alpha
lam1^2) (Newton step).  With random fields the library's step equals the
oracle formula on the oracle's gradients of the same draws.
"""
import math

import numpy as np
import pytest

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


def _lam1(n):
    h = 1.0 / (n - 1)
    return 12.0 / h ** 2 * math.sin(math.pi * h / 2) ** 2


def _hnorm(x, n):
    h = 1.0 / (n - 1)
    return math.sqrt(h ** 3 * float(np.sum(x[1:-1, 1:-1, 1:-1] ** 2)))


def test_adaptive_step_is_newton_step_at_sigma_zero(mm):
    import torch
    grid, M = [9, 17, 33], [4, 3, 2]
    nL, alpha = grid[-1], 1e-3
    yd = inputs.target_sin(nL)
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, sigma2=0.0, theta=3.0, alpha=alpha,
                                rtol=1e-13))
    lam = _lam1(nL)
    cstar = lam / (1.0 + alpha * lam * lam)
    u = torch.as_tensor(2.0 * cstar * yd, device="cuda:0").contiguous()
    ctx.set_batch(M)
    s1 = ctx.step(u, 0.5, adapt_step=True)
    assert s1["tau"] == 0.5
    s2 = ctx.step(u, 0.5, adapt_step=True)
    H = 1.0 / lam ** 2 + alpha
    assert s2["tau"] == pytest.approx(1.0 / H, rel=1e-8)
    assert _rel(u.cpu().numpy(), cstar * yd) <= 1e-8
    ctx.close()


def test_adaptive_step_matches_oracle_formula(mm, orc):
    import torch
    from oracle import controller as ctl
    grid, M = [9, 17, 33], [16, 8, 4]
    nL = grid[-1]
    yd = inputs.target_sin(nL)
    u0 = inputs.control_xyz(nL) + 10.0 * yd
    kw = dict(theta=2.0, alpha=1e-3, sigma2=2.0)
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, rtol=1e-12, **kw))
    u = torch.as_tensor(u0, device="cuda:0").contiguous()
    ctx.set_batch(M)
    tau0 = 0.5
    s1 = ctx.step(u, tau0, adapt=True, adapt_step=True)
    u1 = u.cpu().numpy().copy()
    M1 = s1["M_next"]
    s2 = ctx.step(u, tau0, adapt=True, adapt_step=True)
    pb = orc.make_problem(grid, rtol=1e-14, **kw)
    g0, _ = orc.mlmc_gradient(pb, None, u0, yd, M, first=[0, 0, 0])
    g1, so1 = orc.mlmc_gradient(pb, None, u1, yd, M1, first=list(M))
    n0, n1, d = _hnorm(g0, nL), _hnorm(g1, nL), _hnorm(g1 - g0, nL)
    assert s2["grad"]["grad_norm"] == pytest.approx(n1, rel=1e-8)
    err_sam = ctl.control(so1, M1, grid, theta=2.0, grad_norm=n1, n_levels_max=3)["err_sam"]
    tau1 = ctl.adaptive_step(n1, err_sam, d, tau0, n0)
    assert s2["tau"] == pytest.approx(tau1, rel=1e-6)
    assert _rel(u.cpu().numpy(), u1 - s2["tau"] * g1) <= 1e-8
    ctx.close()


def test_mlsgd_loop_stops(mm):
    import torch
    from paper_2606_09291_amd import mlsgd
    grid, M = [9, 17], [8, 4]
    yd = inputs.target_sin(17)
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, rtol=1e-12))
    u = torch.zeros((17, 17, 17), dtype=torch.float64, device="cuda:0")
    r = mlsgd.run(ctx, u, M, 1.0, 50, eps_tilde=1e9)
    assert r["stop"] == "eps" and r["steps"] == 1
    r = mlsgd.run(ctx, u, M, 1.0, 50, budget_s=0.0)
    assert r["stop"] == "budget" and r["steps"] == 1
    r = mlsgd.run(ctx, u, M, 1.0, 4, adapt_batch=True, adapt_step=True)
    assert r["stop"] == "steps" and r["steps"] == 4
    assert all(h["tau"] >= 0 for h in r["history"]) and r["history"][0]["tau"] == 1.0
    assert r["history"][-1]["J"] < r["history"][0]["J"]
    ctx.close()
