"""autograd.Function of the MLMC objective: backward (adjoint kernels, fields
re-drawn from their seeds) against central finite differences of the forward
and against the FP64 oracle gradient."""
import numpy as np
import pytest

from paper_2606_09291_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_09291_amd as m
    m.lib()
    return m


def _setup(mm, grid, **kw):
    import torch
    nL = grid[-1]
    yd = inputs.target_sin(nL)
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, **kw))
    u = torch.as_tensor(inputs.control_xyz(nL) + 20.0 * yd, device="cuda:0").contiguous()
    return ctx, u, yd


@pytest.mark.parametrize("grid,M,n_dirs,rtol", [([65], [256], 20, 1e-12),
                                                ([9, 17, 33], [32, 8, 4], 8, 1e-13)])
def test_backward_matches_central_differences(mm, grid, M, n_dirs, rtol):
    """Central differences, eps = 1e-5, against <dJ/du, d> from backward, in
    random smooth directions (sine-mode combinations).  The quotient carries
    the noise of the two objectives, |dJ_noise| / eps: each J is exact only
    to about rtol |J| in the solves and to its FP64 rounding floor (about
    1e-14 |J| on these sums), which relative to a small directional
    derivative (one of the three-level directions has |dJ| = 2.4e-3 |J|)
    reaches the order of the 1e-6 bar at eps = 1e-6.  At eps = 1e-5 that
    noise is ten times smaller, while the central quotient's truncation error
    (order eps^2) stays far below the bar: every direction agrees to about
    1e-8 or better.  The three-level case is solved to 1e-13 (its finest
    grid's FP64 residual floor is near 2e-14).  White-noise directions have a
    directional derivative ~sqrt(N) smaller still and would sit at the noise
    floor."""
    import torch
    from paper_2606_09291_amd.autograd import objective
    print("autograd FD", grid, M, rtol, flush=True)
    ctx, u, _ = _setup(mm, grid, theta=1.0, alpha=1e-3, rtol=rtol)
    first = [3] * len(grid)
    uu = u.clone().requires_grad_(True)
    J = objective(uu, ctx, M, first)
    J.backward()
    gE = uu.grad.detach()
    eps = 1e-5
    worst = 0.0
    for d in inputs.random_smooth_directions(grid[-1], n_dirs, 77):
        dt = torch.as_tensor(d, device="cuda:0")
        Jp, _ = ctx.mlmc_objective(u + eps * dt, M, first)
        Jm, _ = ctx.mlmc_objective(u - eps * dt, M, first)
        fd = (Jp - Jm) / (2 * eps)
        an = float(torch.sum(gE * dt))
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-30))
    print("worst relative FD mismatch", worst, flush=True)
    assert worst < 1e-6
    ctx.close()


def test_backward_matches_oracle_gradient(mm, orc):
    """The Euclidean autograd gradient equals h^3 times the oracle's L^2_h
    gradient (sampled single-level 65^3, 256 samples; bar 1e-9)."""
    from paper_2606_09291_amd.autograd import objective
    grid, M = [65], [256]
    print("autograd vs oracle", flush=True)
    ctx, u, yd = _setup(mm, grid, theta=1.0, alpha=1e-3, rtol=1e-12)
    uu = u.clone().requires_grad_(True)
    J = objective(uu, ctx, M, [0])
    J.backward()
    h = 1.0 / 64
    pb = orc.make_problem(grid, theta=1.0, alpha=1e-3, rtol=1e-13)
    go, so = orc.mlmc_gradient(pb, None, u.cpu().numpy(), yd, M, first=[0])
    g = uu.grad.detach().cpu().numpy() / h ** 3
    assert float(np.linalg.norm(g - go) / np.linalg.norm(go)) <= 1e-9
    assert J.item() == pytest.approx(so["J"], rel=1e-10)
    ctx.close()
