"""Degenerate cases of the method on the GPU against the FP64 oracle.

- theta = 0: the entropic risk reduces to the mean misfit, every weight is 1,
  the shifted weight sum is exactly 1 and the gradient is the plain MLMC mean
  of the adjoints plus alpha u.
- The smallest hierarchies: a single 5^3 level (one V-cycle level above the
  3^3 grid, where one Jacobi step is the exact solve) and the pair 5^3, 9^3,
  each with one and with several samples per level.
- One sample on the finest level (the level variance then has no degrees of
  freedom and is reported as 0).
Bars: 1e-9 relative L2 for gradients, 1e-10 relative for objectives.
"""
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


def _run(mm, orc, grid, M, theta, first=None, **kw):
    nL = grid[-1]
    yd = inputs.target_sin(nL)
    u = inputs.control_xyz(nL) + 12.0 * yd
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, theta=theta, rtol=1e-12, **kw),
                     use_tuned=False)
    g, st = ctx.mlmc_gradient(u, M, first=first)
    ctx.close()
    pb = orc.make_problem(grid, theta=theta, rtol=1e-14, **kw)
    go, so = orc.mlmc_gradient(pb, None, u, yd, M, first=first)
    assert st["nonconverged"] == 0
    return g.cpu().numpy(), st, go, so


@pytest.mark.parametrize("grid,M", [([9, 17, 33], [16, 8, 4]), ([17], [24])])
def test_theta_zero_is_risk_neutral(mm, orc, grid, M):
    print("theta 0", grid, M, flush=True)
    g, st, go, so = _run(mm, orc, grid, M, 0.0, sigma2=2.0)
    assert _rel(g, go) <= 1e-9
    assert st["J"] == pytest.approx(so["J"], rel=1e-10)
    # every weight is exp(0) = 1: level 0 contributes M (1/M), the corrections 0
    assert st["EY_shifted"] == pytest.approx(1.0, rel=1e-15, abs=0.0)
    assert not st["truncated"]


@pytest.mark.parametrize("grid,M", [([5], [1]), ([5], [9]), ([5, 9], [6, 3]), ([5, 9], [1, 1])])
def test_smallest_hierarchies(mm, orc, grid, M):
    print("smallest", grid, M, flush=True)
    g, st, go, so = _run(mm, orc, grid, M, 2.0, sigma2=2.0)
    assert _rel(g, go) <= 1e-9
    assert st["J"] == pytest.approx(so["J"], rel=1e-10)


def test_one_sample_on_the_finest_level(mm, orc):
    print("one finest sample", flush=True)
    g, st, go, so = _run(mm, orc, [9, 17, 33], [12, 4, 1], 1.0, first=[3, 1, 7])
    assert _rel(g, go) <= 1e-9
    assert st["J"] == pytest.approx(so["J"], rel=1e-10)
    assert st["m2_dX"][2] == 0.0 and st["m2_dY"][2] == 0.0
