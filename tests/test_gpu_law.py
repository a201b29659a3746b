"""The exponential KL law of Sec. 5 on the GPU against the oracle: draws
bit-exact, and gradient estimates of the paper-law workload (U(-4, 4) draws,
lam_jkl = exp(-pi (j+k+l) 0.15), permuted axes, 125 terms, target
prod sin(2 pi x_d), levels 17^3..65^3 with M = 128/16/2) at moderate and
strong risk aversion (theta = 1, 72).  Bars as for the algebraic law: 1e-9
(FP64) and 1e-8 (mixed) relative L2; both sides solve to rtol 1e-12, the
high-contrast field putting the FP64 residual floor near 1e-13."""
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


def test_exponential_law_draws_bit_exact(mm, orc):
    w = inputs.WORKLOADS["paper_law_65"]
    ctx = mm.Context(mm.Problem(grid_n=w.grid_n, y_d=w.y_d(), K=w.K, law=w.law, rho=w.rho))
    for level, first, count in [(0, 0, 4), (2, 77, 3)]:
        xi = ctx.sample_fields(level, first, count).cpu().numpy()
        for k in range(count):
            assert np.array_equal(xi[k], orc.draws(0, level, first + k, w.K, law=w.law))
    ctx.close()


@pytest.mark.parametrize("precision,theta", [("fp64", 1.0), ("fp64", 72.0), ("mixed", 72.0)])
def test_paper_law_estimate_matches_oracle(mm, orc, precision, theta):
    import torch
    w = inputs.WORKLOADS["paper_law_65"]
    print("paper law", precision, theta, flush=True)
    nL = w.grid_n[-1]
    yd = w.y_d()
    u0 = inputs.control_xyz(nL) + 3.0 * yd
    prec = mm.FP64 if precision == "fp64" else mm.MIXED_FP32
    ctx = mm.Context(mm.Problem(grid_n=w.grid_n, y_d=yd, K=w.K, law=w.law, rho=w.rho,
                                theta=theta, alpha=w.alpha, precision=prec, rtol=1e-12))
    g, st = ctx.mlmc_gradient(torch.as_tensor(u0, device="cuda:0"), w.M)
    assert st["nonconverged"] == 0
    pb = orc.make_problem(w.grid_n, K=w.K, theta=theta, alpha=w.alpha, rtol=1e-12,
                          law=w.law, rho=w.rho)
    go, so = orc.mlmc_gradient(pb, None, u0, yd, w.M)
    assert _rel(g.cpu().numpy(), go) <= (1e-9 if precision == "fp64" else 1e-8)
    assert st["J"] == pytest.approx(so["J"], rel=1e-10)
    assert st["s"] == pytest.approx(so["s"], rel=1e-10)
    ctx.close()
