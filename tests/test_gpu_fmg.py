"""Full-multigrid start of the Krylov solves (MLSGD_FMG=1): b restricted to
every grid, the exact 3^3 solve, then one Chebyshev cycle on each larger grid
from the prolonged solution below; PCG starts from the result.

Only the starting iterate changes, so every solve still meets rtol and the
estimate matches the FP64 oracle to the usual bars (1e-9 FP64, 1e-8 FP32
cycles).  It agrees with the zero-start estimate on the same draws to the
solver tolerance, and no solve takes more iterations than from zero (the
smooth right-hand sides here make the start worth one or two).  Covered: FP64
on dense and padded rows, FP32 and bfloat16-coefficient cycles, and graph
replays."""
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


KW = dict(theta=2.0, alpha=1e-3, sigma2=2.0)
CASES = [
    ("fp64 9..33", [9, 17, 33], [16, 8, 4], "fp64", False),
    ("fp64 17..129 padded", [17, 33, 65, 129], [4, 2, 2, 1], "fp64", False),
    ("mixed 9..65", [9, 17, 33, 65], [16, 8, 4, 2], "mixed", False),
    ("bf16 9..33", [9, 17, 33], [16, 8, 4], "bf16", False),
    ("graph fp64 9..33", [9, 17, 33], [16, 8, 4], "fp64", True),
]


def _estimates(mm, grid, M, precision, graph):
    import torch
    nL = grid[-1]
    yd = inputs.target_sin(nL)
    prec = {"fp64": mm.FP64, "mixed": mm.MIXED_FP32, "bf16": mm.MIXED_BF16}[precision]
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, rtol=1e-12, precision=prec, **KW),
                     use_tuned=False)
    if graph:
        ctx.set_graph(True)
    u = torch.as_tensor(inputs.control_xyz(nL) + 10.0 * yd, device="cuda:0").contiguous()
    out = []
    for r in range(3 if graph else 1):  # graph: capture, then two replays
        first = [r * m for m in M]
        g, st = ctx.mlmc_gradient(u, M, first=first)
        torch.cuda.synchronize()
        out.append((g.cpu().numpy().copy(), st, first))
    ctx.close()
    return out


@pytest.mark.parametrize("name,grid,M,precision,graph", CASES, ids=[c[0] for c in CASES])
def test_fmg_start_matches_oracle(mm, orc, monkeypatch, name, grid, M, precision, graph):
    print("fmg start", name, flush=True)
    res = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("MLSGD_FMG", flag)
        res[flag] = _estimates(mm, grid, M, precision, graph)
    bar = 1e-9 if precision == "fp64" else 1e-8
    pb = orc.make_problem(grid, rtol=1e-14, **KW)
    nL = grid[-1]
    yd = inputs.target_sin(nL)
    u = inputs.control_xyz(nL) + 10.0 * yd
    for (g0, s0, first), (g1, s1, _) in zip(res["0"], res["1"]):
        print("  iterations zero start", s0["iters_state"], s0["iters_adjoint"], "fmg start",
              s1["iters_state"], s1["iters_adjoint"], "difference", _rel(g1, g0), flush=True)
        assert s1["nonconverged"] == 0 and s1["max_relres"] <= 1e-12
        assert s1["iters_state"] <= s0["iters_state"]
        assert s1["iters_adjoint"] <= s0["iters_adjoint"]
        assert _rel(g1, g0) <= 1e-10
        assert s1["J"] == pytest.approx(s0["J"], rel=1e-12)
    go, so = orc.mlmc_gradient(pb, None, u, yd, M, first=res["1"][0][2])
    assert _rel(res["1"][0][0], go) <= bar
    assert res["1"][0][1]["J"] == pytest.approx(so["J"], rel=1e-10)
