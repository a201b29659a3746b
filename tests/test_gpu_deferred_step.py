"""The Krylov step of the iterate deferred into the next matvec
(MLSGD_XDEFER, the default) against the step taken in the update pass.

Both modes form the same x + alpha p from the same operands, one pass later,
and every other quantity (r, p, the scalars) is computed by the same code, so
the results must be bit-identical: gradients, objectives, iteration counts
and residuals.  Covered: MG-PCG in FP64 (dense and padded rows) and with
FP32 V-cycles, plain CG, graph replays, and an iteration cap that ends the
loop with every problem's last step still pending (only the flush before the
residual check applies it)."""
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


CASES = [
    ("fp64 9..33", [9, 17, 33], [16, 8, 4], dict()),
    ("fp64 17..129 padded", [17, 33, 65, 129], [4, 2, 2, 1], dict()),
    ("mixed 17..65", [17, 33, 65], [8, 4, 3], dict(precision="mixed")),
    ("cg 17", [17], [24], dict(solver="cg")),
    ("graph 9..33", [9, 17, 33], [16, 8, 4], dict(graph=True)),
    ("capped at 3 iterations", [9, 17, 33], [16, 8, 4], dict(max_iters=3)),
]


def _estimate(mm, grid, M, opts):
    import torch
    nL = grid[-1]
    yd = inputs.target_sin(nL)
    kw = dict(theta=2.0, alpha=1e-3, sigma2=2.0, rtol=1e-12)
    if opts.get("precision") == "mixed":
        kw["precision"] = mm.MIXED_FP32
    if opts.get("solver") == "cg":
        kw["solver"] = mm.SOLVER_CG
    if "max_iters" in opts:
        kw["max_iters"] = opts["max_iters"]
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, **kw), use_tuned=False)
    if opts.get("graph"):
        ctx.set_graph(True)
    u = torch.as_tensor(inputs.control_xyz(nL) + 10.0 * yd, device="cuda:0").contiguous()
    out = []
    capped = "max_iters" in opts
    for r in range(3 if opts.get("graph") else 1):  # graph: capture, then two replays
        first = [r * m for m in M]
        g, st = ctx.mlmc_gradient(u, M, first=first, allow_noconv=capped)
        torch.cuda.synchronize()
        out.append((g.cpu().numpy().copy(), st))
    ctx.close()
    return out


@pytest.mark.parametrize("name,grid,M,opts", CASES, ids=[c[0] for c in CASES])
def test_deferred_step_is_bit_identical(mm, monkeypatch, name, grid, M, opts):
    print("deferred step", name, flush=True)
    res = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("MLSGD_XDEFER", flag)
        res[flag] = _estimate(mm, grid, M, opts)
    for (g0, s0), (g1, s1) in zip(res["0"], res["1"]):
        assert np.array_equal(g0, g1)
        for key in ("J", "s", "iters_state", "iters_adjoint", "max_relres", "nonconverged"):
            assert s0[key] == s1[key], key
        if "max_iters" in opts:
            # the cap ends the loop with steps pending: had the flush missed
            # one, the deferred run's iterate and residual would differ
            assert s1["iters_state"] == opts["max_iters"] and s1["nonconverged"] > 0
        else:
            assert s1["nonconverged"] == 0
