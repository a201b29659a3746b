"""Restarts after the true-residual check (stopping rule C-13: the true
residual at exit decides; a solve that misses rtol starts again from
b - A x).  Restarts are rare with the default margins, so the test hook
MLSGD_FORCE_RESTART restarts every even-numbered problem after its first
check.  The restart path then runs on half of the problems: the residual
written into their right-hand-side rows, their fresh start, and the second
check of those alone while the others keep their first verdict.  A
restarted problem was already within rtol, so its result moves by at most
the solver tolerance: the estimate equals the unforced one to 1e-10 and the
oracle to 1e-9 (FP64) or 1e-8 (FP32 V-cycles), every solve converges, and
the iteration count grows (the restart ran).  Graph mode replays its
captured restart block the same way."""
import numpy as np
import pytest

from paper_2606_09291_amd import inputs

pytestmark = pytest.mark.gpu

GRID, M = [9, 17, 33], [32, 8, 4]
KW = dict(theta=1.0, alpha=1e-3, sigma2=2.0)


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


@pytest.mark.parametrize("precision,graph", [("fp64", False), ("mixed", False), ("fp64", True)])
def test_forced_restarts_keep_the_estimate(mm, orc, monkeypatch, precision, graph):
    import torch
    print("forced restarts", precision, "graph" if graph else "host-driven", flush=True)
    yd = inputs.target_sin(33)
    u = torch.as_tensor(inputs.control_xyz(33) + 10.0 * yd, device="cuda:0")
    prec = mm.FP64 if precision == "fp64" else mm.MIXED_FP32
    out = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("MLSGD_FORCE_RESTART", flag)
        ctx = mm.Context(mm.Problem(grid_n=GRID, y_d=yd, rtol=1e-12, precision=prec, **KW),
                         use_tuned=False)
        if graph:
            ctx.set_graph(True)
        calls = []
        for r in range(3 if graph else 1):   # graph: the first call captures, two replays
            g, st = ctx.mlmc_gradient(u, M, first=[0] * len(M))
            calls.append((g.cpu().numpy(), st))
        ctx.close()
        for g, st in calls:
            assert st["nonconverged"] == 0 and st["max_relres"] <= 1e-12
        out[flag] = calls
    g0, st0 = out["0"][-1]
    for g1, st1 in out["1"]:
        d = _rel(g1, g0)
        print("forced vs unforced: relative L2", d, "iterations", st0["iters_state"],
              st1["iters_state"], st0["iters_adjoint"], st1["iters_adjoint"], flush=True)
        assert d <= 1e-10
        assert st1["iters_state"] > st0["iters_state"]
        assert st1["iters_adjoint"] > st0["iters_adjoint"]
        assert st1["J"] == pytest.approx(st0["J"], rel=1e-12)
    pb = orc.make_problem(GRID, rtol=1e-13, **KW)
    go, _ = orc.mlmc_gradient(pb, None, u.cpu().numpy(), yd, M, first=[0] * len(M))
    assert _rel(out["1"][-1][0], go) <= (1e-9 if precision == "fp64" else 1e-8)


def test_quiet_iterations_leave_results_unchanged(mm):
    """After its first solve a context runs the first iterations of later
    solves without reading the active count from the host.  Problems that
    converge there are skipped as always, so the estimate of the same draws
    is bit-identical to a fresh context's, and so are the iteration counts."""
    import torch
    print("quiet iterations", flush=True)
    yd = inputs.target_sin(33)
    u = torch.as_tensor(inputs.control_xyz(33) + 10.0 * yd, device="cuda:0")
    mk = lambda: mm.Context(mm.Problem(grid_n=GRID, y_d=yd, rtol=1e-12, **KW), use_tuned=False)
    warm = mk()
    warm.mlmc_gradient(u, M, first=[5] * len(M))     # learns the iteration count
    g_w, st_w = warm.mlmc_gradient(u, M, first=[0] * len(M))
    warm.close()
    fresh = mk()
    g_f, st_f = fresh.mlmc_gradient(u, M, first=[0] * len(M))
    fresh.close()
    assert np.array_equal(g_w.cpu().numpy(), g_f.cpu().numpy())
    assert st_w["iters_state"] == st_f["iters_state"]
    assert st_w["iters_adjoint"] == st_f["iters_adjoint"]
    assert st_w["J"] == st_f["J"]
