"""Graph mode (mlsgd_set_graph): the first call of a batch shape runs on the
host-driven path and captures the shape; every later call replays the
captured graph.  Each replay is checked against the host-driven estimate of
the same draws on a second context, with that context's own launches and
synchronisations between the replays, and with fresh sample offsets on every
call so the per-call uploads are exercised.
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


def _pair(mm, grid, **kw):
    nL = grid[-1]
    mk = lambda: mm.Context(mm.Problem(grid_n=grid, y_d=inputs.target_sin(nL), **kw))
    eager, graph = mk(), mk()
    graph.set_graph(True)
    return eager, graph


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_match_host_driven(mm, precision):
    import torch
    grid, M = [9, 17, 33], [64, 16, 4]
    print("graph replays", precision, flush=True)
    prec = mm.FP64 if precision == "fp64" else mm.MIXED_FP32
    eager, graph = _pair(mm, grid, precision=prec, sigma2=2.0, theta=5.0, rtol=1e-12)
    u = torch.as_tensor(inputs.control_xyz(33) + 5.0 * inputs.target_sin(33), device="cuda:0")
    for r in range(5):   # call 0 captures, calls 1..4 replay
        first = [r * m for m in M]
        g_e, st_e = eager.mlmc_gradient(u, M, first=first)
        torch.cuda.synchronize()
        g_g, st_g = graph.mlmc_gradient(u, M, first=first)
        torch.cuda.synchronize()
        assert st_g["nonconverged"] == 0 and st_g["max_relres"] <= 1e-12
        assert _rel(g_g.cpu().numpy(), g_e.cpu().numpy()) <= 1e-13, r
        assert st_g["J"] == pytest.approx(st_e["J"], rel=1e-13)
        for i in range(len(M)):
            assert st_g["m2_dX"][i] == pytest.approx(st_e["m2_dX"][i], rel=1e-12)
    eager.close()
    graph.close()


def test_graph_objective_and_gradient_shapes(mm):
    """Objective-only and gradient calls are separate shapes; both replay."""
    import torch
    grid, M = [9, 17], [32, 8]
    eager, graph = _pair(mm, grid, rtol=1e-12)
    u = torch.as_tensor(inputs.control_xyz(17), device="cuda:0")
    for r in range(3):
        first = [100 + r * m for m in M]
        J_e, _ = eager.mlmc_objective(u, M, first=first)
        J_g, _ = graph.mlmc_objective(u, M, first=first)
        g_e, _ = eager.mlmc_gradient(u, M, first=first)
        g_g, _ = graph.mlmc_gradient(u, M, first=first)
        torch.cuda.synchronize()
        assert J_g == pytest.approx(J_e, rel=1e-13)
        assert _rel(g_g.cpu().numpy(), g_e.cpu().numpy()) <= 1e-13
    eager.close()
    graph.close()


def test_graph_sgd_trajectory(mm):
    """Three projected SGD steps with running offsets: the graph-mode
    trajectory equals the host-driven one."""
    import torch
    grid, M = [9, 17, 33], [32, 8, 2]
    eager, graph = _pair(mm, grid, rtol=1e-12)
    ue = torch.as_tensor(inputs.control_xyz(33), device="cuda:0").contiguous()
    ug = ue.clone()
    eager.set_batch(M)
    graph.set_batch(M)
    for k in range(3):
        se = eager.step(ue, 10.0)
        sg = graph.step(ug, 10.0)
        torch.cuda.synchronize()
        assert _rel(ug.cpu().numpy(), ue.cpu().numpy()) <= 1e-13, k
        assert sg["grad"]["J"] == pytest.approx(se["grad"]["J"], rel=1e-13)
    eager.close()
    graph.close()
