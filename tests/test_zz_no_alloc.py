"""The allocation-free solve entry point (mlsgd_solve_state_adjoint_noalloc)
against the allocating one (mlsgd_solve_state_adjoint) through the C ABI.

Both run the same kernels; the allocation-free one carves its buffers from
the library's fixed 64 MiB device array.  Bar: FP64 solves within 1e-10
relative L2 of each other (they are expected to agree bit for bit), misfits
within 1e-12, equal iteration counts.  Two calls in a row, the second with
a smaller batch, check that no call depends on what the previous one left in
the shared array.
"""
import numpy as np
import pytest

from paper_2606_09291_amd import inputs

pytestmark = pytest.mark.gpu

LIMIT = 64 << 20


@pytest.fixture(scope="module")
def mm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_09291_amd as m
    m.lib()
    return m


def _rel(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _run_pair(mm, ctx, u, level, coarse, first, count):
    import torch
    n = ctx.problem.grid_n[level - coarse]
    print(f"noalloc: grid {n}^3, level {level}, coarse {coarse}, first {first}, count {count}",
          flush=True)
    y_ref, p_ref, phi_ref, st_ref = ctx.solve_state_adjoint(level, coarse, first, count, u)
    y = torch.full((count, n, n, n), float("nan"), dtype=torch.float64, device=ctx.device)
    p = torch.full_like(y, float("nan"))
    phi = torch.full((count,), float("nan"), dtype=torch.float64, device=ctx.device)
    st, need = ctx.solve_state_adjoint_noalloc(level, coarse, first, count, u, y, p, phi)
    torch.cuda.synchronize()
    assert 0 < need <= LIMIT
    assert st["nonconverged"] == 0 and st_ref["nonconverged"] == 0
    assert st["iterations"] == st_ref["iterations"]
    for j in range(count):
        assert _rel(y[j], y_ref[j]) <= 1e-10
        assert _rel(p[j], p_ref[j]) <= 1e-10
    assert _rel(phi, phi_ref) <= 1e-12
    return need


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_allocating_entry(mm, precision):
    """A 33^3 batch of 6 samples, then a smaller 17^3 coarse-partner batch of 3:
    each equals the allocating entry point's result."""
    grid = [9, 17, 33]
    yd = inputs.target_sin(33)
    u = inputs.control_xyz(33) + 20.0 * yd
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, precision=precision, theta=1.0,
                                rtol=1e-12), use_tuned=False)
    big = _run_pair(mm, ctx, u, 2, 0, 5, 6)
    small = _run_pair(mm, ctx, u, 2, 1, 1, 3)
    assert small < big
    ctx.close()


def test_noalloc_two_65_samples_then_one_17(mm):
    """The largest batch the array holds at 65^3 (two FP64 samples), then a
    single 17^3 sample; a batch that needs more than the array is refused
    before any kernel runs, and the context keeps working."""
    import torch
    grid = [17, 33, 65]
    yd = inputs.target_sin(65)
    u = inputs.control_xyz(65) + 20.0 * yd
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, theta=1.0, rtol=1e-12), use_tuned=False)
    _run_pair(mm, ctx, u, 2, 0, 0, 2)
    y = torch.empty((3, 65, 65, 65), dtype=torch.float64, device=ctx.device)
    with pytest.raises(mm.MlsgdError) as ei:
        ctx.solve_state_adjoint_noalloc(2, 0, 0, 3, u, y, None, None)
    assert ei.value.code == mm.MLSGD_EINVAL
    _run_pair(mm, ctx, u, 0, 0, 7, 1)
    ctx.close()
