"""Device memory of the plan cache.  A context keeps one layout (plan) per
batch shape; beyond eight plans the least recently used one is freed, so a
caller that meets ever new shapes (the adaptive batch controller) keeps a
bounded footprint, and re-tuning frees every plan.  Memory is read with
hipMemGetInfo through torch (device-wide free bytes)."""
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


def _free():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_plan_cache_is_bounded_and_retuning_frees_it(mm):
    import torch
    grid = [9, 17, 33, 65]
    yd = inputs.target_sin(65)
    ctx = mm.Context(mm.Problem(grid_n=grid, y_d=yd, rtol=1e-10), use_tuned=False)
    u = torch.as_tensor(inputs.control_xyz(65), device="cuda:0").contiguous()
    ctx.mlmc_gradient(u, [8, 4, 2, 2])          # context buffers, torch's output cache
    ctx.set_tuning(**ctx.get_tuning())          # drop that plan
    base = _free()
    shapes = [[64, 16, 8, 2 + k] for k in range(20)]   # a new batch shape per call
    for M in shapes:
        ctx.mlmc_gradient(u, M)
    used = base - _free()
    ctx.set_tuning(**ctx.get_tuning())
    freed = _free()
    print("plans in use", used, "after retuning", base - freed, flush=True)
    assert base - freed <= 64 << 20               # every plan freed again
    ctx.mlmc_gradient(u, shapes[-1])
    last = base - _free()                         # one plan of the largest shape
    # the eight most recent shapes at most (sizes grow with the shape: the 20
    # plans together would be about 11 times the last one)
    assert used <= 8.5 * last
    ctx.close()
