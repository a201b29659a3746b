"""The exact coarsest-grid solve of the odd-size hierarchies: the inverse of
the rediscretised operator, computed on the GPU by a blocked Cholesky
factorisation on the FP64 matrix cores (mlsgd_dense_coarse_inverse), against
LAPACK's inverse of the oracle's assembled matrix for the same KL draws.

Bar: relative Frobenius error <= 1e-12 (the operators have condition numbers
of a few hundred at these sizes), and A A^-1 = I to 1e-12.  Sizes cover one
to 22 tiles of 16 unknowns, with and without padding of the last tile
(N = 8, 64, 125, 216, 343).
"""
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


@pytest.mark.parametrize("n,count,sigma2", [(4, 5, 1.0), (6, 3, 2.0), (7, 2, 1.0), (8, 4, 2.0),
                                            (9, 2, 1.0)])
def test_dense_coarse_inverse_matches_lapack(mm, orc, n, count, sigma2):
    print(f"dense inverse n={n} count={count}", flush=True)
    ctx = mm.Context(mm.Problem(grid_n=[9, 17], y_d=inputs.target_sin(17), K=4, sigma2=sigma2,
                                seed=3))
    inv = ctx.dense_coarse_inverse(n, 6, 11, count).cpu().numpy()
    ctx.close()
    N = (n - 2) ** 3
    for j in range(count):
        c = orc.kl_coeffs(3, 6, 11 + j, 4, sigma2)
        A = orc.assemble_dense(n, c)
        ref = np.linalg.inv(A)
        err = np.linalg.norm(inv[j] - ref) / np.linalg.norm(ref)
        assert err <= 1e-12, (j, err)
        assert np.linalg.norm(A @ inv[j] - np.eye(N)) <= 1e-12 * np.sqrt(N)
        assert np.array_equal(inv[j], inv[j].T) or np.max(np.abs(inv[j] - inv[j].T)) <= 1e-15 * np.max(np.abs(ref))


def test_dense_coarse_inverse_rejects_bad_arguments(mm):
    import torch
    ctx = mm.Context(mm.Problem(grid_n=[9, 17], y_d=inputs.target_sin(17)))
    out = torch.empty((1,), dtype=torch.float64, device="cuda:0")
    for n, count in [(3, 1), (10, 1), (6, 0)]:
        rc = ctx.lib.mlsgd_dense_coarse_inverse(ctx._h, n, 6, 0, count, out.data_ptr())
        assert rc == mm.MLSGD_EINVAL
    ctx.close()
