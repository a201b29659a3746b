"""torch.autograd wrapper of the MLMC entropic objective.

``objective(u, ctx, M, first)`` returns the MLMC estimate of
J(u) = theta^-1 log max{1, E^ML[e^{theta Phi}]} + alpha/2 |u|_h^2 (Sec. 2.1,
Sec. 2.2) as a 0-d tensor.  Its backward pass is the library's adjoint path:
the fields are drawn again from their (seed, level, sample) keys, the state
and adjoint problems are solved by the batched kernels, and the L^2_h
gradient is turned into the Euclidean gradient of the vertex array
(h^3 times the Riesz representer on interior vertices, 0 on the boundary).
Nothing but u and the sampling bookkeeping is saved between the passes.
"""
import torch

from . import Context


class EntropicObjective(torch.autograd.Function):
    @staticmethod
    def forward(fctx, u, mctx: Context, M, first):
        J, _ = mctx.mlmc_objective(u, M, first)
        fctx.save_for_backward(u)
        fctx.mctx = mctx
        fctx.M = list(M)
        fctx.first = list(first) if first is not None else None
        return torch.tensor(J, dtype=torch.float64, device=u.device)

    @staticmethod
    def backward(fctx, grad_out):
        (u,) = fctx.saved_tensors
        mctx = fctx.mctx
        g, _ = mctx.mlmc_gradient(u, fctx.M, fctx.first)
        h = 1.0 / (mctx.nfin - 1)
        return grad_out * (h ** 3) * g.reshape(u.shape), None, None, None


def objective(u, mctx: Context, M, first=None):
    """J(u) with autograd support (u: float64 device tensor on the finest grid)."""
    return EntropicObjective.apply(u, mctx, M, first)
