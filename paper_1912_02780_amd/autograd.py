"""torch.autograd wrapper of the HIP forward / backward (argument marshalling only)."""

from __future__ import annotations

import torch

from . import binding as B


class HOTRGFunction(torch.autograd.Function):
    """lnZ/N = HOTRGFunction.apply(T0, chi, n_steps, options).

    T0 is a [l][u][r][d] float64 CUDA tensor.  The backward calls the library's hand-written
    reverse pass with the incoming scalar gradient.
    """

    @staticmethod
    def forward(ctx, T0, chi: int, n_steps: int, options=None):
        plan, lnZ = B.dtrg_hotrg_forward(T0.detach().contiguous(), chi, n_steps, options)
        ctx.plan = plan
        return torch.tensor(lnZ, dtype=torch.float64, device=T0.device)

    @staticmethod
    def backward(ctx, g):
        T0bar, _ = B.dtrg_hotrg_backward(ctx.plan, float(g.item()))
        return T0bar, None, None, None


def lnZ_per_site(T0: torch.Tensor, chi: int, n_steps: int, options=None) -> torch.Tensor:
    return HOTRGFunction.apply(T0, chi, n_steps, options)


def lnZ_and_grad(T0: torch.Tensor, chi: int, n_steps: int, dT0: torch.Tensor | None = None, options=None):
    """(lnZ/N, d(lnZ/N)/dT0, <d(lnZ/N)/dT0, dT0> or None, plan) in one forward and one backward."""
    plan, lnZ = B.dtrg_hotrg_forward(T0, chi, n_steps, options)
    T0bar, ddir = B.dtrg_hotrg_backward(plan, 1.0, dT0)
    return lnZ, T0bar, ddir, plan
