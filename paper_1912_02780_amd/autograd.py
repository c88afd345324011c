"""torch.autograd layer over the HIP forward / backward (argument marshalling only).

``HOTRGFunction.apply(T0, chi, n_steps, options)`` returns ln Z / N as a 0-d float64 tensor on T0's
device; its backward runs the library's hand-written reverse pass (the SRG environment recursion,
extended through the truncated eigensolve) seeded with the incoming gradient, so that any torch
computation that builds T0 (for the Ising model, ``inputs.ising_T0_torch(beta)``) is differentiated
through it by autograd.  The forward's plan (one checkpoint per RG step) is kept until the graph is
released, so a retained graph can be differentiated again.
"""

from __future__ import annotations

import torch

from . import binding as B
from . import inputs as I


class HOTRGFunction(torch.autograd.Function):
    """lnZ/N = HOTRGFunction.apply(T0, chi, n_steps, options).

    T0: [l][u][r][d] CUDA tensor (float64, or cast to it).  options: a ``binding.Options`` or None.
    """

    @staticmethod
    def forward(ctx, T0, chi: int, n_steps: int, options=None):
        if not T0.is_cuda:
            raise TypeError("T0 must be a CUDA tensor")
        t = T0.detach().to(torch.float64).contiguous()
        plan, lnZ = B.dtrg_hotrg_forward(t, int(chi), int(n_steps), options)
        ctx.plan = plan
        ctx.in_dtype = T0.dtype
        return torch.tensor(lnZ, dtype=torch.float64, device=T0.device)

    @staticmethod
    def backward(ctx, g):
        if not ctx.needs_input_grad[0]:
            return None, None, None, None
        T0bar, _ = B.dtrg_hotrg_backward(ctx.plan, float(g.item()))
        return T0bar.to(ctx.in_dtype), None, None, None


def lnZ_per_site(T0: torch.Tensor, chi: int, n_steps: int, options=None) -> torch.Tensor:
    """ln Z / N of the periodic 2^n_steps-site network of T0 (differentiable in T0)."""
    return HOTRGFunction.apply(T0, chi, n_steps, options)


def ising_lnZ_and_energy(beta: float, chi: int, n_steps: int, options=None, device="cuda:0"):
    """Square-lattice Ising model (J = 1, h = 0): (ln Z / N, internal energy per site
    u = -d(ln Z / N)/d beta), with beta entering through the torch-built site tensor and u taken by
    autograd through the library's backward."""
    b = torch.tensor(float(beta), dtype=torch.float64, device=device, requires_grad=True)
    L = lnZ_per_site(I.ising_T0_torch(b), chi, n_steps, options)
    (dL,) = torch.autograd.grad(L, b)
    return float(L.item()), -float(dL.item())


def ising_specific_heat(beta: float, chi: int, n_steps: int, h: float = 1e-4, options=None, device="cuda:0"):
    """Specific heat per site c = beta^2 d^2(ln Z / N)/d beta^2 = -beta^2 du/dbeta, as the central
    difference (step h) of the exact reverse-mode energy at beta +- h, with the Richardson
    combination of steps h and h/2 (error O(h^4))."""
    def du(step):
        return (ising_lnZ_and_energy(beta + step, chi, n_steps, options, device)[1]
                - ising_lnZ_and_energy(beta - step, chi, n_steps, options, device)[1]) / (2.0 * step)
    d1, d2 = du(h), du(h / 2.0)
    return -beta * beta * (4.0 * d2 - d1) / 3.0
