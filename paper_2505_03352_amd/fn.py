"""Differentiation: the chain C -> kappa -> FDTD -> alpha as a
torch.autograd.Function with a hand-written adjoint.

forward(C) sets the design, runs every forward and adjoint right-hand side
(the adjoint sources are unit-amplitude, so one run serves any objective),
and returns the modal coefficients alpha [n_src, n_ports, n_freq].
backward(g) receives torch's gradient for a complex output,
g = 2 dL/d conj(alpha), so the holomorphic-side coefficient the library
expects is coef = dL/dalpha = conj(g)/2; the library returns
sum 2 Re(coef dalpha/dC) = dL/dC.

Nothing is checkpointed: the time-harmonic adjoint needs no time history,
only the steady-state phasors in the design box, which stay resident in the
plan's workspace between forward and backward (about 3 MB per right-hand
side for the 100x100 design).  A plan under pulse excitation works the same
way: its runs accumulate every wavelength's phasors as they go.  A plan serves one live graph at a time; a
second forward on the same plan before backward is detected and rejected.
"""
from __future__ import annotations

import torch

from ._abi import YO_BOTH


class YeeAdjointFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, C: torch.Tensor, plan, beta: float, chunk: int = 100, use_graph: bool = True):
        plan.set_design(C.detach(), beta)
        plan.run(YO_BOTH, chunk=chunk, use_graph=use_graph)
        plan._run_id = getattr(plan, "_run_id", 0) + 1
        ctx.plan = plan
        ctx.run_id = plan._run_id
        return plan.alpha()

    @staticmethod
    def backward(ctx, g_alpha: torch.Tensor):
        plan = ctx.plan
        if getattr(plan, "_run_id", None) != ctx.run_id:
            raise RuntimeError("the plan was run again after this forward; its phasors are gone "
                               "(use one plan per live autograd graph)")
        coef = torch.conj(g_alpha) * 0.5
        gC = plan.gradient(coef.to(torch.complex64).contiguous())
        return gC, None, None, None, None


def modal_coefficients(C: torch.Tensor, plan, beta: float, chunk: int = 100,
                       use_graph: bool = True) -> torch.Tensor:
    """alpha(C), differentiable with respect to C."""
    return YeeAdjointFn.apply(C, plan, beta, chunk, use_graph)


def transmission_objective(alpha: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """sum_k (T_k - |alpha_k|^2)^2 (paper Eq. (9))."""
    return torch.sum((target - alpha.abs() ** 2) ** 2)
