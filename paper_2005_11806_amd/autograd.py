"""torch.autograd wrapper of one Method-I pressure step (Sec. 3.3.1,
Eq. poisson_me1): forward is psv_solve, backward is the library's hand-written
adjoint psv_solve_adjoint. Both run on the caller's current stream.

With rho0=None the splitting uses rho0 = min(rho); the adjoint then routes the
rho0 derivative to the (first) cell that holds the minimum, a subgradient of
min(). A float rho0 is a constant; a 0-dim tensor rho0 receives its gradient
(this synchronises to read it back).
"""
from __future__ import annotations

import torch


class PressureSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, rho, p_prev, plan, rho0=None):
        if p_prev is None:
            p_prev = torch.zeros_like(f)
        r0 = None if rho0 is None else float(rho0)
        p = plan.solve(f, rho=rho, p_prev=p_prev, rho0=r0)
        ctx.plan = plan
        ctx.rho0 = r0
        ctx.rho0_tensor = isinstance(rho0, torch.Tensor)
        ctx.save_for_backward(f, rho, p_prev)
        return p

    @staticmethod
    def backward(ctx, w):
        f, rho, p_prev = ctx.saved_tensors
        need = ctx.needs_input_grad
        want_r0 = ctx.rho0_tensor and len(need) > 4 and need[4]
        g = ctx.plan.adjoint(w.contiguous(), f=f, rho=rho, p_prev=p_prev, rho0=ctx.rho0,
                             grad_f=need[0], grad_rho=need[1], grad_p_prev=need[2],
                             grad_rho0=want_r0)
        g_r0 = torch.tensor(g["rho0"], dtype=torch.float64) if want_r0 else None
        return g["f"], g["rho"], g["p_prev"], None, g_r0


def pressure_solve(f, rho, p_prev, plan, rho0=None):
    """Differentiable Method-I step: p = S(rho0 f + D((1 - rho0/rho_f) G p_prev))."""
    return PressureSolve.apply(f, rho, p_prev, plan, rho0)
