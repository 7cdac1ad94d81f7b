"""torch.autograd wrappers.

PressureSolve: one Method-I pressure step (Sec. 3.3.1, Eq. poisson_me1);
forward is psv_solve, backward is the library's hand-written adjoint
psv_solve_adjoint. Both run on the caller's current stream.

ConvergedSolve: the converged variable-density solve (the fixed point of
Methods I and III, Eq. lap_p); forward is psv_solve_converged, backward the
implicit adjoint psv_solve_converged_adjoint (one more converged solve).

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


class ConvergedSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, rho, plan, iteration, eps_t, max_iter, adj_eps_t):
        p, info = plan.solve_converged(f, rho, iteration=iteration, eps_t=eps_t,
                                       max_iter=max_iter)
        if not info.converged:
            raise RuntimeError(f"converged solve stopped at eps {info.eps:.3e} > {eps_t:.3e}")
        ctx.plan, ctx.iteration, ctx.max_iter = plan, iteration, max_iter
        ctx.adj_eps_t = adj_eps_t
        ctx.save_for_backward(rho, p)
        return p

    @staticmethod
    def backward(ctx, w):
        rho, p = ctx.saved_tensors
        need = ctx.needs_input_grad
        gf, gr, info = ctx.plan.converged_adjoint(
            w.contiguous(), rho, p, iteration=ctx.iteration, eps_t=ctx.adj_eps_t,
            max_iter=ctx.max_iter, grad_f=need[0], grad_rho=need[1])
        if not info.converged:
            raise RuntimeError(f"adjoint solve stopped at eps {info.eps:.3e} > {ctx.adj_eps_t:.3e}")
        return gf, gr, None, None, None, None, None


def converged_solve(f, rho, plan, iteration="method3", eps_t=1e-10, max_iter=200, adj_eps_t=None):
    """Differentiable converged solve of D(rho_f^-1 G p) = f - mean_V(f). eps_t
    bounds the summed absolute residual of the forward solve and adj_eps_t
    (default eps_t) that of the adjoint solve, whose right-hand side is
    V^-1 w. Raises if either loop stops before reaching its threshold."""
    return ConvergedSolve.apply(f, rho, plan, iteration, eps_t, max_iter,
                                eps_t if adj_eps_t is None else adj_eps_t)
