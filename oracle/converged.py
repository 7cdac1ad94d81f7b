"""Oracle (test infrastructure): the converged variable-density pressure
solve and its implicit adjoint.

The fixed point that Methods I and III iterate towards (Sec. 3.3.1; Method
III reaches it exactly, Eq. new_poisson) is the solution of Eq. lap_p,

    A(rho) p = D(rho_f^-1 G p) = f_c,   f_c = f - mean_V(f),   sum_V p = 0,

with rho_f the arithmetic mean of the two cells of a face. Both iterations
are, in pressure form, p <- p + S[omega (f_c - A p)] with S the projected,
gauged constant-coefficient solve and omega = rho0 = min rho (Method I,
Eq. poisson_me1), omega = the harmonic mean of the two phase densities
(Method II, Eq. poisson_laizet; read as those of min rho and max rho) or
omega = rho (cell density, Method III).

A is symmetric in the volume-weighted inner product (V A is symmetric), so
for a loss sum(w p) the gradients are obtained from one more solve with the
same operator instead of differentiating the iterations:

    lambda   = A^+ (V^-1 w)      (zero volume-weighted mean)
    grad_f   = mu = V lambda
    grad_rho = sum over the faces F of each cell of
               (D^T mu)_F (G p)_F / (2 rho_F^2),

where (D^T mu)_F = mu_L/h_L - mu_R/h_R across F (widths normal to F), and
the 1/2 is the derivative of rho_F by either of its two cells.

``solve_dense`` is the definition, a bordered LU solve of the loop-assembled
matrix (tiny grids); ``solve`` iterates in pressure form with the exact
eigenexpansion solve of ``oracle.solve`` (any size the oracle can take).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import dense
from .adjoint import div_transpose
from .operators import face_density, grad, var_coeff_operator
from .solve import solve_const


def _vmean(x, grid):
    v = grid.volume_field()
    return float((v * x).sum() / v.sum())


def solve_dense(f, rho, grid):
    """p with A(rho) p = f - mean_V(f) and zero volume-weighted mean."""
    A = dense.inv_density_matrix(grid, rho)
    p, _ = dense.bordered_solve(A, f, dense.volume_vector(grid))
    return p.reshape(grid.shape)


@dataclass
class Converged:
    p: np.ndarray
    eps: list          # sum |f_c - A p| of every iterate, the first for p_init
    converged: bool


def solve(f, rho, grid, eps_t, max_iter, iteration="method3", p_init=None):
    """Iterate p <- p + S[omega (f_c - A p)] until sum |f_c - A p| <= eps_t or
    max_iter solves; omega = rho (Method III), min rho (Method I) or the
    harmonic mean of min rho and max rho (Method II)."""
    fc = f - _vmean(f, grid)
    if iteration == "method3":
        omega = rho
    elif iteration == "method2":
        a, b = float(np.min(rho)), float(np.max(rho))
        omega = 2.0 * a * b / (a + b)
    else:
        omega = float(np.min(rho))
    p = np.zeros(grid.shape) if p_init is None else np.array(p_init, dtype=np.float64)
    eps = []
    for _ in range(max_iter + 1):
        q = fc - var_coeff_operator(p, rho, grid)
        eps.append(float(np.abs(q).sum()))
        if eps[-1] <= eps_t or len(eps) > max_iter:
            break
        dp, _ = solve_const(omega * q, grid)
        p = p + dp
    return Converged(p, eps, eps[-1] <= eps_t)


def density_gradient(mu, p, rho, grid):
    """grad_rho of sum(w p) given mu = V lambda and the converged p."""
    tx, ty, tz = div_transpose(mu, grid)
    gx, gy, gz = grad(p, grid)
    rx, ry, rz = face_density(rho, grid)
    fx = tx * gx / (2.0 * rx * rx)
    fy = ty * gy / (2.0 * ry * ry)
    fz = np.zeros_like(tz)
    fz[1:grid.nz] = tz[1:grid.nz] * gz[1:grid.nz] / (2.0 * rz[1:grid.nz] ** 2)
    # every face feeds both of its cells
    g = fx + np.roll(fx, 1, axis=2) + fy + np.roll(fy, 1, axis=1)
    return g + fz[1:] + fz[:-1]


def adjoint_dense(w, f, rho, grid):
    """(grad_f, grad_rho) of sum(w p), p = solve_dense(f, rho), by dense solves."""
    vol = grid.volume_field()
    p = solve_dense(f, rho, grid)
    mu = vol * solve_dense(w / vol, rho, grid)
    return mu, density_gradient(mu, p, rho, grid)


def adjoint(w, p, rho, grid, eps_t, max_iter, iteration="method3"):
    """(grad_f, grad_rho, adjoint solve record) of sum(w p) at the converged p,
    with lambda from the iterative solve."""
    vol = grid.volume_field()
    lam = solve(w / vol, rho, grid, eps_t, max_iter, iteration)
    mu = vol * lam.p
    return mu, density_gradient(mu, p, rho, grid), lam
