"""Oracle (test infrastructure): Method III and its iteration (Sec. 3.3.1,
Eq. new_poisson, Algorithm 1).

Method III recasts Eq. lap_p through the correction step (Eq. corr) as the
constant-coefficient equation

    lap p^{s+1} = (1/dt) [ D(rho u*) - rho div u^{n+1} - u^s . grad rho ],

solved together with the correction u^{s+1} = u* - dt rho^-1 grad p^{s+1},
starting from u^0 = u*, until the residual eps = sum over cells of
|div u^{s+1} - div u^{n+1}| falls to eps_t. The first two terms of the
right-hand side do not change over the loop and are formed once.

Readings where the paper is silent (also listed with the design notes):
* rho on faces is the arithmetic mean of the two cells, as for Method I;
* D(rho u) is the MAC divergence of the face flux rho_face u;
* u . grad rho at a cell centre is, per direction, the mean of the two face
  products u_f (rho_neighbour - rho_cell) / width, with the stretched-z
  weights g/h that make it the exact discrete product-rule remainder
  D(rho_face u) - rho D u; with it the recast is exact on the grid: at a fixed
  point div u = div u^{n+1} in every cell;
* the loop is the usual s = 0, 1, ... and stops after at most max_iter
  solves; eps_t is the paper's absolute threshold on the summed residual.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .operators import div, face_density, grad
from .solve import solve_const


@dataclasses.dataclass
class Method3Result:
    p: list            # iterates p^1, p^2, ... (one per solve)
    u: tuple           # (ux, uy, uz) of the last iterate
    eps: list          # residual after each solve
    converged: bool


def advection(ux, uy, uz, rho, grid):
    """u . grad rho at cell centres: per direction the two face products
    u_f (rho_nb - rho_c), weighted by (face gap)/(2 cell width) -- on uniform
    spacing the mean of the two face products u_f (rho_nb - rho_c)/width."""
    out = (ux * (np.roll(rho, -1, axis=2) - rho)
           + np.roll(ux, 1, axis=2) * (rho - np.roll(rho, 1, axis=2))) / (2.0 * grid.dx)
    out = out + (uy * (np.roll(rho, -1, axis=1) - rho)
                 + np.roll(uy, 1, axis=1) * (rho - np.roll(rho, 1, axis=1))) / (2.0 * grid.dy)
    # z: faces k (bottom of cell k) and k+1 (top); wall faces carry u_z = 0
    top = np.zeros(grid.shape)
    bot = np.zeros(grid.shape)
    top[:-1] = uz[1:grid.nz] * (rho[1:] - rho[:-1])
    bot[1:] = uz[1:grid.nz] * (rho[1:] - rho[:-1])
    return out + (top + bot) / (2.0 * grid.h[:, None, None])


def correct(ux, uy, uz, p, rho, dt, grid):
    """Correction step (Eq. corr): u = u* - dt rho_face^-1 G p on every face;
    the wall faces keep u* (zero normal velocity)."""
    rx, ry, rz = face_density(rho, grid)
    gx, gy, gz = grad(p, grid)
    vz = uz.copy()
    vz[1:grid.nz] = uz[1:grid.nz] - dt * gz[1:grid.nz] / rz[1:grid.nz]
    return ux - dt * gx / rx, uy - dt * gy / ry, vz


def fixed_rhs(ux, uy, uz, div_target, rho, dt, grid):
    """(1/dt) [D(rho_face u*) - rho div u^{n+1}], formed once before the loop."""
    rx, ry, rz = face_density(rho, grid)
    fz = np.zeros_like(uz)
    fz[1:grid.nz] = rz[1:grid.nz] * uz[1:grid.nz]
    return (div(rx * ux, ry * uy, fz, grid) - rho * div_target) / dt


def residual(ux, uy, uz, div_target, grid):
    """The loop's residual: sum over cells of |div u - div u^{n+1}|."""
    return float(np.abs(div(ux, uy, uz, grid) - div_target).sum())


def velocity(u_star, p, rho, dt, grid):
    """u(p) = u* - dt rho_face^-1 G p: the velocity a pressure p gives through
    the correction step (Eq. corr); u(0) = u*."""
    return correct(*u_star, p, rho, dt, grid)


def step_map(p, u_star, rhs0, rho, dt, grid):
    """T(p): the pressure that Eq. new_poisson gives when its advective term
    u . grad rho is taken at u(p), i.e. the constant-coefficient solve of
    rhs0 - u(p) . grad rho / dt."""
    u = velocity(u_star, p, rho, dt, grid)
    return solve_const(rhs0 - advection(*u, rho, grid) / dt, grid)[0]


def solve(u_star, div_target, rho, dt, grid, eps_t=1e-14, max_iter=50):
    """Method III as the fixed-point iteration p^{s+1} = T(p^s) of step_map,
    from p^0 = 0 (so u^0 = u*, as Algorithm 1 starts), stopped once the
    residual of u(p^{s+1}) is at most eps_t or after max_iter maps. u_star =
    (ux, uy, uz) on faces (uz with nz+1 planes, zero on the walls); returns
    the iterates, the velocity of the last one and the residuals."""
    rhs0 = fixed_rhs(*u_star, div_target, rho, dt, grid)
    p = np.zeros(grid.shape)
    ps, eps = [], []
    u = tuple(u_star)
    for _ in range(max_iter):
        p = step_map(p, u_star, rhs0, rho, dt, grid)
        u = velocity(u_star, p, rho, dt, grid)
        ps.append(p)
        eps.append(residual(*u, div_target, grid))
        if eps[-1] <= eps_t:
            return Method3Result(ps, u, eps, True)
    return Method3Result(ps, u, eps, False)
