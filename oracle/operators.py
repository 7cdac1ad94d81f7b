"""Oracle (test infrastructure): second-order MAC difference operators and the
Method-I right-hand side.

Face storage convention (all arrays C-order, x fastest):
  Fx[k, j, i]  on the x face between cells i and i+1 (periodic), [nz, ny, nx]
  Fy[k, j, i]  on the y face between cells j and j+1 (periodic), [nz, ny, nx]
  Fz[k, j, i]  on the z face at zf[k], k = 0..nz, [nz+1, ny, nx]; faces 0 and
               nz are the walls, where the pressure flux is zero (homogeneous
               Neumann, the "homogeneous" boundary conditions that Sec. 3.3.1
               requires for the eigenexpansion).

Spatial terms are second-order central differences (Sec. 3.2); the discrete
Laplacian is L = D G, the 7-point operator (flux form on a stretched z grid).
"""
from __future__ import annotations

import numpy as np


def grad(p, grid):
    """G p on faces; zero on the two z walls."""
    gx = (np.roll(p, -1, axis=2) - p) / grid.dx
    gy = (np.roll(p, -1, axis=1) - p) / grid.dy
    gz = np.zeros((grid.nz + 1, grid.ny, grid.nx))
    gz[1:grid.nz] = (p[1:] - p[:-1]) / grid.g[1:grid.nz, None, None]
    return gx, gy, gz


def div(fx, fy, fz, grid):
    """D F at cell centres: sum over directions of (F_plus - F_minus)/width."""
    out = (fx - np.roll(fx, 1, axis=2)) / grid.dx
    out = out + (fy - np.roll(fy, 1, axis=1)) / grid.dy
    out = out + (fz[1:] - fz[:-1]) / grid.h[:, None, None]
    return out


def divergence_of_faces(ux, uy, uz, grid):
    """Discrete divergence of a face field (used to build the test RHS)."""
    return div(ux, uy, uz, grid)


def laplacian(p, grid):
    """7-point L p = D(G p)."""
    return div(*grad(p, grid), grid)


def face_density(rho, grid):
    """Density on faces: arithmetic mean of the two adjacent cells.

    The paper stores all scalars at cell centres (Sec. 3) and does not say how
    rho is carried to the faces where 1/rho multiplies the pressure gradient;
    the arithmetic mean is the reading taken here. Wall faces carry nan (they
    never multiply a nonzero flux)."""
    rx = 0.5 * (rho + np.roll(rho, -1, axis=2))
    ry = 0.5 * (rho + np.roll(rho, -1, axis=1))
    rz = np.full((grid.nz + 1, grid.ny, grid.nx), np.nan)
    rz[1:grid.nz] = 0.5 * (rho[:-1] + rho[1:])
    return rx, ry, rz


def assemble_method1(f, rho, p_prev, rho0, grid):
    """Right-hand side of Method I (Sec. 3.3.1, Eq. poisson_me1):

        r = D[(1 - rho0/rho_face) G p_prev] + rho0 f,

    where f is the user's right-hand side of Eq. lap_p, i.e. it already holds
    (div u* - div u^{n+1}) / dt.
    """
    rx, ry, rz = face_density(rho, grid)
    gx, gy, gz = grad(p_prev, grid)
    bz = np.zeros_like(gz)
    bz[1:grid.nz] = (1.0 - rho0 / rz[1:grid.nz]) * gz[1:grid.nz]
    return div((1.0 - rho0 / rx) * gx, (1.0 - rho0 / ry) * gy, bz, grid) + rho0 * f


def var_coeff_operator(p, rho, grid):
    """D(rho_face^-1 G p): the left-hand side of Eq. lap_p."""
    rx, ry, rz = face_density(rho, grid)
    gx, gy, gz = grad(p, grid)
    fz = np.zeros_like(gz)
    fz[1:grid.nz] = gz[1:grid.nz] / rz[1:grid.nz]
    return div(gx / rx, gy / ry, fz, grid)


def mixture_density(phi, rho_gas, rho_liq):
    """One-fluid density, Sec. 2.2 Eq. eq_22 with the colour Phi = 1 in gas:
    rho = rho_g Phi + rho_l (1 - Phi)."""
    return rho_gas * phi + rho_liq * (1.0 - phi)
