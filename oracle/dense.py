"""Oracle (test infrastructure): dense matrices for tiny grids, assembled entry
by entry with explicit loops (independent of the vectorised stencils in
``operators``), and bordered LU solves of the singular Neumann problems.

Cell flat index: c = (k * ny + j) * nx + i.
"""
from __future__ import annotations

import numpy as np


def _idx(grid, k, j, i):
    return (k * grid.ny + (j % grid.ny)) * grid.nx + (i % grid.nx)


def var_coeff_matrix(grid, face_coeff_x, face_coeff_y, face_coeff_z):
    """Matrix of D(kappa G) with kappa given per face by callables
    face_coeff_x(k, j, i) for the face between (k,j,i) and (k,j,i+1), etc.;
    face_coeff_z(k, j, i) for the face between cells (k-1,j,i) and (k,j,i)."""
    n = grid.n
    A = np.zeros((n, n))
    for k in range(grid.nz):
        for j in range(grid.ny):
            for i in range(grid.nx):
                c = _idx(grid, k, j, i)
                # x faces: east (i+1/2) and west (i-1/2)
                for s in (+1, -1):
                    kap = face_coeff_x(k, j, i) if s > 0 else face_coeff_x(k, j, i - 1)
                    w = kap / (grid.dx * grid.dx)
                    A[c, _idx(grid, k, j, i + s)] += w
                    A[c, c] -= w
                for s in (+1, -1):
                    kap = face_coeff_y(k, j, i) if s > 0 else face_coeff_y(k, j - 1, i)
                    w = kap / (grid.dy * grid.dy)
                    A[c, _idx(grid, k, j + s, i)] += w
                    A[c, c] -= w
                if k + 1 < grid.nz:   # top face k+1, between k and k+1
                    w = face_coeff_z(k + 1, j, i) / (grid.h[k] * (grid.zc[k + 1] - grid.zc[k]))
                    A[c, _idx(grid, k + 1, j, i)] += w
                    A[c, c] -= w
                if k > 0:             # bottom face k, between k-1 and k
                    w = face_coeff_z(k, j, i) / (grid.h[k] * (grid.zc[k] - grid.zc[k - 1]))
                    A[c, _idx(grid, k - 1, j, i)] += w
                    A[c, c] -= w
    return A


def laplacian_matrix(grid):
    one = lambda k, j, i: 1.0  # noqa: E731
    return var_coeff_matrix(grid, one, one, one)


def inv_density_matrix(grid, rho):
    """D(rho_face^-1 G) with rho_face the arithmetic mean of the two cells."""
    rho = np.asarray(rho)
    fx = lambda k, j, i: 2.0 / (rho[k, j, i % grid.nx] + rho[k, j, (i + 1) % grid.nx])  # noqa: E731
    fy = lambda k, j, i: 2.0 / (rho[k, j % grid.ny, i] + rho[k, (j + 1) % grid.ny, i])  # noqa: E731
    fz = lambda k, j, i: 2.0 / (rho[k - 1, j, i] + rho[k, j, i])  # noqa: E731
    return var_coeff_matrix(grid, fx, fy, fz)


def volume_vector(grid):
    v = np.empty(grid.n)
    for k in range(grid.nz):
        v[k * grid.ny * grid.nx:(k + 1) * grid.ny * grid.nx] = grid.dx * grid.dy * grid.h[k]
    return v


def bordered_solve(A, r, vol):
    """Solve [A 1; vol^T 0][p; mu] = [r; 0]: since vol^T A = 0, mu is the
    volume-weighted mean of r and p has zero volume-weighted mean."""
    n = A.shape[0]
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = A
    M[:n, n] = 1.0
    M[n, :n] = vol
    rhs = np.zeros(n + 1)
    rhs[:n] = np.ravel(r)
    sol = np.linalg.solve(M, rhs)
    return sol[:n], sol[n]


def solve_operator(grid):
    """Dense matrix of r -> p for the projected, gauged constant-coefficient solve."""
    A = laplacian_matrix(grid)
    vol = volume_vector(grid)
    n = grid.n
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = A
    M[:n, n] = 1.0
    M[n, :n] = vol
    return np.linalg.inv(M)[:n, :n]
