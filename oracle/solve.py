"""Oracle (test infrastructure): the eigenexpansion solve of one constant-
coefficient step and the Method-I chain.

Sec. 3.3.1: once the variable-coefficient equation (Eq. lap_p) is recast with a
constant coefficient, the Poisson problem is solved exactly by eigenexpansion.
Here that is, for the right-hand side r of one step:

  1. compatibility: remove the volume-weighted mean of r (the Neumann problem
     is singular; the paper is silent on this and on the gauge);
  2. forward DFT along x (half spectrum), then along y;
  3. for every (m, n) != (0, 0): Thomas solve of the wall-normal system;
  4. (0, 0): integrate the flux from the bottom wall, then fix the gauge
     sum_k h_k p_k = 0 (zero volume-weighted mean of p);
  5. inverse DFT along y, real inverse along x, times 1/(Nx Ny).

Method I (Eq. poisson_me1) repeats steps 1-5 on
r = D[(1 - rho0/rho) G p^s] + rho0 f with p^s the previous iterate and
rho0 = min rho; ``n_steps`` such steps form a chain with f, rho, rho0 fixed.
"""
from __future__ import annotations

import dataclasses
import numpy as np

from .dft import rdft_x, dft_y, idft_y, irdft_x
from .tridiag import thomas, z_coefficients, eigen_x, eigen_y
from .operators import assemble_method1, laplacian


@dataclasses.dataclass
class SolveInfo:
    rho0_used: float
    rhs_mean_removed: float
    relres: float
    relres_inf: float


def spectral_rhs(r, grid):
    """Steps 1-2: projected RHS and its 2-D spectrum [nz, ny, nx/2+1]."""
    vol = grid.volume_field()
    mean = float((vol * r).sum() / vol.sum())
    rp = r - mean
    return rp, mean, dft_y(rdft_x(rp))


def zero_mode_column(r00, grid):
    """Step 4 on the (0,0) column: project, integrate the flux, fix the gauge.

    With zero wall flux, D_z G_z x = r gives the face flux
    F_{k+1} = sum_{j<=k} h_j r_j, and x_{k+1} = x_k + g_{k+1} F_{k+1}."""
    r00 = r00 - np.sum(grid.h * r00) / grid.lz
    phi = np.cumsum(grid.h * r00)
    x = np.zeros(grid.nz, dtype=r00.dtype)
    for k in range(grid.nz - 1):
        x[k + 1] = x[k] + grid.g[k + 1] * phi[k]
    return x - np.sum(grid.h * x) / grid.lz


def solve_spectrum(R, grid):
    """Step 3-4: wall-normal solves for every wavenumber pair."""
    a, b, c = z_coefficients(grid)
    lam = (eigen_y(grid)[:, None] + eigen_x(grid)[None, :]).ravel()  # [(n, m)]
    nz = grid.nz
    Rf = R.reshape(nz, -1)
    X = np.zeros_like(Rf)
    # (m, n) = (0, 0) is flat index 0; all other pairs are non-singular.
    X[:, 1:] = thomas(a[:, None], b[:, None] + lam[None, 1:], c[:, None], Rf[:, 1:])
    X[:, 0] = zero_mode_column(Rf[:, 0], grid)
    return X.reshape(R.shape)


def inverse_spectrum(X, grid):
    """Step 5."""
    return irdft_x(idft_y(X), grid.nx) / (grid.nx * grid.ny)


def solve_const(r, grid):
    """Exact solve of L p = r - mean_V(r) with sum_V p = 0. Returns (p, mean)."""
    _, mean, R = spectral_rhs(r, grid)
    return inverse_spectrum(solve_spectrum(R, grid), grid), mean


def relres(r, p, grid):
    """||r_proj - L p||_2 / ||r_proj||_2 (and the max-norm ratio), with r_proj the
    projected RHS of the step and L the 7-point operator applied directly."""
    vol = grid.volume_field()
    rp = r - (vol * r).sum() / vol.sum()
    res = rp - laplacian(p, grid)
    nr = np.linalg.norm(rp.ravel())
    if nr == 0.0:
        return 0.0, 0.0
    return (float(np.linalg.norm(res.ravel()) / nr),
            float(np.abs(res).max() / np.abs(rp).max()))


def method1_step(f, rho, p_prev, rho0, grid):
    """One Method-I step (Eq. poisson_me1). Returns (p, r, mean)."""
    r = assemble_method1(f, rho, p_prev, rho0, grid)
    p, mean = solve_const(r, grid)
    return p, r, mean


def solve(f, grid, rho=None, p_prev=None, rho0=None, n_steps=1, with_relres=True):
    """Chain of n_steps solves. rho None selects the constant-coefficient solve
    p = S(f); otherwise Method I with rho0 = min(rho) unless given and p_prev
    (zeros if None). Returns the list of iterates and their SolveInfo."""
    ps, infos = [], []
    if rho is None:
        p, mean = solve_const(f, grid)
        rr = relres(f, p, grid) if with_relres else (np.nan, np.nan)
        return [p], [SolveInfo(np.nan, mean, *rr)]
    if rho0 is None:
        rho0 = float(rho.min())
    prev = np.zeros(grid.shape) if p_prev is None else p_prev
    for _ in range(n_steps):
        p, r, mean = method1_step(f, rho, prev, rho0, grid)
        rr = relres(r, p, grid) if with_relres else (np.nan, np.nan)
        ps.append(p)
        infos.append(SolveInfo(rho0, mean, *rr))
        prev = p
    return ps, infos
