"""Oracle (test infrastructure): adjoint of one Method-I step.

For loss = sum(w * p) with p = S(A(f, rho, p_prev)), A the Method-I assembly
(Sec. 3.3.1, Eq. poisson_me1) and S the eigenexpansion solve (projection and
gauge included):

* S is self-adjoint in the volume-weighted inner product, so S^T = V S V^-1
  (V = diag of cell volumes) and lambda = S^T w = V S(V^-1 w);
* dL/df      = rho0 lambda;
* dL/dbeta_f = (D^T lambda)_f (G p_prev)_f =: gface, with
  (D^T lambda)_f = lambda_L / h_L - lambda_R / h_R across face f;
* beta_f = 1 - rho0/rho_f and rho_f = (rho_L + rho_R)/2, so each adjacent cell
  receives gface rho0 / (2 rho_f^2);
* dL/drho0   = sum(lambda f) - sum_f gface / rho_f (rho0 as an independent input);
* dL/dp_prev = G^T (beta (D^T lambda)).
"""
from __future__ import annotations

import dataclasses
import numpy as np

from .operators import grad, face_density
from .solve import solve_const


@dataclasses.dataclass
class AdjointResult:
    lam: np.ndarray
    grad_f: np.ndarray
    grad_rho: np.ndarray
    grad_rho0: float
    grad_p_prev: np.ndarray


def div_transpose(lam, grid):
    """D^T lambda on faces (same storage as ``grad``); zero on the walls."""
    dx = (lam - np.roll(lam, -1, axis=2)) / grid.dx
    dy = (lam - np.roll(lam, -1, axis=1)) / grid.dy
    dz = np.zeros((grid.nz + 1, grid.ny, grid.nx))
    h = grid.h[:, None, None]
    dz[1:grid.nz] = lam[:-1] / h[:-1] - lam[1:] / h[1:]
    return dx, dy, dz


def grad_transpose(fx, fy, fz, grid):
    """G^T F at cells: (G p)_f = (p_R - p_L)/d_f, so each face gives -F/d_f to its
    left cell and +F/d_f to its right cell."""
    out = (np.roll(fx, 1, axis=2) - fx) / grid.dx
    out = out + (np.roll(fy, 1, axis=1) - fy) / grid.dy
    fzg = np.zeros_like(fz)
    fzg[1:grid.nz] = fz[1:grid.nz] / grid.g[1:grid.nz, None, None]
    out = out + fzg[:-1] - fzg[1:]
    return out


def adjoint_step(w, f, rho, rho0, p_prev, grid):
    vol = grid.volume_field()
    lam = vol * solve_const(w / vol, grid)[0]
    dtx, dty, dtz = div_transpose(lam, grid)
    gx, gy, gz = grad(p_prev, grid)
    rx, ry, rz = face_density(rho, grid)
    nz = grid.nz
    gfx, gfy = dtx * gx, dty * gy
    gfz = np.zeros_like(gz)
    gfz[1:nz] = dtz[1:nz] * gz[1:nz]
    # d loss / d rho_face, split half to each adjacent cell
    cx = gfx * rho0 / rx ** 2
    cy = gfy * rho0 / ry ** 2
    cz = np.zeros_like(gfz)
    cz[1:nz] = gfz[1:nz] * rho0 / rz[1:nz] ** 2
    grad_rho = 0.5 * (cx + np.roll(cx, 1, axis=2)) + 0.5 * (cy + np.roll(cy, 1, axis=1)) \
        + 0.5 * (cz[:-1] + cz[1:])
    grad_rho0 = float((lam * f).sum() - (gfx / rx).sum() - (gfy / ry).sum()
                      - (gfz[1:nz] / rz[1:nz]).sum())
    bz = np.zeros_like(dtz)
    bz[1:nz] = (1.0 - rho0 / rz[1:nz]) * dtz[1:nz]
    grad_p = grad_transpose((1.0 - rho0 / rx) * dtx, (1.0 - rho0 / ry) * dty, bz, grid)
    return AdjointResult(lam, rho0 * lam, grad_rho, grad_rho0, grad_p)
