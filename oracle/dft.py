"""Oracle (test infrastructure): discrete Fourier transforms by their
definition, in matrix form (one dense matrix product per direction).

Conventions (the paper does not fix them): forward transforms are
unnormalised with exp(-2 pi i j m / N); the inverse carries 1/(Nx Ny); the x
transform of a real field keeps the half spectrum m = 0..Nx/2 (Nyquist mode
included). Exponents use the exact integer reduction (j*m mod N) before the
angle is formed.
"""
from __future__ import annotations

import numpy as np


def _omega(n, rows, cols, sign):
    idx = np.mod(np.outer(rows, cols), n).astype(np.float64)
    return np.exp(sign * 2j * np.pi * idx / n)


def rdft_x(r):
    """R[..., m] = sum_i r[..., i] exp(-2 pi i m i / Nx), m = 0..Nx/2."""
    nx = r.shape[-1]
    w = _omega(nx, np.arange(nx), np.arange(nx // 2 + 1), -1.0)  # [nx, nx/2+1]
    return r @ w


def dft_y(R):
    """Unnormalised forward DFT along axis -2 (y)."""
    ny = R.shape[-2]
    w = _omega(ny, np.arange(ny), np.arange(ny), -1.0)  # [n, j]
    return np.einsum("nj,...jm->...nm", w, R, optimize=True)


def idft_y(R):
    """Unnormalised inverse DFT along axis -2 (y): sum_n R[n] exp(+2 pi i n j / Ny)."""
    ny = R.shape[-2]
    w = _omega(ny, np.arange(ny), np.arange(ny), 1.0)  # [j, n]
    return np.einsum("jn,...nm->...jm", w, R, optimize=True)


def irdft_x(X, nx):
    """Real inverse along x from the half spectrum m = 0..Nx/2, unnormalised:

        x_i = Re X_0 + 2 sum_{m=1}^{Nx/2-1} Re(X_m exp(+2 pi i m i / Nx)) + Re X_{Nx/2} (-1)^i

    (Hermitian symmetry X_{Nx-m} = conj(X_m) for a real result)."""
    m = np.arange(nx // 2 + 1)
    wt = np.full(nx // 2 + 1, 2.0)
    wt[0] = 1.0
    wt[nx // 2] = 1.0
    w = _omega(nx, m, np.arange(nx), 1.0) * wt[:, None]  # [m, i]
    return (X @ w).real
