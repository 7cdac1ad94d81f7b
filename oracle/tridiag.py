"""Oracle (test infrastructure): wall-normal tridiagonal systems and the
eigenvalues of the periodic directions (Sec. 3.3.1, eigenexpansion).

After the two periodic transforms, the 7-point operator decouples into one
tridiagonal system per wavenumber pair (m, n):

    a_k x_{k-1} + (b_k + lx[m] + ly[n]) x_k + c_k x_{k+1} = R_k,

with a_k = 1/(h_k g_k), c_k = 1/(h_k g_{k+1}), b_k = -(a_k + c_k) and the wall
terms a_0 = c_{nz-1} = 0 (zero wall flux).
"""
from __future__ import annotations

import numpy as np


def z_coefficients(grid):
    nz = grid.nz
    a = np.zeros(nz)
    c = np.zeros(nz)
    k = np.arange(1, nz)
    a[k] = 1.0 / (grid.h[k] * grid.g[k])
    k = np.arange(0, nz - 1)
    c[k] = 1.0 / (grid.h[k] * grid.g[k + 1])
    b = -(a + c)
    return a, b, c


def eigen_x(grid):
    """Eigenvalues of the periodic second difference in x for m = 0..Nx/2,
    in the cancellation-free form -4 sin^2(pi m / Nx) / dx^2."""
    m = np.arange(grid.nx // 2 + 1)
    return -4.0 * np.sin(np.pi * m / grid.nx) ** 2 / grid.dx ** 2


def eigen_y(grid):
    n = np.arange(grid.ny)
    return -4.0 * np.sin(np.pi * n / grid.ny) ** 2 / grid.dy ** 2


def thomas(a, b, c, d):
    """Textbook Thomas algorithm for a_k x_{k-1} + b_k x_k + c_k x_{k+1} = d_k,
    vectorised over trailing axes: a, b, c, d have shape [nz, ...]
    (broadcastable); a[0] and c[nz-1] are ignored."""
    nz = d.shape[0]
    shape = np.broadcast(b[0], d[0]).shape
    cp = np.zeros((nz,) + shape)
    dp = np.zeros((nz,) + np.broadcast(b[0], d[0]).shape, dtype=np.result_type(d, b))
    piv = b[0] * np.ones(shape)
    cp[0] = c[0] / piv
    dp[0] = d[0] / piv
    for k in range(1, nz):
        piv = b[k] - a[k] * cp[k - 1]
        cp[k] = c[k] / piv
        dp[k] = (d[k] - a[k] * dp[k - 1]) / piv
    x = np.zeros_like(dp)
    x[nz - 1] = dp[nz - 1]
    for k in range(nz - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x
