"""FP64 CPU oracle for the eigenexpansion pressure solve -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product path (the HIP library and its Python
binding) never calls it and shares no code with it.

What it computes, from Dalla Barba et al., "An interface capturing method for
liquid-gas flows at low-Mach number" (arXiv:2005.11806):

* the variable-density pressure equation of Sec. 3.3 (Eq. lap_p),
  div(rho^-1 grad p) = f, with f the user's right-hand side;
* its constant-coefficient recast by Method I (Sec. 3.3.1, Eq. poisson_me1):
  lap p^{s+1} = div[(1 - rho0/rho) grad p^s] + rho0 f, rho0 = min rho;
* one step solved exactly by eigenexpansion (Sec. 3.3.1): forward DFTs in
  the two periodic directions, one tridiagonal solve per wavenumber pair in
  the wall-normal direction, inverse DFTs;
* the adjoint of one step (gradients of sum(w p));
* Method III (Sec. 3.3.1, Eq. new_poisson) and its loop (Algorithm 1): the
  recast through the correction step, iterated with the velocity until the
  summed divergence residual reaches its threshold (``oracle.method3``).

Every routine is the plain definition: matrix-form DFTs, a textbook Thomas
sweep, explicit stencils. Parity-pinned by ``tests/test_oracle_*.py``
against closed forms, dense LU solves, numpy.fft, scipy banded solves and
brute-force Jacobians. Functions without such a pin say "parity unpinned".
"""
from .grid import Grid
from .operators import (face_density, grad, div, laplacian, assemble_method1,
                        mixture_density, divergence_of_faces)
from .dft import rdft_x, dft_y, idft_y, irdft_x
from .tridiag import thomas, z_coefficients, eigen_x, eigen_y
from .solve import solve_const, method1_step, solve, relres, SolveInfo
from .adjoint import adjoint_step
from . import dense
from . import method3

__all__ = [
    "Grid", "face_density", "grad", "div", "laplacian", "assemble_method1", "mixture_density",
    "divergence_of_faces", "rdft_x", "dft_y", "idft_y", "irdft_x", "thomas", "z_coefficients",
    "eigen_x", "eigen_y", "solve_const", "method1_step", "solve", "relres", "SolveInfo",
    "adjoint_step", "dense", "method3",
]
