"""Cross-check of the wall-normal solve by a DCT in z on uniform grids.

With homogeneous Neumann walls (the reading of Sec. 3.3.1's homogeneous
pressure condition) and uniform spacing h, the cell-centred 3-point z
operator is diagonalised by the DCT-II basis cos(pi m (k + 1/2) / nz), with
eigenvalue -4 sin^2(pi m / (2 nz)) / h^2: the eigenexpansion of Sec. 3.3.1
then holds in z as well as in x and y. `dct_solve` below is built from
scipy's DCT-II and numpy's FFTs only; it shares nothing with the oracle's
Thomas sweeps or the GPU's chunked partition method, and both are compared
with it (the oracle here on the CPU, the GPU in the `gpu` tests).
"""
import numpy as np
import pytest
import scipy.fft

import oracle as O


def dct_solve(r, nx, ny, nz, lx, ly, lz, dct_type=2, zarg_den=None):
    """L p = r - mean(r), mean(p) = 0, on a uniform periodic-x/y, Neumann-z
    grid: DCT-II in z, FFTs in y and x, division by the eigenvalues.
    (dct_type and zarg_den exist only to plant slips in the test below: the
    z transform's type and the denominator of the z eigenvalue's angle.)"""
    dx, dy, dz = lx / nx, ly / ny, lz / nz
    zden = 2 * nz if zarg_den is None else zarg_den
    r = r - r.mean()  # uniform cells: the volume-weighted mean is the plain mean
    R = np.fft.fft2(scipy.fft.dct(r, type=dct_type, axis=0, norm="ortho"), axes=(1, 2))
    lam = ((-4.0 * np.sin(np.pi * np.arange(nz) / zden) ** 2 / dz ** 2)[:, None, None]
           + (-4.0 * np.sin(np.pi * np.arange(ny) / ny) ** 2 / dy ** 2)[None, :, None]
           + (-4.0 * np.sin(np.pi * np.arange(nx) / nx) ** 2 / dx ** 2)[None, None, :])
    lam[0, 0, 0] = 1.0
    X = R / lam
    X[0, 0, 0] = 0.0
    x = np.fft.ifft2(X, axes=(1, 2)).real
    return scipy.fft.idct(x, type=dct_type, axis=0, norm="ortho")


SHAPES = [(16, 12, 10), (32, 1, 24), (24, 18, 9)]


def _case(nx, ny, nz, seed):
    rng = np.random.default_rng([200511806, 77, nx, ny, nz, seed])
    lx, ly, lz = 1.0, ny / nx, nz / nx
    return rng.standard_normal((nz, ny, nx)), (lx, ly, lz)


@pytest.mark.parametrize("shape", SHAPES)
def test_dct_solve_meets_the_stencil(shape):
    """The DCT solve is a solution: the oracle's directly applied 7-point
    stencil leaves a relative residual at rounding level, and p has zero mean."""
    nx, ny, nz = shape
    r, (lx, ly, lz) = _case(nx, ny, nz, 0)
    g = O.Grid(nx, ny, nz, lx, ly, lz)
    p = dct_solve(r, nx, ny, nz, lx, ly, lz)
    rr, _ = O.relres(r, p, g)
    assert rr < 1e-13
    assert abs(p.mean()) < 1e-13 * np.abs(p).max()


@pytest.mark.parametrize("shape", SHAPES)
def test_oracle_thomas_path_equals_dct_solve(shape):
    nx, ny, nz = shape
    r, (lx, ly, lz) = _case(nx, ny, nz, 1)
    g = O.Grid(nx, ny, nz, lx, ly, lz)
    p, mean = O.solve_const(r, g)
    ref = dct_solve(r, nx, ny, nz, lx, ly, lz)
    assert np.abs(p - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(mean - r.mean()) <= 1e-14 * np.abs(r).max()


def test_cross_check_rejects_planted_slips():
    """The comparison would catch a wrong z basis or eigenvalue: DCT-I in z,
    and sin(pi m / nz) in place of sin(pi m / (2 nz)), both miss the oracle."""
    nx, ny, nz = 16, 12, 10
    r, (lx, ly, lz) = _case(nx, ny, nz, 2)
    p, _ = O.solve_const(r, O.Grid(nx, ny, nz, lx, ly, lz))
    for slip in (dict(dct_type=1), dict(zarg_den=nz)):
        bad = dct_solve(r, nx, ny, nz, lx, ly, lz, **slip)
        assert np.abs(p - bad).max() > 1e-3 * np.abs(p).max(), slip


@pytest.mark.gpu
@pytest.mark.parametrize("shape,kc", [((128, 1, 256), 8), ((48, 32, 42), 4), ((64, 64, 64), 16)])
def test_gpu_partition_solve_equals_dct_solve(gpu, shape, kc):
    """The GPU's chunked partition solve (local elimination, interface scan,
    back substitution) against the DCT solve: the paper's 2-D 128 x 256 grid
    and two 3-D grids, the first with a ragged last chunk (42 = 10 x 4 + 2)."""
    from tests.gpu_util import dev, host, say
    nx, ny, nz = shape
    r, (lx, ly, lz) = _case(nx, ny, nz, 3)
    say(f"dct cross-check {shape} kc {kc}")
    plan = gpu.Plan(gpu.Grid(nx, ny, nz, lx, ly, lz), method="const", chunk_rows=kc)
    p = host(plan.solve(dev(r)))
    ref = dct_solve(r, nx, ny, nz, lx, ly, lz)
    assert np.abs(p - ref).max() <= 1e-11 * np.abs(ref).max()
