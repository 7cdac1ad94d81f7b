"""Pins of the FP64 oracle against results fixed by mathematics, independent
libraries and brute force (no GPU). Each test names the passage or fact it
checks; each is chosen so that a plausible slip (dropped term, wrong sign or
index, transposed operand, wrong spacing on a stretched grid) fails."""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
from oracle import dense, adjoint as oadj
import workloads as W


def _rng(s=0):
    return np.random.default_rng([7, s])


def _grid(nx, ny, nz, stretched=False, lz=None):
    lz = lz if lz is not None else nz / nx
    zf = W.tanh_faces(nz, lz, 1.5) if stretched else None
    return O.Grid(nx, ny, nz, 1.0, 1.0, lz, zf)


# ---------------------------------------------------------------- transforms
@pytest.mark.parametrize("nx,ny", [(8, 6), (12, 18), (32, 96)])
def test_dft_matches_numpy_fft(nx, ny):
    """Matrix-form DFTs against numpy.fft (an independent FFT library)."""
    r = _rng(1).standard_normal((3, ny, nx))
    Rx = O.rdft_x(r)
    assert np.allclose(Rx, np.fft.rfft(r, axis=-1), rtol=0, atol=1e-12)
    R = O.dft_y(Rx)
    assert np.allclose(R, np.fft.fft(Rx, axis=-2), rtol=0, atol=1e-11)
    back = O.idft_y(R)
    assert np.allclose(back, ny * np.fft.ifft(R, axis=-2), rtol=0, atol=1e-10)
    x = O.irdft_x(back, nx) / (nx * ny)
    assert np.allclose(x, r, rtol=0, atol=1e-13)
    assert np.allclose(O.irdft_x(Rx, nx), nx * np.fft.irfft(Rx, n=nx, axis=-1), atol=1e-11)


def test_parseval():
    r = _rng(2).standard_normal((2, 16, 24))
    F = O.dft_y(O.rdft_x(r))
    # half spectrum: interior m counted twice
    wt = np.full(24 // 2 + 1, 2.0)
    wt[0] = wt[-1] = 1.0
    e_spec = (np.abs(F) ** 2 * wt).sum() / (16 * 24)
    assert np.isclose(e_spec, (r ** 2).sum(), rtol=1e-13)


# ---------------------------------------------------------------- tridiagonal
def test_thomas_matches_scipy_banded():
    r = _rng(3)
    nz, ns = 40, 7
    a = r.uniform(0.5, 1.0, nz)
    c = r.uniform(0.5, 1.0, nz)
    shift = -r.uniform(0.1, 50.0, ns)
    b = -(a + c)
    d = r.standard_normal((nz, ns)) + 1j * r.standard_normal((nz, ns))
    x = O.thomas(a[:, None], b[:, None] + shift[None, :], c[:, None], d)
    for s in range(ns):
        ab = np.zeros((3, nz))
        ab[0, 1:] = c[:-1]
        ab[1] = b + shift[s]
        ab[2, :-1] = a[1:]
        ref = scipy.linalg.solve_banded((1, 1), ab, d[:, s])
        assert np.allclose(x[:, s], ref, rtol=1e-13, atol=1e-14)


def test_z_coefficients_reproduce_flux_form():
    """a_k, b_k, c_k applied to a column equal D_z G_z of that column."""
    g = _grid(2, 2, 9, stretched=True, lz=1.3)
    a, b, c = O.z_coefficients(g)
    col = _rng(4).standard_normal(9)
    p = np.broadcast_to(col[:, None, None], g.shape).copy()
    Lp = O.laplacian(p, g)[:, 0, 0]
    tri = b * col
    tri[1:] += a[1:] * col[:-1]
    tri[:-1] += c[:-1] * col[1:]
    assert np.allclose(tri, Lp, rtol=1e-13, atol=1e-10)
    assert a[0] == 0.0 and c[-1] == 0.0


# ---------------------------------------------------------------- solve pins
@pytest.mark.parametrize("shape,mode", [((32, 32, 32), (1, 2, 3)), ((12, 8, 10), (5, 3, 9)),
                                        ((96, 64, 24), (47, 31, 1))])
def test_manufactured_eigenmode_closed_form(shape, mode):
    """cos(2 pi a x) cos(2 pi b y) cos(pi m z / Lz) is an exact eigenvector of the
    uniform-grid 7-point operator with eigenvalue
    -4 sin^2(pi a/Nx)/dx^2 - 4 sin^2(pi b/Ny)/dy^2 - 4 sin^2(pi m/(2 Nz))/dz^2."""
    nx, ny, nz = shape
    spec = W.uniform_grid(nx, ny, nz)
    g = O.Grid.from_spec(spec)
    a, b, m = mode
    M = W.manufactured_mode(spec, a, b, m)
    dz = g.lz / nz
    lam = (-4 * np.sin(np.pi * a / nx) ** 2 / g.dx ** 2 - 4 * np.sin(np.pi * b / ny) ** 2 / g.dy ** 2
           - 4 * np.sin(np.pi * m / (2 * nz)) ** 2 / dz ** 2)
    assert np.allclose(O.laplacian(M, g), lam * M, rtol=0, atol=1e-9 * abs(lam))
    p, mean = O.solve_const(M, g)
    assert abs(mean) < 1e-14
    assert np.abs(p - M / lam).max() <= 1e-13 * np.abs(M / lam).max()


@pytest.mark.parametrize("shape,stretched", [((6, 4, 5), False), ((4, 6, 6), True),
                                             ((8, 8, 7), True)])
def test_solve_matches_dense_bordered_lu(shape, stretched):
    g = _grid(*shape, stretched=stretched)
    r = _rng(5).standard_normal(g.shape) + 0.3
    p, mean = O.solve_const(r, g)
    A = dense.laplacian_matrix(g)
    pd, mu = dense.bordered_solve(A, r, dense.volume_vector(g))
    assert np.abs(p.ravel() - pd).max() <= 1e-12 * np.abs(pd).max()
    assert np.isclose(mean, mu, rtol=1e-12)


def test_dense_laplacian_matches_stencil():
    g = _grid(6, 4, 7, stretched=True, lz=1.0)
    A = dense.laplacian_matrix(g)
    p = _rng(6).standard_normal(g.shape)
    assert np.allclose(A @ p.ravel(), O.laplacian(p, g).ravel(), rtol=0, atol=1e-10)


def test_relres_and_gauge_32cubed():
    c = W.const32()
    g = O.Grid.from_spec(c.grid)
    f = O.divergence_of_faces(*c.faces, g) + c.extra_rhs
    (p,), (info,) = O.solve(f, g)
    assert info.relres < 1e-13
    assert abs((g.volume_field() * p).sum()) < 1e-14 * np.abs(p).max() * g.lx * g.ly * g.lz
    # divergence of a field with zero wall flux has zero volume-weighted mean
    assert abs(info.rhs_mean_removed) < 1e-13


def test_zero_mode_column_integration():
    """(0,0) column: result satisfies the singular Neumann tridiagonal system
    after projection and has zero h-weighted mean."""
    g = _grid(2, 2, 11, stretched=True, lz=2.0)
    r00 = _rng(8).standard_normal(11) + 0.5
    from oracle.solve import zero_mode_column
    x = zero_mode_column(r00, g)
    a, b, c = O.z_coefficients(g)
    Lx = b * x
    Lx[1:] += a[1:] * x[:-1]
    Lx[:-1] += c[:-1] * x[1:]
    rp = r00 - np.sum(g.h * r00) / g.lz
    assert np.allclose(Lx, rp, atol=1e-12)
    assert abs(np.sum(g.h * x)) < 1e-14


# ---------------------------------------------------------------- invariants
def test_invariants_flux_form_and_symmetry():
    g = _grid(6, 4, 7, stretched=True, lz=1.5)
    r = _rng(9)
    ux, uy, uz = (r.standard_normal(g.shape), r.standard_normal(g.shape),
                  r.standard_normal((g.nz + 1, g.ny, g.nx)))
    uz[0] = uz[-1] = 0.0
    vol = g.volume_field()
    assert abs((vol * O.divergence_of_faces(ux, uy, uz, g)).sum()) < 1e-13
    A = dense.laplacian_matrix(g)
    VA = dense.volume_vector(g)[:, None] * A
    assert np.abs(VA - VA.T).max() < 1e-12 * np.abs(VA).max()
    assert np.abs(A @ np.ones(g.n)).max() < 1e-9


def test_mixture_density_limits():
    """Eq. eq_22 with Phi = 1 in gas."""
    phi = np.array([0.0, 1.0, 0.25])
    rg = np.array([2.0, 3.0, 5.0])
    rho = O.mixture_density(phi, rg, 1000.0)
    assert rho[0] == 1000.0 and rho[1] == 3.0
    assert np.isclose(rho[2], 0.25 * 5 + 0.75 * 1000)


# ---------------------------------------------------------------- Method I
def _two_phase_tiny(g, seed=10, ratio=1000.0):
    r = _rng(seed)
    rho = 1.0 + (ratio - 1.0) * r.random(g.shape)
    return rho


@pytest.mark.parametrize("stretched", [False, True])
def test_method1_fixed_point(stretched):
    """Eq. poisson_me1: if p_prev solves D(rho_f^-1 G p) = f exactly (dense LU of
    an independently assembled variable-coefficient matrix), one Method-I
    step returns it unchanged."""
    g = _grid(4, 6, 5, stretched=stretched, lz=1.0)
    rho = _two_phase_tiny(g)
    B = dense.inv_density_matrix(g, rho)
    vol = dense.volume_vector(g)
    f = _rng(11).standard_normal(g.n)
    ps, _ = dense.bordered_solve(B, f, vol)
    f_c = (B @ ps).reshape(g.shape)  # the compatible part of f
    p1, _, _ = O.method1_step(f_c, rho, ps.reshape(g.shape), float(rho.min()), g)
    assert np.abs(p1.ravel() - ps).max() <= 1e-12 * np.abs(ps).max()


def test_method1_constant_density_is_textbook_poisson():
    g = _grid(6, 4, 5, stretched=True, lz=1.0)
    rho = np.full(g.shape, 3.7)
    f = _rng(12).standard_normal(g.shape)
    junk = _rng(13).standard_normal(g.shape)
    p, _, _ = O.method1_step(f, rho, junk, 3.7, g)
    pd, _ = dense.bordered_solve(dense.laplacian_matrix(g), 3.7 * f, dense.volume_vector(g))
    assert np.abs(p.ravel() - pd).max() <= 1e-12 * np.abs(pd).max()


def test_method1_energy_norm_contraction():
    """The Method-I error e = p^s - p* obeys ||G e^{s+1}|| <= beta_max ||G e^s||
    in the face-volume-weighted norm, beta_max = 1 - rho0/max(rho_face)."""
    g = _grid(6, 4, 6, stretched=True, lz=1.0)
    rho = _two_phase_tiny(g, seed=14, ratio=50.0)
    B = dense.inv_density_matrix(g, rho)
    vol = dense.volume_vector(g)
    ps, _ = dense.bordered_solve(B, _rng(15).standard_normal(g.n), vol)
    f = (B @ ps).reshape(g.shape)
    rho0 = float(rho.min())
    rx, ry, rz = O.face_density(rho, g)
    beta_max = 1.0 - rho0 / max(rx.max(), ry.max(), np.nanmax(rz))

    def enorm(e):
        gx, gy, gz = O.grad(e.reshape(g.shape), g)
        wz = g.dx * g.dy * np.concatenate([[0.0], g.g[1:g.nz], [0.0]])
        # -<e, L e>_V: x and y faces weigh the cell volume, z faces dx dy g_k
        return np.sqrt((gx ** 2 * g.volume_field()).sum() + (gy ** 2 * g.volume_field()).sum()
                       + (gz ** 2 * wz[:, None, None]).sum())

    p = np.zeros(g.shape)
    prev = enorm(p.ravel() - ps)
    for _ in range(5):
        p, _, _ = O.method1_step(f, rho, p, rho0, g)
        cur = enorm(p.ravel() - ps)
        assert cur <= beta_max * prev * (1 + 1e-12)
        prev = cur


def test_o2_convergence_on_tanh_grid():
    """Second-order convergence of the discrete solution to the continuous
    solution of lap p = s on the tanh-stretched grid."""
    errs = []
    for n in (8, 16, 32):
        zf = W.tanh_faces(2 * n, 2.0, 1.5)
        g = O.Grid(n, n, 2 * n, 1.0, 1.0, 2.0, zf)
        x = (np.arange(n) + 0.5) / n
        z = g.zc
        exact = (np.cos(np.pi * z / 2.0)[:, None, None] * np.cos(2 * np.pi * x)[None, :, None]
                 * np.cos(2 * np.pi * x)[None, None, :])
        lam = -(8 * np.pi ** 2 + (np.pi / 2.0) ** 2)
        p, _ = O.solve_const(lam * exact, g)
        e = exact - (g.volume_field() * exact).sum() / (g.lx * g.ly * g.lz)
        errs.append(np.abs(p - e).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)


# ---------------------------------------------------------------- adjoint
def test_solve_transpose_identity():
    """S^T = V S V^-1 for the projected, gauged solve (dense)."""
    g = _grid(4, 4, 5, stretched=True, lz=1.0)
    S = dense.solve_operator(g)
    v = dense.volume_vector(g)
    assert np.abs(S.T - v[:, None] * S / v[None, :]).max() < 1e-11 * np.abs(S).max()


def _loss(w, f, rho, rho0, p_prev, g):
    p, _, _ = O.method1_step(f, rho, p_prev, rho0, g)
    return float((w * p).sum())


def test_adjoint_bruteforce_jacobian():
    """Every column of the Jacobians w.r.t. f and p_prev by a forward solve of a
    unit vector (the step is affine in each), against the adjoint."""
    g = _grid(4, 4, 4, stretched=True, lz=1.0)
    r = _rng(16)
    rho = 1.0 + 99.0 * r.random(g.shape)
    rho0 = float(rho.min())
    f, pp, w = r.standard_normal(g.shape), r.standard_normal(g.shape), r.standard_normal(g.shape)
    res = oadj.adjoint_step(w, f, rho, rho0, pp, g)
    base = _loss(w, f, rho, rho0, pp, g)
    gf = np.zeros(g.n)
    gp = np.zeros(g.n)
    for c in range(g.n):
        e = np.zeros(g.n)
        e[c] = 1.0
        e = e.reshape(g.shape)
        gf[c] = _loss(w, f + e, rho, rho0, pp, g) - base
        gp[c] = _loss(w, f, rho, rho0, pp + e, g) - base
    assert np.allclose(res.grad_f.ravel(), gf, rtol=1e-9, atol=1e-11)
    assert np.allclose(res.grad_p_prev.ravel(), gp, rtol=1e-9, atol=1e-11)


def test_adjoint_density_central_differences():
    g = _grid(4, 4, 3, stretched=True, lz=1.0)
    r = _rng(17)
    rho = 1.0 + 9.0 * r.random(g.shape)
    rho0 = 0.5  # independent input, below min(rho)
    f, pp, w = r.standard_normal(g.shape), r.standard_normal(g.shape), r.standard_normal(g.shape)
    res = oadj.adjoint_step(w, f, rho, rho0, pp, g)
    h = 1e-4  # truncation ~ (h/rho)^2 ~ 1e-8 relative; rounding ~ 1e-12
    fd = np.zeros(g.n)
    for c in range(g.n):
        e = np.zeros(g.n)
        e[c] = h
        e = e.reshape(g.shape)
        fd[c] = (_loss(w, f, rho + e, rho0, pp, g) - _loss(w, f, rho - e, rho0, pp, g)) / (2 * h)
    assert np.allclose(res.grad_rho.ravel(), fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())
    fd0 = (_loss(w, f, rho, rho0 + h, pp, g) - _loss(w, f, rho, rho0 - h, pp, g)) / (2 * h)
    assert np.isclose(res.grad_rho0, fd0, rtol=1e-6)


def test_adjoint_dot_product_identity():
    """<w, dp/df v> = <grad_f, v> on a stretched grid."""
    g = _grid(8, 6, 7, stretched=True, lz=1.0)
    r = _rng(18)
    rho = 1.0 + 999.0 * r.random(g.shape)
    rho0 = float(rho.min())
    f, pp, w, v = (r.standard_normal(g.shape) for _ in range(4))
    res = oadj.adjoint_step(w, f, rho, rho0, pp, g)
    jv = O.solve_const(rho0 * v, g)[0]
    assert np.isclose((w * jv).sum(), (res.grad_f * v).sum(), rtol=1e-11)


@pytest.mark.parametrize("stretched", [False, True])
def test_two_dimensional_solve_matches_dense(stretched):
    """ny = 1 (one periodic cell in y, the paper's two-dimensional cases):
    the eigenexpansion solve equals dense bordered LU of the 5-point x-z
    operator, and the y fluxes vanish."""
    g = O.Grid(12, 1, 7, 1.0, 0.4, 1.3, W.tanh_faces(7, 1.3, 1.5) if stretched else None)
    f = _rng(40).standard_normal(g.shape)
    p, _ = O.solve_const(f, g)
    pd, _ = dense.bordered_solve(dense.laplacian_matrix(g), f, dense.volume_vector(g))
    assert np.abs(p.ravel() - pd).max() <= 1e-12 * np.abs(pd).max()
    gx, gy, gz = O.grad(p, g)
    assert np.all(gy == 0.0)
