"""Pins of two oracle functions that the other pins only exercise indirectly:
the relative residual (``oracle.relres``) and the Method-I chain
(``oracle.solve`` with n_steps > 1). No GPU.

Both references below are built without the oracle's vectorised stencils or
its spectral solve: the operators are the loop-assembled dense matrices of
``oracle.dense`` and the compatibility projection is an explicit matrix.

* relres: ||P r - A p||_2 / ||P r||_2 with A the 7-point operator, P the
  volume-weighted projection I - 1 v^T / (1^T v) and unweighted 2-norms over
  cells (the reading of "relative residual" for the step's constant-coefficient
  system; the projection is the compatibility condition of the singular
  Neumann problem, Sec. 3.3.1).
* chain: Method I (Sec. 3.3.1, Eq. poisson_me1) repeated, each step
  p_{s+1} = A^+ (B p_s + rho0 f) with B = D((1 - rho0/rho_f) G) assembled
  face by face and A^+ the bordered LU solve (zero volume-weighted mean),
  p_0 = p_prev, rho0 fixed over the chain (given, or min rho).

The last test plants plausible slips in copies of the two functions and checks
that the pins reject every one of them.
"""
import numpy as np
import pytest

import oracle as O
from oracle import dense
import workloads as W


def _rng(s):
    return np.random.default_rng([11, s])


def _tanh_grid(nx, ny, nz, lz=1.3):
    return O.Grid(nx, ny, nz, 1.0, 1.0, lz, W.tanh_faces(nz, lz, 1.5))


def _dense_relres(g, r, p):
    A = dense.laplacian_matrix(g)
    v = dense.volume_vector(g)
    P = np.eye(g.n) - np.outer(np.ones(g.n), v) / v.sum()
    rp = P @ np.ravel(r)
    res = rp - A @ np.ravel(p)
    return np.linalg.norm(res) / np.linalg.norm(rp)


def _dense_step_matrices(g, rho, rho0):
    rho = np.asarray(rho)
    bx = lambda k, j, i: 1.0 - 2.0 * rho0 / (rho[k, j, i % g.nx] + rho[k, j, (i + 1) % g.nx])  # noqa: E731
    by = lambda k, j, i: 1.0 - 2.0 * rho0 / (rho[k, j % g.ny, i] + rho[k, (j + 1) % g.ny, i])  # noqa: E731
    bz = lambda k, j, i: 1.0 - 2.0 * rho0 / (rho[k - 1, j, i] + rho[k, j, i])  # noqa: E731
    return dense.laplacian_matrix(g), dense.var_coeff_matrix(g, bx, by, bz), dense.volume_vector(g)


def _dense_chain(g, f, rho, rho0, p_prev, n_steps):
    """Iterates and right-hand sides of n_steps Method-I steps (dense)."""
    A, B, v = _dense_step_matrices(g, rho, rho0)
    prev = np.ravel(p_prev)
    ps, rs = [], []
    for _ in range(n_steps):
        r = B @ prev + rho0 * np.ravel(f)
        p, _ = dense.bordered_solve(A, r, v)
        ps.append(p.reshape(g.shape))
        rs.append(r.reshape(g.shape))
        prev = p
    return ps, rs


def _relres_cases():
    """(grid, r, p): a non-compatible r (nonzero volume-weighted mean) on a
    stretched grid with p far from the solution, and with p close to it."""
    g = _tanh_grid(4, 6, 7)
    r = _rng(1).standard_normal(g.shape) + 0.7
    p_far = _rng(2).standard_normal(g.shape)
    p_sol, _ = O.solve_const(r, g)
    p_near = p_sol + 1e-7 * _rng(3).standard_normal(g.shape)
    return [(g, r, p_far), (g, r, p_near)]


# The two residuals are formed by different operators (dense rows against the
# vectorised stencil), so they agree to rounding: about eps ||P r|| in absolute
# terms, whatever the size of the residual itself.
_RTOL, _ATOL = 1e-10, 1e-13


def _relres_pin_holds(relres_fn):
    for g, r, p in _relres_cases():
        ref = _dense_relres(g, r, p)
        got = relres_fn(r, p, g)[0]
        if not abs(got - ref) <= _RTOL * ref + _ATOL:
            return False
    return True


def test_relres_matches_explicit_projection_and_dense_residual():
    for g, r, p in _relres_cases():
        ref = _dense_relres(g, r, p)
        got, got_inf = O.relres(r, p, g)
        assert abs(got - ref) <= _RTOL * ref + _ATOL, (got, ref)
        # max-norm companion: same residual, max norms
        A = dense.laplacian_matrix(g)
        v = dense.volume_vector(g)
        rp = np.ravel(r) - (v @ np.ravel(r)) / v.sum()
        res = rp - A @ np.ravel(p)
        assert abs(got_inf - np.abs(res).max() / np.abs(rp).max()) <= _RTOL * got_inf + _ATOL


def _chain_inputs(seed=4):
    g = _tanh_grid(4, 6, 5, lz=1.0)
    r = _rng(seed)
    rho = 1.0 + 999.0 * r.random(g.shape)
    f = r.standard_normal(g.shape)
    p_prev = r.standard_normal(g.shape)
    return g, f, rho, p_prev


def _chain_pin_holds(solve_fn, n_steps=3):
    g, f, rho, p_prev = _chain_inputs()
    for rho0 in (None, 0.8 * float(rho.min())):
        r0 = float(rho.min()) if rho0 is None else rho0
        ref_p, ref_r = _dense_chain(g, f, rho, r0, p_prev, n_steps)
        ps, infos = solve_fn(f, g, rho, p_prev, rho0=rho0, n_steps=n_steps)
        if len(ps) != n_steps:
            return False
        for p, info, pr, rr in zip(ps, infos, ref_p, ref_r):
            if not np.abs(p - pr).max() <= 1e-11 * np.abs(pr).max():
                return False
            if info.rho0_used != r0:
                return False
            if not abs(info.relres - _dense_relres(g, rr, p)) <= 1e-9 * max(info.relres, 1e-16):
                # both residuals sit at rounding level; compare them loosely in absolute terms
                if not (info.relres < 1e-12 and _dense_relres(g, rr, p) < 1e-12):
                    return False
    return True


@pytest.mark.parametrize("n_steps", [1, 3])
def test_chain_matches_dense_method1_steps(n_steps):
    """oracle.solve(..., n_steps=k) equals k dense Method-I steps with
    p_prev <- p and rho0 fixed (given, or min rho)."""
    assert _chain_pin_holds(O.solve, n_steps)


def test_chain_iterates_differ_step_to_step():
    """The chain moves (a frozen iterate would pass a one-step check only)."""
    g, f, rho, p_prev = _chain_inputs()
    ps, _ = O.solve(f, g, rho, p_prev, n_steps=3)
    assert np.abs(ps[2] - ps[1]).max() > 1e-6 * np.abs(ps[2]).max()


# ------------------------------------------------------------ planted slips
def _relres_unprojected(r, p, grid):
    res = r - O.laplacian(p, grid)
    return float(np.linalg.norm(res) / np.linalg.norm(r)), 0.0


def _relres_projected_residual_only(r, p, grid):
    vol = grid.volume_field()
    rp = r - (vol * r).sum() / vol.sum()
    return float(np.linalg.norm(rp - O.laplacian(p, grid)) / np.linalg.norm(r)), 0.0


def _relres_volume_weighted(r, p, grid):
    vol = grid.volume_field()
    rp = r - (vol * r).sum() / vol.sum()
    res = rp - O.laplacian(p, grid)
    return float(np.sqrt((vol * res ** 2).sum() / (vol * rp ** 2).sum())), 0.0


def _relres_plain_mean(r, p, grid):
    rp = r - r.mean()
    return float(np.linalg.norm(rp - O.laplacian(p, grid)) / np.linalg.norm(rp)), 0.0


def _chain_variant(slip):
    def solve(f, grid, rho, p_prev, rho0=None, n_steps=1):
        r0 = float(rho.min()) if (rho0 is None or slip == "rho0_ignored") else rho0
        prev = np.zeros(grid.shape) if slip == "start_from_zero" else p_prev
        ps, infos = [], []
        for s in range(n_steps):
            if slip == "rho0_given_only_first_step" and s > 0:
                r0 = float(rho.min())
            p, r, mean = O.method1_step(f, rho, prev, r0, grid)
            rr = O.relres(f if slip == "relres_of_f" else r, p, grid)
            ps.append(p)
            infos.append(O.SolveInfo(r0, mean, *rr))
            if slip != "prev_not_updated":
                prev = p
        return ps, infos
    return solve


@pytest.mark.parametrize("slip", [_relres_unprojected, _relres_projected_residual_only,
                                  _relres_volume_weighted, _relres_plain_mean])
def test_relres_pin_rejects_planted_slip(slip):
    assert _relres_pin_holds(O.relres)
    assert not _relres_pin_holds(slip)


@pytest.mark.parametrize("slip", ["prev_not_updated", "start_from_zero", "rho0_ignored",
                                  "rho0_given_only_first_step", "relres_of_f"])
def test_chain_pin_rejects_planted_slip(slip):
    assert _chain_pin_holds(_chain_variant(None))
    assert not _chain_pin_holds(_chain_variant(slip))
