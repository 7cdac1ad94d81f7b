"""Pins of the converged variable-density solve and its implicit adjoint
(Sec. 3.3.1, Eq. lap_p as the common fixed point of Methods I, II and III), on
the CPU:

* the dense solution satisfies the vectorised stencil D(rho_f^-1 G p) = f_c
  (a second assembly) and has zero volume-weighted mean;
* the three pressure-form iterations (weights min rho, the harmonic mean of
  min and max rho, and rho) reach the dense solution;
* on a rising-bubble-shaped 2-D snapshot (density ratio 10) Method III needs
  fewer iterations than Method II, and Method II fewer than Method I, the
  ordering the paper reports (Sec. 4, rising bubble), all to one fixed point;
* grad_f is the exact Jacobian row of sum(w p) (brute force over unit
  right-hand sides; the map is linear);
* grad_rho matches central differences of sum(w p) in every cell;
* the iterative adjoint equals the dense one."""
import numpy as np
import pytest

import oracle as O
from oracle import converged as C
import workloads as W


def _rng(s=0):
    return np.random.default_rng([47, s])


def _grid(nx, ny, nz, stretched):
    lz = 0.9
    return O.Grid(nx, ny, nz, 1.0, 0.7, lz, W.tanh_faces(nz, lz, 1.5) if stretched else None)


def _density(g, r, ratio):
    """Positive field with max/min ~ ratio: a smooth bump plus noise."""
    x = (np.arange(g.nx) + 0.5) / g.nx
    s = np.cos(2 * np.pi * x)[None, None, :] * np.cos(np.pi * g.zc / g.lz)[:, None, None]
    s = s + 0.5 * r.standard_normal(g.shape)
    s = (s - s.min()) / (s.max() - s.min())
    return np.exp(np.log(ratio) * s)


def _loss(w, f, rho, g):
    return float((w * C.solve_dense(f, rho, g)).sum())


@pytest.mark.parametrize("stretched", [False, True])
def test_dense_solution_satisfies_stencil(stretched):
    g = _grid(5, 4, 6, stretched)
    r = _rng(1)
    rho = _density(g, r, 20.0)
    f = r.standard_normal(g.shape)
    p = C.solve_dense(f, rho, g)
    v = g.volume_field()
    fc = f - (v * f).sum() / v.sum()
    res = O.operators.var_coeff_operator(p, rho, g) - fc
    assert np.abs(res).max() <= 1e-11 * np.abs(fc).max()
    assert abs((v * p).sum()) <= 1e-13 * np.abs(v * p).sum()


@pytest.mark.parametrize("iteration", ["method1", "method2", "method3"])
def test_iterations_reach_dense_solution(iteration):
    g = _grid(6, 4, 8, True)
    r = _rng(2)
    rho = _density(g, r, 10.0)
    f = r.standard_normal(g.shape)
    pd = C.solve_dense(f, rho, g)
    eps_t = 1e-11 * np.abs(f).sum()
    res = C.solve(f, rho, g, eps_t, 2000, iteration)
    assert res.converged
    assert all(b < a for a, b in zip(res.eps[:5], res.eps[1:5]))
    assert np.abs(res.p - pd).max() <= 1e-9 * np.abs(pd).max()


def test_method3_weight_needs_fewer_iterations():
    g = _grid(8, 6, 8, False)
    r = _rng(3)
    rho = _density(g, r, 10.0)
    f = r.standard_normal(g.shape)
    eps_t = 1e-10 * np.abs(f).sum()
    n1 = len(C.solve(f, rho, g, eps_t, 3000, "method1").eps)
    n3 = len(C.solve(f, rho, g, eps_t, 3000, "method3").eps)
    assert n3 < n1


@pytest.mark.parametrize("stretched", [False, True])
def test_grad_f_is_jacobian_row(stretched):
    g = _grid(4, 3, 5, stretched)
    r = _rng(4)
    rho = _density(g, r, 15.0)
    w = r.standard_normal(g.shape)
    f = r.standard_normal(g.shape)
    grad_f, _ = C.adjoint_dense(w, f, rho, g)
    jac = np.empty(g.n)
    for c in range(g.n):
        e = np.zeros(g.n)
        e[c] = 1.0
        jac[c] = _loss(w, e.reshape(g.shape), rho, g)
    assert np.abs(grad_f.ravel() - jac).max() <= 1e-10 * np.abs(jac).max()


@pytest.mark.parametrize("stretched", [False, True])
def test_grad_rho_by_central_differences(stretched):
    g = _grid(4, 3, 5, stretched)
    r = _rng(5)
    rho = _density(g, r, 15.0)
    w = r.standard_normal(g.shape)
    f = r.standard_normal(g.shape)
    _, grad_rho = C.adjoint_dense(w, f, rho, g)
    fd = np.empty(g.n)
    for c in range(g.n):
        d = np.zeros(g.n)
        d[c] = 1e-5 * rho.ravel()[c]
        d = d.reshape(g.shape)
        fd[c] = (_loss(w, f, rho + d, g) - _loss(w, f, rho - d, g)) / (2 * d.ravel()[c])
    assert np.abs(grad_rho.ravel() - fd).max() <= 1e-6 * np.abs(fd).max()


def test_iterative_adjoint_equals_dense():
    g = _grid(6, 5, 7, True)
    r = _rng(6)
    rho = _density(g, r, 10.0)
    w = r.standard_normal(g.shape)
    f = r.standard_normal(g.shape)
    gf_d, gr_d = C.adjoint_dense(w, f, rho, g)
    p = C.solve(f, rho, g, 1e-12 * np.abs(f).sum(), 500).p
    vol = g.volume_field()
    gf, gr, lam = C.adjoint(w, p, rho, g, 1e-12 * np.abs(w / vol).sum(), 500)
    assert lam.converged
    assert np.abs(gf - gf_d).max() <= 1e-9 * np.abs(gf_d).max()
    assert np.abs(gr - gr_d).max() <= 1e-9 * np.abs(gr_d).max()


def test_iteration_ordering_on_rising_bubble_snapshot():
    case = W.rising_bubble_2d(64, 128)
    g = O.Grid.from_spec(case.grid)
    f = O.divergence_of_faces(*case.faces, g)
    rho = O.mixture_density(case.phi, case.rho_gas, case.rho_liq)
    eps_t = 1e-10 * np.abs(f).sum()
    res = {it: C.solve(f, rho, g, eps_t, 1000, it) for it in ("method1", "method2", "method3")}
    n = {it: len(r.eps) - 1 for it, r in res.items()}
    assert all(r.converged for r in res.values())
    assert n["method3"] < n["method2"] < n["method1"]
    ref = res["method3"].p
    for r in res.values():
        assert np.abs(r.p - ref).max() <= 1e-8 * np.abs(ref).max()
