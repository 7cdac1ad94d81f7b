"""The plan-free entry point that allocates nothing (psv_solve_static): its
tables and workspace live in one static device array, so it must give the
same result as psv_solve through a plan with built-in shapes, call after call,
whatever the previous call left in the array. Called through the C ABI."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_2005_11806_amd import _abi
from tests.gpu_util import dev, host, oracle_inputs, rel_max_err, say

pytestmark = pytest.mark.gpu


def _static_solve(gpu, grid, f, rho, p_prev, n_steps, method=_abi.PSV_SPLIT_RHO0, rho0=0.0,
                  chunk_rows=0):
    lib = _abi.load()
    g, _keep = grid._c()
    o = _abi.psv_opts()
    lib.psv_opts_default(C.byref(o))
    o.method = method
    o.chunk_rows = chunk_rows
    out = torch.full(grid.shape, np.nan, dtype=torch.float64, device="cuda:0")
    st = lib.psv_solve_static(C.byref(g), C.byref(o), C.c_void_p(f.data_ptr()),
                              C.c_void_p(rho.data_ptr()) if rho is not None else None,
                              float(rho0),
                              C.c_void_p(p_prev.data_ptr()) if p_prev is not None else None,
                              C.c_void_p(out.data_ptr()), int(n_steps),
                              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    _abi.check(st)
    return out


def _case(shape, stretched, seed):
    nx, ny, nz = shape
    lz = nz / nx
    spec = W.GridSpec(nx, ny, nz, 1.0, 1.0, lz, W.tanh_faces(nz, lz, 1.5) if stretched else None)
    return W.two_phase_case(f"static{seed}", spec, 5, seed, n_spheres=4)


def test_static_solve_matches_plan_on_consecutive_calls(gpu):
    """Two calls in a row, the second on a smaller grid (the array still holds
    the first call's tables and spectrum): each equals psv_solve of a plan
    with built-in launch shapes and the FP64 oracle."""
    for shape, stretched, n_steps, seed in (((64, 48, 40), True, 2, 1), ((24, 18, 10), False, 1, 2)):
        case = _case(shape, stretched, seed)
        g, f, rho, pp = oracle_inputs(case)
        grid = gpu.Grid.from_spec(case.grid)
        df, dr, dp = dev(f), dev(rho), dev(pp)
        say(f"static solve {shape} stretched={stretched} steps={n_steps}")
        p_static = _static_solve(gpu, grid, df, dr, dp, n_steps)
        p_plan = gpu.Plan(grid, autotune=0).solve(df, rho=dr, p_prev=dp, n_steps=n_steps)
        a, b = host(p_static), host(p_plan)
        e = rel_max_err(a, b)
        ps, _ = O.solve(f, g, rho, pp, n_steps=n_steps, with_relres=False)
        eo = rel_max_err(a, ps[-1])
        say(f"  vs psv_solve {e:.2e} (bit-identical: {bool(np.array_equal(a, b))}), vs oracle {eo:.2e}")
        assert e <= 1e-14
        assert eo <= 1e-11


def test_static_solve_constant_coefficient_and_given_rho0(gpu):
    """CONST method (rho unused) and an explicit rho0, chunk rows fixed, after
    the calls above have filled the array."""
    case = _case((32, 32, 20), True, 3)
    g, f, rho, pp = oracle_inputs(case)
    grid = gpu.Grid.from_spec(case.grid)
    df, dr, dp = dev(f), dev(rho), dev(pp)
    p_const = _static_solve(gpu, grid, df, None, None, 1, method=_abi.PSV_CONST, chunk_rows=4)
    ref, _ = O.solve_const(f, g)
    assert rel_max_err(host(p_const), ref) <= 1e-11
    r0 = 0.5 * float(rho.min())
    p_r0 = _static_solve(gpu, grid, df, dr, dp, 1, rho0=r0)
    (po,), _ = O.solve(f, g, rho, pp, rho0=r0, with_relres=False)
    assert rel_max_err(host(p_r0), po) <= 1e-11


def test_static_solve_rejects_what_it_cannot_hold(gpu):
    lib = _abi.load()
    o = _abi.psv_opts()
    lib.psv_opts_default(C.byref(o))
    x = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    big, _k = gpu.Grid(256, 256, 256)._c()
    st = lib.psv_solve_static(C.byref(big), C.byref(o), C.c_void_p(x.data_ptr()),
                              C.c_void_p(x.data_ptr()), 0.0, None, C.c_void_p(x.data_ptr()), 1, None)
    assert st == _abi.PSV_ERR_UNSUPPORTED_SIZE
    o.precision = _abi.PSV_MIXED
    small, _k2 = gpu.Grid(16, 16, 8)._c()
    st = lib.psv_solve_static(C.byref(small), C.byref(o), C.c_void_p(x.data_ptr()),
                              C.c_void_p(x.data_ptr()), 0.0, None, C.c_void_p(x.data_ptr()), 1, None)
    assert st == _abi.PSV_ERR_INVALID_ARG
