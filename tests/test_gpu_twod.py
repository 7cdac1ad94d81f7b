"""Two-dimensional x-z problems (ny = 1: one periodic cell in y, so no y
fluxes), the setting of the paper's own test cases (Sec. 4), on its grid
sizes: Method-I chains, mixed refinement and the Method-III loop against the
FP64 oracle through the C ABI."""
import pytest

import oracle as O
from oracle import method3 as M3
import workloads as W
from tests.gpu_util import dev, host, oracle_inputs, rel_max_err, say

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-11


def _spec(nx, nz, lz, stretched):
    return W.GridSpec(nx, 1, nz, 1.0, 1.0 / nx, lz, W.tanh_faces(nz, lz, 1.5) if stretched else None)


@pytest.mark.parametrize("nx,nz,lz,stretched", [(128, 256, 2.0, False), (128, 256, 2.0, True),
                                                 (512, 512, 1.0, False), (16, 128, 8.0, True)])
def test_two_dimensional_method1_chain(gpu, nx, nz, lz, stretched):
    spec = _spec(nx, nz, lz, stretched)
    case = W.two_phase_case("twod", spec, 1, 21, n_spheres=3)
    g, f, rho, pp = oracle_inputs(case)
    say(f"2-D method1 {nx}x{nz} stretched={stretched}")
    plan = gpu.Plan(gpu.Grid.from_spec(spec))
    ps, _ = O.solve(f, g, rho, pp, n_steps=2)
    p, info = plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp), n_steps=2, info=True)
    err = rel_max_err(host(p), ps[1])
    say(f"  err {err:.3e} relres {info.relres:.3e}")
    assert err <= TOL_FP64 and info.relres <= 1e-12


def test_two_dimensional_mixed(gpu):
    spec = _spec(128, 256, 2.0, True)
    case = W.two_phase_case("twod_mixed", spec, 2, 22, n_spheres=3)
    g, f, rho, pp = oracle_inputs(case)
    plan = gpu.Plan(gpu.Grid.from_spec(spec), precision="mixed")
    p, info = plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp), info=True)
    (po,), _ = O.solve(f, g, rho, pp)
    assert info.relres <= 1e-10
    assert rel_max_err(host(p), po) <= 1e-8


def test_two_dimensional_method3(gpu):
    spec = _spec(128, 256, 2.0, False)
    case = W.method3_case("twod_m3", spec, 5, n_spheres=3)
    g = O.Grid.from_spec(spec)
    rho = O.mixture_density(case.base.phi, case.base.rho_gas, case.base.rho_liq)
    faces = case.base.faces
    ref = M3.solve(faces, case.div_target, rho, case.dt, g, eps_t=0.0, max_iter=3)
    plan = gpu.Plan(gpu.Grid.from_spec(spec))
    U = tuple(dev(u) for u in faces)
    p, u, info = plan.solve_method3(U, dev(case.div_target), dev(rho), case.dt, eps_t=0.0,
                                    max_iter=3, u_out=True)
    say(f"2-D method3: p {rel_max_err(host(p), ref.p[2]):.2e} eps {info.eps:.4e} vs {ref.eps[2]:.4e}")
    assert rel_max_err(host(p), ref.p[2]) <= TOL_FP64
    assert max(rel_max_err(host(a), b) for a, b in zip(u, ref.u)) <= TOL_FP64
    assert abs(info.eps - ref.eps[2]) <= 1e-8 * ref.eps[2]


@pytest.mark.parametrize("kc", [4, 8, 16])
@pytest.mark.parametrize("nz,stretched", [(100, True), (13, False), (3, True)])
def test_two_dimensional_ragged_chunks(gpu, kc, nz, stretched):
    """The z passes of ny = 1 problems handle a partial last chunk (nz not a
    multiple of the chunk rows, and nz below them) for every chunk size, FP64
    and mixed, against the oracle."""
    spec = _spec(64, nz, nz / 64, stretched)
    case = W.two_phase_case("twod_ragged", spec, 1, 23 + nz, n_spheres=2)
    g, f, rho, pp = oracle_inputs(case)
    ps, _ = O.solve(f, g, rho, pp, n_steps=2, with_relres=False)
    for precision, tol in (("fp64", TOL_FP64), ("mixed", 1e-8)):
        plan = gpu.Plan(gpu.Grid.from_spec(spec), precision=precision, chunk_rows=kc)
        assert plan.launch_shape()[1] == kc
        p, info = plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp), n_steps=2, info=True)
        err = rel_max_err(host(p), ps[1])
        say(f"2-D ragged nz={nz} kc={kc} {precision}: err {err:.2e} relres {info.relres:.2e}")
        assert err <= tol
        assert info.relres <= (1e-12 if precision == "fp64" else 1e-10)
