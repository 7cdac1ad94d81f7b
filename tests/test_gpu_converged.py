"""GPU parity of the converged variable-density solve (psv_solve_converged:
the common fixed point of Methods I, II and III, Sec. 3.3.1, Eq. lap_p) and its
implicit adjoint (psv_solve_converged_adjoint) against the FP64 oracle's
pressure-form iterations and adjoint, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import converged as C
import workloads as W
from tests.gpu_util import dev, host, oracle_inputs, rel_max_err, say

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-11

SHAPES = [((24, 18, 20), True), ((32, 32, 24), False), ((16, 48, 13), True), ((64, 1, 40), True)]


def _case(shape, stretched, problem=1):
    nx, ny, nz = shape
    lz = nz / nx
    spec = W.GridSpec(nx, ny, nz, 1.0, 1.0 if ny > 1 else 1.0 / nx, lz,
                      W.tanh_faces(nz, lz, 1.5) if stretched else None)
    case = W.converged_case("conv", spec, problem, n_spheres=4)
    g, f, rho, _ = oracle_inputs(case)
    return spec, g, f, rho, case.w


@pytest.mark.parametrize("iteration", ["method1", "method2", "method3"])
@pytest.mark.parametrize("shape,stretched", SHAPES)
def test_converged_iterates(gpu, shape, stretched, iteration):
    """Fixed iteration counts (eps_t = 0): every iterate at the FP64 tolerance.
    f carries a nonzero mean, which the solve removes."""
    spec, g, f, rho, _ = _case(shape, stretched)
    f = f + 0.37
    plan = gpu.Plan(gpu.Grid.from_spec(spec))
    F, R = dev(f), dev(rho)
    say(f"converged {iteration} {shape} stretched={stretched}")
    for k in (1, 3):
        ref = C.solve(f, rho, g, 0.0, k, iteration)
        p, info = plan.solve_converged(F, R, iteration=iteration, eps_t=0.0, max_iter=k)
        ep = rel_max_err(host(p), ref.p)
        say(f"  k={k}: p {ep:.2e} eps {info.eps:.4e} vs {ref.eps[-1]:.4e}")
        assert info.iterations == k and not info.converged
        assert ep <= TOL_FP64
        assert abs(info.eps - ref.eps[-1]) <= 1e-8 * ref.eps[-1]
        assert abs(info.eps_start - ref.eps[0]) <= 1e-12 * ref.eps[0]


@pytest.mark.parametrize("iteration", ["method1", "method2", "method3"])
def test_converged_solution(gpu, iteration):
    spec, g, f, rho, _ = _case((32, 32, 32), True, 2)
    e0 = np.abs(f).sum()
    eps_t = 1e-11 * e0
    ref = C.solve(f, rho, g, eps_t, 500, iteration)
    assert ref.converged
    plan = gpu.Plan(gpu.Grid.from_spec(spec))
    p, info = plan.solve_converged(dev(f), dev(rho), iteration=iteration, eps_t=eps_t,
                                   max_iter=500)
    say(f"{iteration}: {info.iterations} solves (oracle {len(ref.eps) - 1}), eps {info.eps:.3e}")
    assert info.converged and info.eps <= eps_t
    assert abs(info.iterations - (len(ref.eps) - 1)) <= 1
    assert rel_max_err(host(p), ref.p) <= 1e-8
    # the returned p satisfies the variable-coefficient equation (oracle stencil)
    res = O.operators.var_coeff_operator(host(p), rho, g) - f
    assert np.abs(res).sum() <= 2.0 * eps_t


def test_converged_mixed_and_warm_start(gpu):
    spec, g, f, rho, _ = _case((32, 32, 32), False, 3)
    eps_t = 1e-10 * np.abs(f).sum()
    ref = C.solve(f, rho, g, eps_t, 200)
    plan = gpu.Plan(gpu.Grid.from_spec(spec), precision="mixed")
    p, info = plan.solve_converged(dev(f), dev(rho), eps_t=eps_t, max_iter=200)
    say(f"mixed: {info.iterations} solves (oracle {len(ref.eps) - 1}), eps {info.eps:.3e}")
    assert info.converged and info.iterations <= len(ref.eps) + 3
    assert rel_max_err(host(p), ref.p) <= 1e-7
    # warm start from a converged p: no further solve is needed
    plan64 = gpu.Plan(gpu.Grid.from_spec(spec))
    q = dev(ref.p)
    p2, info2 = plan64.solve_converged(dev(f), dev(rho), eps_t=2 * eps_t, max_iter=5, p_init=q,
                                       out=q)
    assert info2.converged and info2.iterations == 0 and np.isnan(info2.eps_start)
    assert rel_max_err(host(p2), ref.p) == 0.0


@pytest.mark.parametrize("iteration", ["method1", "method2", "method3"])
@pytest.mark.parametrize("shape,stretched", [((24, 18, 20), True), ((32, 32, 24), False),
                                             ((64, 1, 40), True)])
def test_converged_adjoint(gpu, shape, stretched, iteration):
    spec, g, f, rho, w = _case(shape, stretched, 4)
    vol = g.volume_field()
    eps_f = 1e-12 * np.abs(f).sum()
    eps_a = 1e-12 * np.abs(w / vol).sum()
    p_ref = C.solve(f, rho, g, eps_f, 1000, iteration).p
    gf_ref, gr_ref, lam = C.adjoint(w, p_ref, rho, g, eps_a, 1000, iteration)
    assert lam.converged
    plan = gpu.Plan(gpu.Grid.from_spec(spec))
    R = dev(rho)
    p, info = plan.solve_converged(dev(f), R, iteration=iteration, eps_t=eps_f, max_iter=1000)
    assert info.converged
    gf, gr, ainfo = plan.converged_adjoint(dev(w), R, p, iteration=iteration, eps_t=eps_a,
                                           max_iter=1000)
    ef, er = rel_max_err(host(gf), gf_ref), rel_max_err(host(gr), gr_ref)
    say(f"adjoint {iteration} {shape}: {ainfo.iterations} solves, grad_f {ef:.2e} grad_rho {er:.2e}")
    assert ainfo.converged and abs(ainfo.iterations - (len(lam.eps) - 1)) <= 1
    assert ef <= 1e-9 and er <= 1e-9


def test_converged_autograd(gpu):
    """torch.autograd through ConvergedSolve, against the oracle adjoint and a
    central difference of the GPU forward along a random density direction."""
    import paper_2005_11806_amd as psv
    spec, g, f, rho, w = _case((24, 24, 16), True, 5)
    vol = g.volume_field()
    eps_t = 1e-12 * np.abs(f).sum()
    adj_eps = 1e-12 * np.abs(w / vol).sum()
    plan = gpu.Plan(gpu.Grid.from_spec(spec))
    F = dev(f).requires_grad_(True)
    R = dev(rho).requires_grad_(True)
    Wt = dev(w)
    p = psv.converged_solve(F, R, plan, eps_t=eps_t, max_iter=500, adj_eps_t=adj_eps)
    (p * Wt).sum().backward()
    p_ref = C.solve(f, rho, g, eps_t, 500).p
    gf_ref, gr_ref, _ = C.adjoint(w, p_ref, rho, g, adj_eps, 500)
    assert rel_max_err(host(F.grad), gf_ref) <= 1e-9
    assert rel_max_err(host(R.grad), gr_ref) <= 1e-9
    d = W.fd_directions(W.CONFIG_IDS["converged"], 1, g.shape)[0]
    h = 1e-4

    def loss(r):
        q, _ = plan.solve_converged(dev(f), dev(r), eps_t=eps_t, max_iter=500)
        return float((host(q) * w).sum())
    fd = (loss(rho * (1 + h * d)) - loss(rho * (1 - h * d))) / (2 * h)
    an = float((host(R.grad) * rho * d).sum())
    say(f"autograd: directional {an:.10e} fd {fd:.10e}")
    assert abs(an - fd) <= 1e-6 * abs(fd)


def test_converged_input_errors(gpu):
    import paper_2005_11806_amd as psv
    from paper_2005_11806_amd import _abi
    spec, g, f, rho, w = _case((16, 16, 8), False, 6)
    plan = gpu.Plan(gpu.Grid.from_spec(spec))
    F, R = dev(f), dev(rho)
    with pytest.raises(psv.PsvError):
        plan.solve_converged(F, R, max_iter=0)
    with pytest.raises(psv.PsvError):
        plan.solve_converged(F, R, eps_t=-1.0)
    with pytest.raises(psv.PsvError):   # p_out aliasing f
        plan.solve_converged(F, R, out=F)
    lib = psv.lib()
    import ctypes
    out = torch.empty_like(F)
    st = lib.psv_solve_converged(plan._h, ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(R.data_ptr()),
                                 4, 0.0, 3, None, ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), None)
    assert st == _abi.PSV_ERR_INVALID_ARG
    p, _ = plan.solve_converged(F, R, max_iter=2)
    with pytest.raises(psv.PsvError):   # grad_rho without p
        plan.converged_adjoint(dev(w), R, None, max_iter=2)
    with pytest.raises(ValueError):     # iteration from neither method
        plan.converged_adjoint(dev(w), R, p, iteration="method4", max_iter=2)


def test_iteration_counts_rising_bubble(gpu):
    """Methods I, II and III on the rising-bubble-shaped 2-D snapshot at the
    paper's grid (128 x 256, density ratio 10): the GPU counts equal the
    oracle's within one, III < II < I, and all reach one fixed point."""
    case = W.rising_bubble_2d(128, 256)
    g, f, rho, _ = oracle_inputs(case)
    eps_t = 1e-10 * np.abs(f).sum()
    plan = gpu.Plan(gpu.Grid.from_spec(case.grid))
    F, R = dev(f), dev(rho)
    counts, ps = {}, {}
    for it in ("method1", "method2", "method3"):
        ref = C.solve(f, rho, g, eps_t, 1000, it)
        p, info = plan.solve_converged(F, R, iteration=it, eps_t=eps_t, max_iter=1000)
        say(f"{it}: {info.iterations} solves (oracle {len(ref.eps) - 1})")
        assert info.converged and abs(info.iterations - (len(ref.eps) - 1)) <= 1
        counts[it], ps[it] = info.iterations, host(p)
    assert counts["method3"] < counts["method2"] < counts["method1"]
    for it in ("method1", "method2"):
        assert rel_max_err(ps[it], ps["method3"]) <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_converged_direct_stencil(gpu, precision):
    """The converged solve with the forward pass reading its stencil
    neighbours directly (the choice the autotuner makes at 128^3)."""
    spec, g, f, rho, _ = _case((32, 24, 20), True, 7)
    eps_t = 1e-11 * np.abs(f).sum()
    ref = C.solve(f, rho, g, eps_t, 300)
    plan = gpu.Plan(gpu.Grid.from_spec(spec), precision=precision, x_stencil="direct")
    p, info = plan.solve_converged(dev(f), dev(rho), eps_t=eps_t, max_iter=300)
    assert info.converged and abs(info.iterations - (len(ref.eps) - 1)) <= 2
    assert rel_max_err(host(p), ref.p) <= 1e-8
