"""GPU parity of the FP64 and mixed-precision solves against the FP64 oracle,
through the C ABI.

Tolerances (FP64 path): one step is an exact linear solve; the GPU uses FFTs
(O(log N) rounding growth), the oracle matrix-form DFTs (O(N) growth), so the
two agree to a small multiple of N eps in the max norm relative to max|p|
(N <= 512 here: bound 1e-11). The residual of each step's constant-
coefficient system is gated at relres <= 1e-12 (FP64) and <= 1e-10 (mixed).
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import dev, host, oracle_inputs, rel_max_err, say

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-11


def test_const32_manufactured_and_divergence_rhs(gpu):
    """32^3 constant coefficient: RHS = div(u) + manufactured cos mode."""
    case = W.const32()
    g, f, _, _ = oracle_inputs(case)
    say(f"const32 {g.shape}")
    plan = gpu.Plan(gpu.Grid.from_spec(case.grid), method="const")
    p, info = plan.solve(dev(f), info=True)
    (po,), (oi,) = O.solve(f, g)
    err = rel_max_err(host(p), po)
    say(f"  err {err:.3e} relres {info.relres:.3e} (oracle {oi.relres:.3e})")
    assert err <= TOL_FP64
    assert info.relres <= 1e-12
    assert abs(info.rhs_mean_removed) < 1e-12
    # the manufactured mode alone is an exact eigenvector: p = M / Lambda
    M = case.extra_rhs
    lam = (-4 * np.sin(np.pi * 1 / 32) ** 2 - 4 * np.sin(np.pi * 2 / 32) ** 2
           - 4 * np.sin(np.pi * 3 / 64) ** 2) * 32 ** 2
    pm = host(plan.solve(dev(M)))
    assert rel_max_err(pm, M / lam) <= 1e-13


SHAPES = [
    ((12, 18, 10), True),   # radix 3 in x (M = 6) and y; stretched z
    ((32, 48, 17), False),  # odd nz
    ((96, 64, 24), True),   # 96 = 3 * 32
    ((8, 6, 2), False),     # smallest z
    ((64, 32, 40), True),
    ((1024, 6, 5), True),   # longest x line: one line per block, over 64 KiB of LDS
    ((768, 4, 4), False),   # runtime-length x FFT (M = 384) with over 64 KiB of LDS
]


@pytest.mark.parametrize("shape,stretched", SHAPES)
def test_method1_chain_small(gpu, shape, stretched):
    nx, ny, nz = shape
    lz = 1.3
    spec = W.GridSpec(nx, ny, nz, 1.0, 0.9, lz, W.tanh_faces(nz, lz, 1.5) if stretched else None)
    case = W.two_phase_case("small", spec, 1, 7, n_spheres=4)
    g, f, rho, pp = oracle_inputs(case)
    say(f"method1 {shape} stretched={stretched}")
    plan = gpu.Plan(gpu.Grid.from_spec(spec))
    ps, infos = O.solve(f, g, rho, pp, n_steps=3)
    for s in (1, 2, 3):
        p, info = plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp), n_steps=s, info=True)
        err = rel_max_err(host(p), ps[s - 1])
        say(f"  step {s}: err {err:.3e} relres {info.relres:.3e} rho0 {info.rho0_used}")
        assert err <= TOL_FP64
        assert info.relres <= 1e-12
        assert info.rho0_used == float(rho.min())


def test_method1_constant_density_equals_const_solve(gpu):
    """rho = const makes beta = 0: one step equals S(rho0 f) whatever p_prev."""
    spec = W.GridSpec(16, 24, 12, 1.0, 1.0, 1.0, W.tanh_faces(12, 1.0, 1.5))
    r = np.random.default_rng(3)
    f = r.standard_normal(spec.nz * spec.ny * spec.nx).reshape(12, 24, 16)
    pp = r.standard_normal(f.shape)
    rho = np.full(f.shape, 2.5)
    gm = gpu.Grid.from_spec(spec)
    p1 = host(gpu.Plan(gm).solve(dev(f), rho=dev(rho), p_prev=dev(pp)))
    p2 = host(gpu.Plan(gm, method="const").solve(dev(2.5 * f)))
    assert rel_max_err(p1, p2) <= 1e-13


def test_vd128_ten_step_chain(gpu):
    """128^3, 20 spheres, rho_l = 1000, 10 chained Method-I steps: per-step parity."""
    case = W.vd128()
    g, f, rho, pp = oracle_inputs(case)
    say("vd128 chain")
    plan = gpu.Plan(gpu.Grid.from_spec(case.grid))
    fd, rd, pd = dev(f), dev(rho), dev(pp)
    ps, infos = O.solve(f, g, rho, pp, n_steps=10, with_relres=False)
    for s in (1, 2, 10):
        p, info = plan.solve(fd, rho=rd, p_prev=pd, n_steps=s, info=True)
        err = rel_max_err(host(p), ps[s - 1])
        say(f"  step {s}: err {err:.3e} relres {info.relres:.3e}")
        assert err <= TOL_FP64
        assert info.relres <= 1e-12
    # in-place chaining (p_prev aliases p_out) gives the same iterate
    q = pd.clone()
    plan.solve(fd, rho=rd, p_prev=q, n_steps=10, out=q)
    assert rel_max_err(host(q), ps[9]) <= TOL_FP64


def test_vd128_chain_as_benchmarked(gpu):
    """The 128^3 ten-step chain in the configuration the benchmark times:
    autotuned launch shapes, captured once in a graph and replayed. Every
    replay (with eager work and a synchronisation between replays) matches the
    oracle's tenth iterate element by element."""
    case = W.vd128()
    g, f, rho, pp = oracle_inputs(case)
    ps, _ = O.solve(f, g, rho, pp, n_steps=10, with_relres=False)
    plan = gpu.Plan(gpu.Grid.from_spec(case.grid), autotune=2)
    say(f"vd128 graph replay, launch shape {plan.launch_shape()}")
    fd, rd, pd = dev(f), dev(rho), dev(pp)
    out = torch.empty_like(fd)

    def step():
        plan.solve(fd, rho=rd, p_prev=pd, n_steps=10, out=out)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        err = rel_max_err(host(out), ps[9])
        say(f"  replay {rep}: err {err:.3e}")
        assert err <= TOL_FP64
    del graph


@pytest.mark.parametrize("shape", [(64, 64, 128), (96, 48, 64)])
def test_mixed_refinement_small(gpu, shape):
    nx, ny, nz = shape
    spec = W.GridSpec(nx, ny, nz, 1.0, 1.0, 2.0, W.tanh_faces(nz, 2.0, 1.5))
    case = W.two_phase_case("mixed_small", spec, 2, 5, n_spheres=30)
    g, f, rho, pp = oracle_inputs(case)
    say(f"mixed {shape}")
    plan = gpu.Plan(gpu.Grid.from_spec(spec), precision="mixed", tol=1e-10)
    p, info = plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp), info=True)
    (po,), (oi,) = O.solve(f, g, rho, pp)
    err = rel_max_err(host(p), po)
    rr = O.relres(O.assemble_method1(f, rho, pp, float(rho.min()), g), host(p), g)[0]
    say(f"  err {err:.3e} relres {info.relres:.3e} (host recheck {rr:.3e}) steps {info.refine_steps}")
    assert info.relres <= 1e-10
    assert rr <= 1e-10
    assert 1 <= info.refine_steps <= 3
    assert err <= 1e-8


# Every chunk size of the wall-normal partition against the oracle: ragged
# last chunks (nz not a multiple of kc), a single chunk shorter than kc,
# three planes only, and runtime-length y FFTs (ny = 18, 6).
KC_SHAPES = [
    ((32, 48, 17), False),
    ((12, 18, 10), True),
    ((64, 32, 40), True),
    ((16, 64, 3), False),
    ((8, 6, 9), True),
]


@pytest.mark.parametrize("kc", [4, 8, 16])
@pytest.mark.parametrize("shape,stretched", KC_SHAPES)
def test_chunk_rows_fp64(gpu, kc, shape, stretched):
    nx, ny, nz = shape
    spec = W.GridSpec(nx, ny, nz, 1.0, 0.9, 1.1, W.tanh_faces(nz, 1.1, 1.5) if stretched else None)
    case = W.two_phase_case("chunks", spec, 1, 11, n_spheres=3)
    g, f, rho, pp = oracle_inputs(case)
    say(f"chunk rows {kc} {shape} stretched={stretched}")
    plan = gpu.Plan(gpu.Grid.from_spec(spec), chunk_rows=kc)
    assert plan.launch_shape()[1] == kc
    ps, _ = O.solve(f, g, rho, pp, n_steps=2)
    p, info = plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp), n_steps=2, info=True)
    err = rel_max_err(host(p), ps[1])
    say(f"  err {err:.3e} relres {info.relres:.3e}")
    assert err <= TOL_FP64
    assert info.relres <= 1e-12


# The interface systems (2 ceil(nz/kc) rows per pair) are spread over up to 64
# lanes with 2, 4 or 16 register rows each; long columns reach every layout
# (rows 38, 200, 516, 512 and 1024).
@pytest.mark.parametrize("shape,kc,stretched", [((8, 8, 300), 16, True), ((8, 8, 400), 4, False),
                                                ((8, 6, 1030), 4, True), ((8, 4, 2048), 8, False),
                                                ((4, 4, 2048), 4, True)])
def test_interface_lane_layouts(gpu, shape, kc, stretched):
    nx, ny, nz = shape
    lz = nz / 64.0
    spec = W.GridSpec(nx, ny, nz, 1.0, 0.9, lz, W.tanh_faces(nz, lz, 1.5) if stretched else None)
    case = W.two_phase_case("lanes", spec, 1, 13, n_spheres=3)
    g, f, rho, pp = oracle_inputs(case)
    say(f"interface lanes {shape} kc={kc} stretched={stretched}")
    plan = gpu.Plan(gpu.Grid.from_spec(spec), chunk_rows=kc)
    ps, _ = O.solve(f, g, rho, pp, n_steps=2)
    p, info = plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp), n_steps=2, info=True)
    err = rel_max_err(host(p), ps[1])
    say(f"  err {err:.3e} relres {info.relres:.3e}")
    assert err <= TOL_FP64
    assert info.relres <= 1e-12


@pytest.mark.parametrize("kc", [4, 8, 16])
def test_chunk_rows_mixed(gpu, kc):
    spec = W.GridSpec(48, 32, 37, 1.0, 1.0, 1.5, W.tanh_faces(37, 1.5, 1.5))
    case = W.two_phase_case("chunks_mixed", spec, 2, 12, n_spheres=6)
    g, f, rho, pp = oracle_inputs(case)
    say(f"mixed chunk rows {kc}")
    plan = gpu.Plan(gpu.Grid.from_spec(spec), precision="mixed", chunk_rows=kc)
    p, info = plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp), info=True)
    (po,), _ = O.solve(f, g, rho, pp)
    err = rel_max_err(host(p), po)
    say(f"  err {err:.3e} relres {info.relres:.3e} steps {info.refine_steps}")
    assert info.relres <= 1e-10
    assert err <= 1e-8


def test_density_and_divergence_kernels(gpu):
    spec = W.GridSpec(24, 16, 10, 1.0, 1.0, 1.0, W.tanh_faces(10, 1.0, 1.5))
    case = W.two_phase_case("aux", spec, 1, 3, n_spheres=5)
    g = O.Grid.from_spec(spec)
    plan = gpu.Plan(gpu.Grid.from_spec(spec))
    rho = host(plan.density_from_colour(dev(case.phi), dev(case.rho_gas), case.rho_liq))
    assert rel_max_err(rho, O.mixture_density(case.phi, case.rho_gas, case.rho_liq)) <= 1e-15
    div = host(plan.divergence(*(dev(u) for u in case.faces)))
    ref = O.divergence_of_faces(*case.faces, g)
    assert np.abs(div - ref).max() <= 1e-13 * np.abs(ref).max()


def test_input_checks(gpu):
    import paper_2005_11806_amd as psv
    spec = W.uniform_grid(8, 8, 8)
    plan = gpu.Plan(gpu.Grid.from_spec(spec), check_inputs=True)
    f = np.zeros(spec.nz * 64).reshape(8, 8, 8)
    rho = np.ones_like(f)
    f_bad = f.copy()
    f_bad[3, 2, 1] = np.nan
    with pytest.raises(psv.PsvError) as e:
        plan.solve(dev(f_bad), rho=dev(rho))
    assert e.value.status == psv._abi.PSV_ERR_NONFINITE
    r_bad = rho.copy()
    r_bad[0, 0, 0] = -1.0
    with pytest.raises(psv.PsvError) as e:
        plan.solve(dev(f), rho=dev(r_bad))
    assert e.value.status == psv._abi.PSV_ERR_INVALID_ARG
    with pytest.raises(psv.PsvError) as e:
        plan.solve(dev(f), rho=dev(rho), rho0=2.0)
    assert e.value.status == psv._abi.PSV_ERR_INVALID_ARG
    plan.solve(dev(f), rho=dev(rho))  # valid inputs still pass


def test_misaligned_field_pointers_rejected(gpu):
    """Contiguous views at an 8-byte offset are refused before any launch."""
    import torch
    import paper_2005_11806_amd as psv
    spec = W.uniform_grid(8, 8, 8)
    plan = gpu.Plan(gpu.Grid.from_spec(spec))
    base = torch.zeros(8 * 64 + 1, dtype=torch.float64, device="cuda")
    odd = base[1:].view(8, 8, 8)
    rho = dev(np.ones((8, 8, 8)))
    for call in (lambda: plan.solve(odd, rho=rho),
                 lambda: plan.solve(rho, rho=odd),
                 lambda: plan.solve(rho, rho=rho, out=odd),
                 lambda: plan.adjoint(odd, rho=rho, p_prev=rho),
                 lambda: plan.solve_converged(odd, rho, max_iter=1)):
        with pytest.raises(psv.PsvError) as e:
            call()
        assert e.value.status == psv._abi.PSV_ERR_INVALID_ARG
    p = plan.solve(rho, rho=rho)  # aligned inputs still pass
    assert np.isfinite(host(p)).all()


# The forward x pass reads its stencil neighbours either from rows staged in
# LDS or directly from global memory; both against the oracle, including
# periodic wrap in x and y, ny = 1, stretched z, runtime-length and 1024-point
# lines and the FP64 residual of the mixed refinement. Without staging the x
# neighbours come by lane exchange for half-lengths 16, 32, 64 (groups of
# lanes, one line per group), 128 and 512 (64 pairs of a line per wave, edge
# lanes load theirs) and by loads for 48 and the runtime lengths. The FP64
# staged rows, bins and twiddles of compile-time lengths arrive by
# direct-to-LDS loads in 64-entry chunks: half-lengths 48, 96 and 192 end
# each row with a partial chunk.
@pytest.mark.parametrize("shape,stretched", [((12, 18, 10), True), ((32, 48, 17), False),
                                             ((64, 1, 40), True), ((1024, 6, 5), True),
                                             ((8, 6, 2), False), ((128, 4, 6), True),
                                             ((256, 6, 5), False), ((96, 6, 5), True),
                                             ((192, 6, 7), True), ((384, 6, 4), False)])
@pytest.mark.parametrize("x_stencil", ["staged", "direct"])
def test_x_stencil_variants(gpu, shape, stretched, x_stencil):
    nx, ny, nz = shape
    lz = 1.3
    spec = W.GridSpec(nx, ny, nz, 1.0, 0.9 if ny > 1 else 1.0 / nx, lz,
                      W.tanh_faces(nz, lz, 1.5) if stretched else None)
    case = W.two_phase_case("xst", spec, 1, 8, n_spheres=4)
    g, f, rho, pp = oracle_inputs(case)
    say(f"x stencil {x_stencil} {shape} stretched={stretched}")
    ps, _ = O.solve(f, g, rho, pp, n_steps=2)
    plan = gpu.Plan(gpu.Grid.from_spec(spec), x_stencil=x_stencil)
    p, info = plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp), n_steps=2, info=True)
    assert rel_max_err(host(p), ps[1]) <= TOL_FP64 and info.relres <= 1e-12
    mixed = gpu.Plan(gpu.Grid.from_spec(spec), precision="mixed", x_stencil=x_stencil)
    p, info = mixed.solve(dev(f), rho=dev(rho), p_prev=dev(pp), info=True)
    assert info.relres <= 1e-10 and rel_max_err(host(p), ps[0]) <= 1e-8


# Forward x tile orders over the XCDs: line windows (each XCD takes 1/8 of
# every plane's tiles, plane after plane) and contiguous plane ranges. Only
# the block-to-tile map differs, so the two must agree bit for bit; a tile
# visited twice or never would not. 16 and 24 tiles per plane use windows
# (2 and 3 tiles each); 12 fall back to plane ranges.
@pytest.mark.parametrize("shape,lines", [((64, 64, 24), 4), ((32, 96, 20), 4), ((64, 48, 9), 4)])
def test_x_tile_orders_agree(gpu, shape, lines):
    nx, ny, nz = shape
    spec = W.GridSpec(nx, ny, nz, 1.0, 1.0, 0.8, W.tanh_faces(nz, 0.8, 1.5))
    case = W.two_phase_case("xorder", spec, 1, 12, n_spheres=4)
    g, f, rho, pp = oracle_inputs(case)
    say(f"x tile orders {shape}, {ny // lines} tiles per plane")
    out = {}
    for prec in ("fp64", "mixed"):
        plan = gpu.Plan(gpu.Grid.from_spec(spec), precision=prec)
        for order in (1, 0):
            plan.set_shape(lines_x=lines, lines_x_inv=lines, chunk_rows=4, x_staged=1, x_order=order)
            out[prec, order] = host(plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp)))
        assert np.array_equal(out[prec, 0], out[prec, 1])
    ps, _ = O.solve(f, g, rho, pp, with_relres=False)
    assert rel_max_err(out["fp64", 1], ps[0]) <= TOL_FP64
