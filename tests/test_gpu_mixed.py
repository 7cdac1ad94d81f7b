"""Mixed-precision refinement driven on the device: without info the sweeps
are enqueued with device-side checks (no host synchronisation), so the solve
can be captured in a HIP graph; every replay must equal the eager solve and
the oracle, and the per-sweep relative residuals reported by info must fall
sweep by sweep to the tolerance."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import dev, host, oracle_inputs, rel_max_err, say

pytestmark = pytest.mark.gpu


def _case(shape, stretched, seed):
    nx, ny, nz = shape
    lz = 2.0 * nz / nx
    spec = W.GridSpec(nx, ny, nz, 1.0, 1.0, lz, W.tanh_faces(nz, lz, 1.5) if stretched else None)
    return W.two_phase_case("mixed_dev", spec, 2, seed, n_spheres=6)


@pytest.mark.parametrize("shape,stretched,n_steps", [((64, 48, 96), True, 1), ((96, 32, 40), False, 3)])
def test_mixed_relres_history(gpu, shape, stretched, n_steps):
    case = _case(shape, stretched, 60 + n_steps)
    g, f, rho, pp = oracle_inputs(case)
    plan = gpu.Plan(gpu.Grid.from_spec(case.grid), precision="mixed")
    p, info = plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp), n_steps=n_steps, info=True)
    hist = info.relres_sweep
    say(f"{shape}: sweeps {info.refine_steps}, relres per sweep {['%.2e' % h for h in hist]}")
    # the history covers the last step of the chain; refine_steps counts every step's sweeps
    assert 2 <= len(hist) <= info.refine_steps + 1
    if n_steps == 1:
        assert len(hist) == info.refine_steps + 1
    assert hist[-1] == info.relres and info.relres <= 1e-10
    assert all(hist[i + 1] < hist[i] for i in range(len(hist) - 1))
    ps, _ = O.solve(f, g, rho, pp, n_steps=n_steps, with_relres=False)
    assert rel_max_err(host(p), ps[-1]) <= 1e-8


def test_mixed_solve_in_a_graph(gpu):
    """psv_solve (mixed, no info) captured once and replayed three times, with
    eager work and synchronisations between the replays: each replay equals
    the eager solve bit for bit and the oracle to the mixed tolerance."""
    case = _case((64, 64, 64), True, 71)
    g, f, rho, pp = oracle_inputs(case)
    plan = gpu.Plan(gpu.Grid.from_spec(case.grid), precision="mixed")
    F, R, P = dev(f), dev(rho), dev(pp)
    ref, info = plan.solve(F, rho=R, p_prev=P, info=True)
    ref = host(ref)
    eager = host(plan.solve(F, rho=R, p_prev=P))  # device-checked sweeps, no info
    assert np.array_equal(eager, ref)
    out = torch.empty_like(F)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.solve(F, rho=R, p_prev=P, out=out)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.solve(F, rho=R, p_prev=P, out=out)
    (po,), _ = O.solve(f, g, rho, pp, with_relres=False)
    for rep in range(3):
        out.fill_(float("nan"))
        junk = torch.rand(512, 512, dtype=torch.float64, device="cuda:0") @ torch.rand(
            512, 512, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = host(out)
        say(f"replay {rep}: equal to eager {np.array_equal(got, ref)}, vs oracle "
            f"{rel_max_err(got, po):.2e}, sweeps {info.refine_steps}")
        assert np.array_equal(got, ref)
        assert rel_max_err(got, po) <= 1e-8
        assert torch.isfinite(junk).all()
    del graph


def test_mixed_spare_sweeps_when_they_run(gpu):
    """With a tolerance no sweep reaches, all max_refine sweeps run on the
    device. The x passes after the first refinement run on a capped grid
    (1024 blocks looping over 2304 tiles here, in line windows). The iterate
    keeps improving: its residual against the oracle's right-hand side, with
    the oracle's operator, ends at the FP64 floor, far below what one sweep
    reaches (a tile left out would leave a residual of order 1)."""
    case = _case((64, 128, 72), True, 83)
    g, f, rho, pp = oracle_inputs(case)
    plan = gpu.Plan(gpu.Grid.from_spec(case.grid), precision="mixed", tol=1e-30, max_refine=4)
    plan.set_shape(lines_x=4, lines_x_inv=4, chunk_rows=8, x_staged=1, x_order=1)
    p = host(plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp)))  # device-checked sweeps
    ps, r, _ = O.method1_step(f, rho, pp, float(rho.min()), g)
    rr, _ = O.relres(r, p, g)
    rr_oracle, _ = O.relres(r, ps, g)
    say(f"4 sweeps on capped grids: relres {rr:.2e} (oracle's own {rr_oracle:.2e}), "
        f"err vs oracle {rel_max_err(p, ps):.2e}")
    assert rr <= max(1e-12, 10 * rr_oracle)
    assert rel_max_err(p, ps) <= 1e-8
