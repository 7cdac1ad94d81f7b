"""Batched uneven solves (psv_batch_*) against standalone solves and the FP64
oracle: every problem of the batch must match its own single solve at the
same precision and the oracle to the path's tolerance, on graph replays."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import dev, host, oracle_inputs, rel_max_err, say

pytestmark = pytest.mark.gpu

SMALL = [((16, 12, 10), True), ((32, 32, 16), False), ((24, 18, 33), True), ((12, 48, 8), False),
         ((64, 32, 24), True), ((8, 6, 3), False)]


def _cases(shapes, seed0=20):
    out = []
    for i, (shape, stretched) in enumerate(shapes):
        nx, ny, nz = shape
        lz = nz / nx
        spec = W.GridSpec(nx, ny, nz, 1.0, 1.0, lz, W.tanh_faces(nz, lz, 1.5) if stretched else None)
        out.append(W.two_phase_case(f"b{i}", spec, 3, seed0 + i, n_spheres=3))
    return out


@pytest.mark.parametrize("executor", ["passes", "persistent"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("mixed", 1e-8)])
def test_small_uneven_batch(gpu, precision, tol, executor):
    cases = _cases(SMALL)
    ins = [oracle_inputs(c) for c in cases]
    grids = [gpu.Grid.from_spec(c.grid) for c in cases]
    say(f"executor {executor}")
    batch = gpu.Batch(grids, precision=precision, executor=executor)
    fs = [dev(x[1]) for x in ins]
    rs = [dev(x[2]) for x in ins]
    ps = [dev(x[3]) for x in ins]
    for rep in range(3):  # first call captures the graph, later calls replay it
        outs, infos = batch.solve(fs, rs, ps, info=True)
        for i, (g, f, rho, pp) in enumerate(ins):
            single = gpu.Plan(grids[i], precision=precision).solve(fs[i], rho=rs[i], p_prev=ps[i])
            (po,), _ = O.solve(f, g, rho, pp, with_relres=False)
            e1 = rel_max_err(host(outs[i]), host(single))
            e2 = rel_max_err(host(outs[i]), po)
            if rep == 0:
                say(f"{precision} problem {i} {g.shape}: vs single {e1:.2e}, vs oracle {e2:.2e}, "
                    f"relres {infos[i].relres:.2e} steps {infos[i].refine_steps}")
            assert e2 <= tol, (i, e2)
            assert e1 <= (1e-12 if precision == "fp64" else 1e-8), (i, e1)
            assert infos[i].relres <= (1e-12 if precision == "fp64" else 1e-10)
            assert infos[i].rho0_used == float(rho.min())


@pytest.mark.parametrize("executor,kc", [("passes", 4), ("passes", 8), ("persistent", 4)])
def test_small_uneven_batch_chunk_rows(gpu, executor, kc):
    """Fixed chunk rows of the wall-normal partition in every problem of the
    batch (ragged last chunks included), FP64 against the oracle."""
    cases = _cases(SMALL, seed0=60)
    ins = [oracle_inputs(c) for c in cases]
    grids = [gpu.Grid.from_spec(c.grid) for c in cases]
    say(f"executor {executor} chunk rows {kc}")
    batch = gpu.Batch(grids, precision="fp64", executor=executor, chunk_rows=kc)
    outs, infos = batch.solve([dev(x[1]) for x in ins], [dev(x[2]) for x in ins],
                              [dev(x[3]) for x in ins], info=True)
    for i, (g, f, rho, pp) in enumerate(ins):
        (po,), _ = O.solve(f, g, rho, pp, with_relres=False)
        e = rel_max_err(host(outs[i]), po)
        assert e <= 1e-11, (i, e)
        assert infos[i].relres <= 1e-12


def test_batch_explicit_rho0_and_const(gpu):
    cases = _cases(SMALL[:3], seed0=40)
    ins = [oracle_inputs(c) for c in cases]
    grids = [gpu.Grid.from_spec(c.grid) for c in cases]
    rho0s = [0.5 * float(x[2].min()) for x in ins]
    b = gpu.Batch(grids, precision="fp64")
    outs = b.solve([dev(x[1]) for x in ins], [dev(x[2]) for x in ins], [dev(x[3]) for x in ins],
                   rho0s=rho0s)
    for i, (g, f, rho, pp) in enumerate(ins):
        (po,), _ = O.solve(f, g, rho, pp, rho0=rho0s[i], with_relres=False)
        assert rel_max_err(host(outs[i]), po) <= 1e-11
    bc = gpu.Batch(grids, precision="fp64", method="const")
    outs = bc.solve([dev(x[1]) for x in ins])
    for i, (g, f, rho, pp) in enumerate(ins):
        assert rel_max_err(host(outs[i]), O.solve_const(f, g)[0]) <= 1e-11


@pytest.mark.parametrize("executor", ["passes", "persistent"])
def test_batch64_uneven_mixed(gpu, executor):
    """64 problems drawn from {64^3, 96x96x128, 128^3, 128x128x192}, mixed
    precision: each matches its standalone mixed solve; a sample of 6 matches
    the FP64 oracle."""
    cases = W.batch()
    grids = [gpu.Grid.from_spec(c.grid) for c in cases]
    say(f"batch of {len(cases)}: " + ", ".join(f"{c.grid.nx}x{c.grid.ny}x{c.grid.nz}" for c in cases[:8]) + " ...")
    ins = []
    for c in cases:
        g = O.Grid.from_spec(c.grid)
        f = O.divergence_of_faces(*c.faces, g)
        rho = O.mixture_density(c.phi, c.rho_gas, c.rho_liq)
        ins.append((g, f, rho, c.p_prev))
    fs = [dev(x[1]) for x in ins]
    rs = [dev(x[2]) for x in ins]
    ps = [dev(x[3]) for x in ins]
    batch = gpu.Batch(grids, precision="mixed", executor=executor)
    say(f"executor {executor}")
    outs, infos = batch.solve(fs, rs, ps, info=True)
    outs, infos = batch.solve(fs, rs, ps, info=True)  # replay
    assert max(i.relres for i in infos) <= 1e-10
    say(f"  max relres {max(i.relres for i in infos):.2e}, steps {sorted(set(i.refine_steps for i in infos))}")
    for i in range(len(cases)):
        single = gpu.Plan(grids[i], precision="mixed").solve(fs[i], rho=rs[i], p_prev=ps[i])
        assert rel_max_err(host(outs[i]), host(single)) <= 1e-8, i
    sizes = np.array([c.grid.n for c in cases])
    sample = sorted(set([int(np.argmin(sizes)), int(np.argmax(sizes))] + list(range(0, 64, 16))))
    for i in sample:
        g, f, rho, pp = ins[i]
        (po,), _ = O.solve(f, g, rho, pp, with_relres=False)
        e = rel_max_err(host(outs[i]), po)
        say(f"  problem {i} {g.shape}: vs oracle {e:.2e}")
        assert e <= 1e-8


@pytest.mark.parametrize("executor", ["passes", "persistent"])
def test_calls_queued_back_to_back_keep_their_buffers(gpu, executor):
    """Two calls queued behind long work on the stream, each with its own
    inputs and outputs: the second call rewrites the host pointer table only
    after the first call's copy of it has run, so each call solves its own
    problems."""
    ins_a = [oracle_inputs(c) for c in _cases(SMALL[:3], seed0=80)]
    ins_b = [oracle_inputs(c) for c in _cases(SMALL[:3], seed0=90)]
    grids = [gpu.Grid.from_spec(c.grid) for c in _cases(SMALL[:3], seed0=80)]
    b = gpu.Batch(grids, precision="fp64", executor=executor)
    fa, ra, pa = ([dev(x[j]) for x in ins_a] for j in (1, 2, 3))
    fb, rb, pb = ([dev(x[j]) for x in ins_b] for j in (1, 2, 3))
    b.solve(fa, ra, pa)  # captures the graph
    torch.cuda.synchronize()
    x = torch.rand(2048, 2048, dtype=torch.float64, device="cuda:0") / 2048
    y = x
    for _ in range(8):  # milliseconds of work ahead of the two calls
        y = y @ x
    outs_a = b.solve(fa, ra, pa)
    outs_b = b.solve(fb, rb, pb)
    torch.cuda.synchronize()
    assert torch.isfinite(y).all()
    for ins, outs, tag in ((ins_a, outs_a, "first"), (ins_b, outs_b, "second")):
        for i, (g, f, rho, pp) in enumerate(ins):
            (po,), _ = O.solve(f, g, rho, pp, with_relres=False)
            e = rel_max_err(host(outs[i]), po)
            say(f"{executor} {tag} call, problem {i}: vs oracle {e:.2e}")
            assert e <= 1e-11, (tag, i, e)


@pytest.mark.parametrize("x_stencil", ["staged", "direct"])
def test_small_batch_each_stencil_variant(gpu, x_stencil):
    """Every problem's forward x tiles in the given stencil variant (the batch
    launches one pass per variant in use), FP64 and mixed, against the
    oracle."""
    cases = _cases(SMALL, seed0=110)
    ins = [oracle_inputs(c) for c in cases]
    grids = [gpu.Grid.from_spec(c.grid) for c in cases]
    for precision, tol in (("fp64", 1e-11), ("mixed", 1e-8)):
        b = gpu.Batch(grids, precision=precision, x_stencil=x_stencil)
        outs, infos = b.solve([dev(x[1]) for x in ins], [dev(x[2]) for x in ins],
                              [dev(x[3]) for x in ins], info=True)
        for i, (g, f, rho, pp) in enumerate(ins):
            (po,), _ = O.solve(f, g, rho, pp, with_relres=False)
            e = rel_max_err(host(outs[i]), po)
            say(f"{x_stencil} {precision} problem {i} {g.shape}: vs oracle {e:.2e}")
            assert e <= tol, (i, e)
            assert infos[i].relres <= (1e-12 if precision == "fp64" else 1e-10)


@pytest.mark.parametrize("executor", ["passes", "persistent"])
def test_batch64_autotuned(gpu, executor, tmp_path, monkeypatch):
    """The 64-problem batch with every problem's launch shapes tuned
    (autotune = 2: lines per forward and inverse x block, chunk rows and the
    stencil variant of its grid): each problem matches the batch in built-in
    shapes, a sample matches the FP64 oracle, and the shapes the batch ran
    with are the ones a plan of the same grid reads back from the cache."""
    monkeypatch.setenv("PSV_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    cases = W.batch()
    grids = [gpu.Grid.from_spec(c.grid) for c in cases]
    ins = []
    for c in cases:
        g = O.Grid.from_spec(c.grid)
        ins.append((g, O.divergence_of_faces(*c.faces, g),
                    O.mixture_density(c.phi, c.rho_gas, c.rho_liq), c.p_prev))
    fs, rs, ps = ([dev(x[j]) for x in ins] for j in (1, 2, 3))
    tuned = gpu.Batch(grids, precision="mixed", executor=executor, autotune=2)
    plain = gpu.Batch(grids, precision="mixed", executor=executor, autotune=0)
    outs, infos = tuned.solve(fs, rs, ps, info=True)
    outs, infos = tuned.solve(fs, rs, ps, info=True)  # replay
    ref, _ = plain.solve(fs, rs, ps, info=True)
    # the grids tuned earlier in this process come from its in-process cache
    # and add no line to the file
    cache = tmp_path / "tune.txt"
    lines = cache.read_text().strip().splitlines() if cache.exists() else []
    say(f"{executor}: tuned shapes {lines}")
    assert len(lines) <= len({(g.nx, g.ny, g.nz) for g in grids})
    shapes = {(g.nx, g.ny, g.nz): gpu.Plan(g, precision="mixed", autotune=1).launch_shape()
              for g in grids}
    say(f"  (lines per x block, chunk rows) per grid: {shapes}")
    assert max(i.relres for i in infos) <= 1e-10
    for i in range(len(cases)):
        assert rel_max_err(host(outs[i]), host(ref[i])) <= 1e-8, i
    sizes = np.array([c.grid.n for c in cases])
    sample = sorted(set([int(np.argmin(sizes)), int(np.argmax(sizes)), 5, 37]))
    for i in sample:
        g, f, rho, pp = ins[i]
        (po,), _ = O.solve(f, g, rho, pp, with_relres=False)
        e = rel_max_err(host(outs[i]), po)
        say(f"  problem {i} {g.shape}: vs oracle {e:.2e}")
        assert e <= 1e-8
