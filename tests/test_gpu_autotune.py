"""Autotuned launch shapes: the tuned plan solves to the same result as the
default one, and the choice is cached (in-process and in PSV_AUTOTUNE_CACHE)."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import dev, host, oracle_inputs, rel_max_err, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotuned_plan_matches_default(gpu, precision, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PSV_AUTOTUNE_CACHE", str(cache))
    spec = W.GridSpec(48, 64, 40, 1.0, 1.0, 1.0, W.tanh_faces(40, 1.0, 1.5))
    case = W.two_phase_case("tune", spec, 1, 77, n_spheres=5)
    g, f, rho, pp = oracle_inputs(case)
    gm = gpu.Grid.from_spec(spec)
    p_def, i_def = gpu.Plan(gm, precision=precision).solve(dev(f), rho=dev(rho), p_prev=dev(pp), info=True)
    p_tun, i_tun = gpu.Plan(gm, precision=precision, autotune=2).solve(dev(f), rho=dev(rho),
                                                                        p_prev=dev(pp), info=True)
    e = rel_max_err(host(p_tun), host(p_def))
    lines = cache.read_text().strip().splitlines() if cache.exists() else []
    say(f"{precision}: tuned vs default {e:.2e}, cache entries {lines}")
    assert e <= (1e-12 if precision == "fp64" else 1e-9)
    assert i_tun.relres <= (1e-12 if precision == "fp64" else 1e-10)
    (po,), _ = O.solve(f, g, rho, pp, with_relres=False)
    assert rel_max_err(host(p_tun), po) <= (1e-11 if precision == "fp64" else 1e-8)


def test_cache_entries_of_every_format(tmp_path):
    """Cache lines written with 3 to 6 fields (lines per block, chunk rows,
    then optionally the inverse pass's lines per block, the stencil choice
    and the forward tile order) are all honoured; a fresh process reads
    them. Missing choices take the built-in ones (staged rows, line windows)."""
    import json
    import subprocess
    import sys
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{arch}:32x32x24:fp64:method1 2 4\n"
                     f"{arch}:48x32x24:fp64:method1 4 8 2\n"
                     f"{arch}:64x32x24:fp64:method1 8 4 2 0\n"
                     f"{arch}:96x32x24:fp64:method1 4 8 2 1 0\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = (
        "import json, sys\n"
        f"sys.path.insert(0, {root!r})\n"
        "import paper_2005_11806_amd as psv\n"
        "out = {}\n"
        "for nx in (32, 48, 64, 96):\n"
        "    plan = psv.Plan(psv.Grid(nx, 32, 24, 1.0, 1.0, 1.0), autotune=1)\n"
        "    out[nx] = plan.get_shape()\n"
        "print(json.dumps(out))\n")
    env = dict(os.environ, PSV_AUTOTUNE_CACHE=str(cache))
    res = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True,
                         timeout=240)
    assert res.returncode == 0, res.stderr[-2000:]
    shapes = json.loads(res.stdout.strip().splitlines()[-1])
    say(f"cached shapes {shapes}")
    def sh(lx, kc, li, st, order):
        return {"lines_x": lx, "lines_x_inv": li, "chunk_rows": kc, "x_staged": st, "x_order": order}
    assert shapes == {"32": sh(2, 4, 2, 1, 1), "48": sh(4, 8, 2, 1, 1), "64": sh(8, 4, 2, 0, 1),
                      "96": sh(4, 8, 2, 1, 0)}


def test_cache_only_mode_never_times(gpu, tmp_path, monkeypatch):
    """autotune = 1 looks the plan up in the cache and otherwise keeps the
    built-in shapes without timing anything (no cache entry appears);
    autotune = 2 tunes and adds the entry, which a later autotune = 1 plan of
    the same key then uses."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PSV_AUTOTUNE_CACHE", str(cache))
    gm = gpu.Grid(64, 48, 36, 1.0, 1.0, 36 / 64)
    base = gpu.Plan(gm, autotune=0).launch_shape()
    only = gpu.Plan(gm, autotune=1).launch_shape()
    assert only == base
    assert not cache.exists() or cache.read_text().strip() == ""
    tuned = gpu.Plan(gm, autotune=2).launch_shape()
    lines = cache.read_text().strip().splitlines()
    say(f"built-in {base}, tuned {tuned}, cache {lines}")
    assert len(lines) == 1 and ":64x48x36:fp64:method1 " in lines[0]
    assert gpu.Plan(gm, autotune=1).launch_shape() == tuned


def test_shape_api_round_trip_and_checks(gpu):
    """psv_plan_get_shape / psv_plan_set_shape: every field round-trips, a
    shape set by hand solves like the built-in one, bad fields are rejected
    and leave the plan as it was."""
    spec = W.GridSpec(64, 32, 16, 1.0, 1.0, 0.5, W.tanh_faces(16, 0.5, 1.5))
    case = W.two_phase_case("shape", spec, 1, 78, n_spheres=3)
    g, f, rho, pp = oracle_inputs(case)
    plan = gpu.Plan(gpu.Grid.from_spec(spec))
    ref = host(plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp)))
    plan.set_shape(lines_x=8, lines_x_inv=4, chunk_rows=4, x_staged=0, x_order=0)
    assert plan.get_shape() == {"lines_x": 8, "lines_x_inv": 4, "chunk_rows": 4, "x_staged": 0,
                                "x_order": 0}
    assert plan.launch_shape() == (8, 4)
    p = host(plan.solve(dev(f), rho=dev(rho), p_prev=dev(pp)))
    assert rel_max_err(p, ref) <= 1e-12
    for bad in ({"lines_x": 3}, {"lines_x_inv": 0}, {"chunk_rows": 5}, {"x_staged": 2},
                {"x_order": -1}):
        with pytest.raises(gpu.PsvError):
            plan.set_shape(**bad)
    assert plan.get_shape()["lines_x"] == 8  # a rejected call changes nothing
