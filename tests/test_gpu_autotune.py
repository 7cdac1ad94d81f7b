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
    p_tun, i_tun = gpu.Plan(gm, precision=precision, autotune=1).solve(dev(f), rho=dev(rho),
                                                                        p_prev=dev(pp), info=True)
    e = rel_max_err(host(p_tun), host(p_def))
    lines = cache.read_text().strip().splitlines() if cache.exists() else []
    say(f"{precision}: tuned vs default {e:.2e}, cache entries {lines}")
    assert e <= (1e-12 if precision == "fp64" else 1e-9)
    assert i_tun.relres <= (1e-12 if precision == "fp64" else 1e-10)
    (po,), _ = O.solve(f, g, rho, pp, with_relres=False)
    assert rel_max_err(host(p_tun), po) <= (1e-11 if precision == "fp64" else 1e-8)
