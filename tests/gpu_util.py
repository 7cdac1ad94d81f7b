"""Helpers shared by the GPU tests: host<->device copies and oracle-side input
derivation (f as the discrete divergence, rho from the colour function)."""
import numpy as np
import torch

import oracle as O


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def oracle_inputs(case):
    """(grid, f, rho, p_prev) of a workload case, derived with the oracle's own
    divergence and mixture rule."""
    g = O.Grid.from_spec(case.grid)
    f = O.divergence_of_faces(*case.faces, g)
    if case.extra_rhs is not None:
        f = f + case.extra_rhs
    rho = None if case.phi is None else O.mixture_density(case.phi, case.rho_gas, case.rho_liq)
    return g, f, rho, case.p_prev


def rel_max_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def say(msg):
    print(msg, flush=True)
