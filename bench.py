#!/usr/bin/env python3
"""Throughput of the eigenexpansion pressure solve on one MI355X.

Default workload (c3_fp64): one Method-I pressure solve per step on the
256x256x512 grid with tanh-stretched z (alpha 1.5), periodic x/y, walls in z,
two-phase density (200 smoothed spheres, liquid 1000, gas 1-5), rho0 =
min(rho) computed on the device, FP64, replayed from a captured HIP graph.
`value` counts grid points solved per second. The same JSON line carries the
comparisons the metric asks for, each at relres <= 1e-10 and with its error
against the FP64 oracle:

* mixed_c3: the same problem with FP32 transforms and tridiagonal sweeps and
  FP64 residual refinement;
* batched_c4: 64 uneven problems from {64^3, 96x96x128, 128^3, 128x128x192},
  solved one plan at a time in FP64, and as one batch (per-pass batched
  launches or one persistent launch, FP64 or mixed);
* iterated_128: the converged variable-density solve on 128^3 (Method III
  weights) where each iteration is an eigenexpansion solve, FP64 against FP32
  solves inside the same loop.

    python bench.py [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line. Inputs are generated on the host (seeded), copied to
the device and turned into f (discrete divergence) and rho (mixture rule) by
the library before timing starts; the timed regions hold only solves.

The roofline object describes the kernel with the largest share of the
headline solve's GPU time, measured with HIP events around each of its
launches (psv_trace_*) in an eager pass of the same K steps on the launch
stream. The CPU baseline is the FP64 oracle on the same grid and inputs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pressure-solve grid pts/s + HBM GB/s % peak; mixed/batched vs FP64 GPU at fixed residual"
HBM_PEAK_GBS = 8000.0
COPY_PROBE_BYTES = 256 << 20

WORKLOADS = {
    "vd128": dict(desc="128^3 uniform, Method I (rho0=min rho), 20 spheres, rho_l=1000, rho_g=1-5, "
                       "10 chained solves per step", precision="fp64", n_steps=10),
    "mixed_tanh": dict(desc="256x256x512 tanh-stretched z (alpha 1.5), Method I, 200 spheres, "
                            "FP32 bulk + FP64 refinement to relres 1e-10", precision="mixed", n_steps=1),
    "fp64_tanh": dict(desc="256x256x512 tanh-stretched z (alpha 1.5), Method I, 200 spheres, FP64",
                      precision="fp64", n_steps=1),
    "const32": dict(desc="32^3 uniform constant-coefficient solve, RHS = div(u) + cos mode",
                    precision="fp64", n_steps=1),
}


def make_case(name):
    import workloads as W
    if name == "vd128":
        return W.vd128()
    if name in ("mixed_tanh", "fp64_tanh"):
        return W.mixed_tanh()
    if name == "const32":
        return W.const32()
    raise ValueError(name)


def kernel_bytes(name, nx, ny, nz, kc=None):
    """Algorithmic HBM bytes of one launch: what the pass must read and write
    at least (inputs once, outputs once; spectrum = (nx/2+1) ny nz complex;
    kc = rows per chunk of the z partition, whose 2 ceil(nz/kc) interface rows
    per wavenumber pair the interface pass reads with their three real
    factors and writes back)."""
    n = nx * ny * nz
    ns = (nx // 2 + 1) * ny * nz
    c = 8 if name.endswith("fp32") else 16  # bytes per complex spectrum element
    if name.startswith("fwd_x_method1"):
        return 3 * 8 * n + c * ns
    if name.startswith("fwd_x_resid"):
        return 2 * 8 * n + c * ns
    if name.startswith("fwd_x_const"):
        return 8 * n + c * ns
    if name.startswith("fwd_x_method3"):
        return 3 * 8 * n + c * ns
    if name.startswith("yz_"):
        return 2 * c * ns
    if name.startswith("z_interface"):
        if kc is None:
            return None
        rows = 2 * -(-nz // kc) * (nx // 2 + 1) * ny
        return rows * (2 * c + 3 * c // 2)
    if name.startswith("inv_x_add"):
        return c * ns + 2 * 8 * n
    if name.startswith("inv_x"):
        return c * ns + 8 * n
    if name == "min_rho":
        return 8 * n
    if name == "residual_fp64":
        return 2 * 8 * n
    if name == "adjoint_faces":
        return 4 * 8 * n + 2 * 8 * n  # x, f, rho, p_prev in; grad_f, grad_rho out
    if name == "correct_velocity":
        return 5 * 8 * n + 3 * 8 * n  # u* (3), p, rho in; u (3) out
    return None


def kernel_row(name, rec, spec, kc):
    """Launch count, average duration and algorithmic GB/s of one kernel."""
    launches, total_ms = rec
    avg_us = 1e3 * total_ms / launches
    b = kernel_bytes(name, spec.nx, spec.ny, spec.nz, kc)
    return {"launches": launches, "avg_us": avg_us,
            "alg_gbs": (b / (avg_us * 1e-6) / 1e9) if b else None}


def source_digest():
    """Digest of the device-code sources (.hip, .hpp): counter traffic taken
    on other kernels is not reported."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2005_11806_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if not f.endswith((".hip", ".hpp")):
            continue
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_path(workload):
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs (profiles/traffic_<workload>.json), if they were taken on the current
    kernel sources; else None."""
    path = traffic_path(workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_digest") != source_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


def trace_name(rocprof_name):
    """Library trace name of a rocprofv3 kernel name (None if not ours)."""
    n = rocprof_name
    prec = "fp32" if "<float" in n else "fp64"
    if "k_fwd_x<" in n:
        mode = n.split("k_fwd_x<")[1].split(",")[2].strip()
        return f"fwd_x_{['const', 'method1', 'resid', 'method3'][int(mode)]}_{prec}"
    if "k_inv_x<" in n:
        mode = n.split("k_inv_x<")[1].split(",")[2].strip()
        return f"inv_x_{['store', 'add', 'scale'][int(mode)]}_{prec}"
    if "k_yz<" in n:
        inv = n.split("k_yz<")[1].split(",")[3].split(">")[0].strip()
        return f"yz_{'inv' if inv == 'true' else 'fwd'}_{prec}"
    if "k_ifc<" in n:
        return f"z_interface_{prec}"
    if "k_min_partial" in n or "k_min_final" in n:
        return "min_rho"
    if "k_residual" in n:
        return "residual_fp64"
    return None


def ingest_pmc(fetch_csv, write_csv, workload, command):
    """Writes profiles/traffic_<workload>.json from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of `bench.py --copy-probe`:
    each counter is scaled by what it reads for the 256 MiB device copy."""
    import csv
    import collections
    out = {"source_digest": source_digest(), "workload": workload, "command": command,
           "counters": "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (KiB per dispatch)", "kernels": {}}
    per_launch = {}
    for path, key in ((fetch_csv, "fetch"), (write_csv, "write")):
        probe = []
        # library launches are named by trace name; min_rho is two dispatches
        sums = collections.defaultdict(float)
        counts = collections.defaultdict(int)
        for r in csv.DictReader(open(path)):
            v = float(r["Counter_Value"]) * 1024.0
            if "copyBuffer" in r["Kernel_Name"]:
                probe.append(v)
            name = trace_name(r["Kernel_Name"])
            if name:
                sums[name] += v
                if "k_min_final" not in r["Kernel_Name"]:
                    counts[name] += 1
        # the probe's three 256 MiB copies are the largest copies of the run
        # (input uploads are staged in much smaller copy dispatches)
        probe = sorted(probe)[-3:]
        scale = COPY_PROBE_BYTES / (sum(probe) / len(probe))
        out[f"{key}_scale"] = scale
        for name in sums:
            per_launch.setdefault(name, {})[key] = sums[name] * scale / counts[name]
    for name, d in per_launch.items():
        f, w = d.get("fetch", 0.0), d.get("write", 0.0)
        out["kernels"][name] = {"fetch_bytes_per_launch": f, "write_bytes_per_launch": w,
                                "bytes_per_launch": f + w}
    with open(traffic_path(workload), "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps(out["kernels"], indent=1))


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [i["num_threads"] for i in threadpool_info() if i.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return os.cpu_count() or 1


def host_info():
    """CPU model, usable cores and the BLAS library numpy runs on."""
    import numpy  # noqa: F401  (BLAS is only visible once numpy is loaded)
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        for i in threadpool_info():
            if i.get("user_api") == "blas":
                blas = {"vendor": i.get("internal_api"), "version": i.get("version"),
                        "threads": i.get("num_threads")}
    except Exception:
        pass
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "nproc": ncpu, "blas": blas}


def oracle_solves(f, g, rho, p_prev, budget_s=15.0):
    """Times the FP64 oracle's Method-I solve of one step on the host: as many
    solves of the same inputs as fit in about budget_s seconds (at least
    one). Returns (p of the solve, seconds per solve, solves timed)."""
    import oracle as O
    times = []
    p = None
    while not times or (sum(times) + times[-1] <= budget_s):
        t0 = time.perf_counter()
        (p,), _ = O.solve(f, g, rho, p_prev, n_steps=1, with_relres=False)
        times.append(time.perf_counter() - t0)
    return p, sum(times) / len(times), len(times)


def cpu_baseline(case, n_steps_target, budget_s=15.0):
    """The FP64 oracle on the host: solves of the same workload, one call per
    step (Method-I steps chained through p_prev, as the GPU step chains them),
    as many as fit in about budget_s seconds (at least one)."""
    import oracle as O
    g = O.Grid.from_spec(case.grid)
    f = O.divergence_of_faces(*case.faces, g)
    if case.extra_rhs is not None:
        f = f + case.extra_rhs
    rho = None if case.phi is None else O.mixture_density(case.phi, case.rho_gas, case.rho_liq)
    rho0 = None if rho is None else float(rho.min())
    prev = case.p_prev
    steps, total = 0, 0.0
    while steps == 0 or total < budget_s:
        t0 = time.perf_counter()
        (p,), _ = O.solve(f, g, rho, prev, rho0=rho0, n_steps=1, with_relres=False)
        total += time.perf_counter() - t0
        steps += 1
        if rho is not None:
            prev = p
    kind = "constant-coefficient solve(s)" if rho is None else "chained Method-I step(s)"
    return {"value": g.n * steps / total, "unit": "grid_pts/s", "cores": blas_threads(),
            "kind": "oracle",
            "sample": f"{steps} {kind} of the same grid and inputs ({g.nx}x{g.ny}x{g.nz}), "
                      f"matrix-form DFT + textbook Thomas, {total:.1f} s"}


BATCH_WORKLOADS = {
    "batch64": ("mixed", "default", "64 problems from {64^3, 96x96x128, 128^3, 128x128x192}, "
                "Method I, FP32 bulk + FP64 refinement to relres 1e-10, batched per-pass launches "
                "in one HIP graph"),
    "batch64_persistent": ("mixed", "persistent", "same 64 problems, FP32 + FP64 refinement, one "
                           "persistent launch over the task queue in one HIP graph"),
    "batch64_fp64": ("fp64", "default", "same 64 problems, FP64, batched per-pass launches in one "
                     "HIP graph"),
    "batch64_fp64_seq": ("fp64", None, "same 64 problems, FP64, one plan per problem solved in "
                         "sequence (graph-replayed)"),
}


# Passes of the mixed refinement that a device flag can skip: once the solve
# has converged their launches return at once, so their average launch time
# mixes full and empty launches and says nothing about bandwidth.
GATED = ("fwd_x_resid_fp32", "inv_x_add_fp32")


def dominant_kernel(summary):
    """The kernel with the largest total time among those whose every launch
    does its whole pass."""
    names = [k for k in summary if k not in GATED] or list(summary)
    return max(names, key=lambda k: summary[k][1])


def traced_roofline(plan, step, spec):
    """Runs one traced step and returns the roofline object of its dominant
    kernel (per-kernel event timing on the plan's launch stream). A first
    traced step fills the trace's event pool and is discarded: creating its
    events leaves gaps between the launches in which the GPU slows down."""
    import torch
    settle(step)
    plan.trace(True)
    step()
    torch.cuda.synchronize()
    plan.trace_summary()
    step()
    torch.cuda.synchronize()
    summary = plan.trace_summary()
    plan.trace(False)
    dom = dominant_kernel(summary)
    launches, total_ms = summary[dom]
    avg_s = total_ms / launches * 1e-3
    kc = plan.launch_shape()[1]
    alg = kernel_bytes(dom, spec.nx, spec.ny, spec.nz, kc)
    ach = alg / avg_s / 1e9 if alg else None
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS if ach else None, "traffic": None, "kernel": dom,
            "avg_launch_us": avg_s * 1e6, "algorithmic_bytes": alg, "chunk_rows": kc,
            "kernels": {k: kernel_row(k, v, spec, kc) for k, v in
                        sorted(summary.items(), key=lambda kv: -kv[1][1])}}


METHOD3_WORKLOADS = {
    "method3_128": ("fp64", "128^3 uniform, Method III with its loop (Algorithm 1), 20 spheres, "
                    "rho_l=10, rho_g=1-5, target divergence in the gas, dt=1e-3, to "
                    "eps <= 1e-10 eps(u*); FP64 solves"),
    "method3_128_mixed": ("mixed", "same Method III problem and threshold; FP32 solves inside the "
                          "loop (the loop corrects them)"),
}


def bench_method3(args):
    """Pressure solves per second of Method III's whole loop (grid points /
    time per Algorithm-1 call), iterations and the dominant kernel."""
    import torch
    import paper_2005_11806_amd as psv
    import workloads as W
    prec, desc = METHOD3_WORKLOADS[args.workload]
    case = W.method3_128()
    spec = case.base.grid
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    plan = psv.Plan(psv.Grid.from_spec(spec), precision=prec, autotune=args.autotune)
    U = tuple(to(u) for u in case.base.faces)
    T = to(case.div_target)
    R = plan.density_from_colour(to(case.base.phi), to(case.base.rho_gas), case.base.rho_liq)
    p = torch.empty(spec.nz, spec.ny, spec.nx, dtype=torch.float64, device=dev)
    _, _, info = plan.solve_method3(U, T, R, case.dt, eps_t=0.0, max_iter=1, out=p)
    eps_t = 1e-10 * info.eps_start

    def step():
        return plan.solve_method3(U, T, R, case.dt, eps_t=eps_t, max_iter=500, out=p, u_out=True)

    _, _, info = step()
    settle(step)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = 1e3 * el / args.steps
    line = {
        "metric": METRIC, "value": spec.n * args.steps / el, "unit": "grid_pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic (seeded generators in workloads/)",
        "config": {"workload": f"{args.workload}: {desc}", "grid": [spec.nx, spec.ny, spec.nz],
                   "iterations": info.iterations, "converged": info.converged,
                   "eps": info.eps, "eps_start": info.eps_start,
                   "ms_per_iteration": ms / max(info.iterations, 1)},
        "roofline": traced_roofline(plan, step, spec),
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


GRAD_WORKLOADS = {
    "grad256": ("fp64", "256^3 two-phase Method-I step, forward solve + hand-written adjoint "
                "(grad_f, grad_rho with rho0 = min rho routed to its argmin), FP64"),
    "grad256_mixed": ("mixed", "same forward + adjoint with FP32 solves and FP64 refinement"),
}


def bench_grad(args):
    """Forward + adjoint pairs per second on the 256^3 two-phase step."""
    import torch
    import paper_2005_11806_amd as psv
    import workloads as W
    prec, desc = GRAD_WORKLOADS[args.workload]
    case = W.grad256()
    spec = case.grid
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    plan = psv.Plan(psv.Grid.from_spec(spec), precision=prec, autotune=args.autotune)
    f = plan.divergence(*(to(u) for u in case.faces))
    rho = plan.density_from_colour(to(case.phi), to(case.rho_gas), case.rho_liq)
    pp, w = to(case.p_prev), to(case.w)
    out = torch.empty(spec.nz, spec.ny, spec.nx, dtype=torch.float64, device=dev)

    def step():
        plan.solve(f, rho=rho, p_prev=pp, out=out)
        return plan.adjoint(w, f=f, rho=rho, p_prev=pp)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    line = {
        "metric": METRIC, "value": spec.n * args.steps / el, "unit": "grid_pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic (seeded generators in workloads/)",
        "config": {"workload": f"{args.workload}: {desc}", "grid": [spec.nx, spec.ny, spec.nz]},
        "roofline": traced_roofline(plan, step, spec),
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


CONVERGED_WORKLOADS = {
    "converged128": ("fp64", "method3", "128^3 uniform two-phase, 20 spheres, rho_l=10, rho_g=1-5: "
                     "converged variable-density solve (weights rho) to eps <= 1e-10 eps(0), then "
                     "its implicit adjoint (grad_f, grad_rho) to the same relative threshold; FP64"),
    "converged128_mixed": ("mixed", "method3", "same forward + implicit adjoint with FP32 solves "
                           "inside both loops"),
    "converged128_method1": ("fp64", "method1", "same problem with the Method-I weight min rho "
                             "in both loops; FP64"),
    "converged128_method2": ("fp64", "method2", "same problem with the Method-II weight (harmonic "
                             "mean of min and max rho) in both loops; FP64"),
}


def bench_converged(args):
    """Forward + implicit-adjoint pairs per second of the converged solve."""
    import torch
    import paper_2005_11806_amd as psv
    import workloads as W
    prec, iteration, desc = CONVERGED_WORKLOADS[args.workload]
    case = W.converged_128()
    spec = case.grid
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    plan = psv.Plan(psv.Grid.from_spec(spec), precision=prec, autotune=args.autotune)
    f = plan.divergence(*(to(u) for u in case.faces))
    rho = plan.density_from_colour(to(case.phi), to(case.rho_gas), case.rho_liq)
    w = to(case.w)
    p = torch.empty(spec.nz, spec.ny, spec.nx, dtype=torch.float64, device=dev)
    _, i0 = plan.solve_converged(f, rho, iteration=iteration, max_iter=1, out=p)
    _, _, a0 = plan.converged_adjoint(w, rho, p, iteration=iteration, max_iter=1)
    eps_f, eps_a = 1e-10 * i0.eps_start, 1e-10 * a0.eps_start

    def step():
        _, fi = plan.solve_converged(f, rho, iteration=iteration, eps_t=eps_f, max_iter=2000, out=p)
        _, _, ai = plan.converged_adjoint(w, rho, p, iteration=iteration, eps_t=eps_a,
                                          max_iter=2000)
        return fi, ai

    fi, ai = step()
    settle(step)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = 1e3 * el / args.steps
    line = {
        "metric": METRIC, "value": spec.n * args.steps / el, "unit": "grid_pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic (seeded generators in workloads/)",
        "config": {"workload": f"{args.workload}: {desc}", "grid": [spec.nx, spec.ny, spec.nz],
                   "forward_iterations": fi.iterations, "adjoint_iterations": ai.iterations,
                   "converged": fi.converged and ai.converged,
                   "ms_per_iteration": ms / max(fi.iterations + ai.iterations, 1)},
        "roofline": traced_roofline(plan, step, spec),
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


METHODS2D_WORKLOADS = {
    "bubble2d_methods": ("fp64", "128x256 x-z snapshot shaped like the rising-bubble case (one "
                         "bubble of diameter 0.5 at (0.5, 0.5), density ratio 10): converged "
                         "solves by Methods I, II and III to eps <= 1e-10 eps(0); value is "
                         "Method III's rate, the config holds every method's iterations and time"),
}


def bench_methods2d(args):
    """Converged solves of the 2-D rising-bubble snapshot by the three methods."""
    import torch
    import paper_2005_11806_amd as psv
    import workloads as W
    prec, desc = METHODS2D_WORKLOADS[args.workload]
    case = W.rising_bubble_2d()
    spec = case.grid
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    plan = psv.Plan(psv.Grid.from_spec(spec), precision=prec, autotune=args.autotune)
    f = plan.divergence(*(to(u) for u in case.faces))
    rho = plan.density_from_colour(to(case.phi), to(case.rho_gas), case.rho_liq)
    p = torch.empty(spec.nz, spec.ny, spec.nx, dtype=torch.float64, device=dev)
    eps_t = 1e-10 * float(f.abs().sum())
    per = {}
    for it in ("method1", "method2", "method3"):
        def step(it=it):
            return plan.solve_converged(f, rho, iteration=it, eps_t=eps_t, max_iter=5000, out=p)[1]
        info = step()
        settle(step)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        per[it] = {"iterations": info.iterations, "converged": info.converged,
                   "ms": 1e3 * el / args.steps, "pts_per_s": spec.n * args.steps / el}
    m3 = per["method3"]
    line = {
        "metric": METRIC, "value": m3["pts_per_s"], "unit": "grid_pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": m3["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generators in workloads/)",
        "config": {"workload": f"{args.workload}: {desc}", "grid": [spec.nx, spec.ny, spec.nz],
                   "methods": per,
                   "iterations_I_over_III": per["method1"]["iterations"] / m3["iterations"],
                   "iterations_II_over_III": per["method2"]["iterations"] / m3["iterations"]},
        "roofline": traced_roofline(
            plan, lambda: plan.solve_converged(f, rho, iteration="method3", eps_t=eps_t,
                                               max_iter=5000, out=p), spec),
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def bench_batch(args):
    """Throughput of the 64-problem uneven batch (total grid points per second)."""
    import torch
    import paper_2005_11806_amd as psv
    import workloads as W
    prec, executor, desc = BATCH_WORKLOADS[args.workload]
    cases = W.batch()
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    grids = [psv.Grid.from_spec(c.grid) for c in cases]
    plans = [psv.Plan(g, precision=prec, autotune=args.autotune) for g in grids]
    fs = [pl.divergence(*(to(u) for u in c.faces)) for pl, c in zip(plans, cases)]
    rs = [pl.density_from_colour(to(c.phi), to(c.rho_gas), c.rho_liq) for pl, c in zip(plans, cases)]
    ps = [to(c.p_prev) for c in cases]
    outs = [torch.empty_like(f) for f in fs]
    ntot = sum(c.grid.n for c in cases)
    if executor is None:
        infos = [pl.solve(f, rho=r, p_prev=p, out=o, info=True)[1] for pl, f, r, p, o in
                 zip(plans, fs, rs, ps, outs)]

        def step():
            for pl, f, r, p, o in zip(plans, fs, rs, ps, outs):
                pl.solve(f, rho=r, p_prev=p, out=o)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        run = graph.replay
    else:
        batch = psv.Batch(grids, precision=prec, executor=executor, autotune=args.autotune)
        _, infos = batch.solve(fs, rs, ps, outs, info=True)

        def run():
            batch.solve(fs, rs, ps, outs)
    settle(run)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = 1e3 * el / args.steps
    alg = 32.0 * ntot  # f, rho, p_prev in, p out (FP64)
    ach = alg / (el / args.steps) / 1e9
    line = {
        "metric": METRIC, "value": ntot * args.steps / el, "unit": "grid_pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic (seeded generators in workloads/)",
        "config": {"workload": f"{args.workload}: {desc}", "problems": len(cases), "cells": ntot,
                   "max_relres": max(i.relres for i in infos),
                   "refine_steps": sorted(set(i.refine_steps for i in infos))},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": "whole batch",
                     "algorithmic_bytes": alg},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


SETTLE_S = 0.3


def settle(run):
    """Untimed calls of run() for about SETTLE_S seconds: after the host-side
    set-up the GPU starts at lower clocks, and the first few dozen solves of a
    256x256x512 grid run up to 40% slower than the steady state that a
    sustained job sees (per-dispatch kernel traces show the ramp)."""
    import torch
    t0 = time.perf_counter()
    while True:
        for _ in range(10):
            run()
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= SETTLE_S:
            return


def _timed(run, steps, warmup):
    """Seconds per call of run(): the settle phase, warmup untimed calls, then
    exactly `steps` calls between two device synchronisations."""
    import torch
    settle(run)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _graphed(step):
    """step() captured once in a HIP graph (after one eager warm-up call on a
    side stream); returns the replay function."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    return graph.replay


def _batch_leg(args):
    """C4: 64 uneven problems, one plan at a time (FP64) against the batched
    executors, each at its relres, with a sample of problems against the
    oracle."""
    import numpy as np
    import torch
    import oracle as O
    import paper_2005_11806_amd as psv
    import workloads as W
    cases = W.batch()
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    grids = [psv.Grid.from_spec(c.grid) for c in cases]
    plans = [psv.Plan(g, precision="fp64", autotune=args.autotune) for g in grids]
    fs = [pl.divergence(*(to(u) for u in c.faces)) for pl, c in zip(plans, cases)]
    rs = [pl.density_from_colour(to(c.phi), to(c.rho_gas), c.rho_liq) for pl, c in zip(plans, cases)]
    ps = [to(c.p_prev) for c in cases]
    ntot = sum(c.grid.n for c in cases)
    sizes = np.array([c.grid.n for c in cases])
    sample = sorted({int(np.argmin(sizes)), int(np.argmax(sizes))})
    refs = {}
    for i in sample:
        g = O.Grid.from_spec(cases[i].grid)
        f = O.divergence_of_faces(*cases[i].faces, g)
        rho = O.mixture_density(cases[i].phi, cases[i].rho_gas, cases[i].rho_liq)
        (refs[i],), _ = O.solve(f, g, rho, cases[i].p_prev, with_relres=False)

    def err(outs):
        return max(float(np.abs(outs[i].cpu().numpy() - refs[i]).max() / np.abs(refs[i]).max())
                   for i in sample)

    out = {"workload": "64 problems from {64^3, 96x96x128, 128^3, 128x128x192}, Method I, "
                       "20 spheres each, rho0 = min rho", "problems": len(cases), "cells": ntot,
           "oracle_sample": [[cases[i].grid.nx, cases[i].grid.ny, cases[i].grid.nz] for i in sample]}
    seq_out = [torch.empty_like(f) for f in fs]
    infos = [pl.solve(f, rho=r, p_prev=p, out=o, info=True)[1]
             for pl, f, r, p, o in zip(plans, fs, rs, ps, seq_out)]

    def seq_step():
        for pl, f, r, p, o in zip(plans, fs, rs, ps, seq_out):
            pl.solve(f, rho=r, p_prev=p, out=o)
    t = _timed(_graphed(seq_step), args.steps, args.warmup)
    out["fp64_sequential"] = {"ms": 1e3 * t, "pts_per_s": ntot / t,
                              "max_relres": max(i.relres for i in infos), "err_vs_oracle": err(seq_out)}
    t_seq = t
    for name, prec, ex in (("fp64_batched", "fp64", "default"), ("mixed_batched", "mixed", "default"),
                           ("mixed_persistent", "mixed", "persistent")):
        b = psv.Batch(grids, precision=prec, executor=ex, autotune=args.autotune)
        outs = [torch.empty_like(f) for f in fs]
        _, binf = b.solve(fs, rs, ps, outs, info=True)
        t = _timed(lambda: b.solve(fs, rs, ps, outs), args.steps, args.warmup)
        out[name] = {"ms": 1e3 * t, "pts_per_s": ntot / t, "speedup_vs_fp64_sequential": t_seq / t,
                     "max_relres": max(i.relres for i in binf),
                     "refine_steps": sorted(set(i.refine_steps for i in binf)),
                     "err_vs_oracle": err(outs)}
        b.close()
    return out


def _iterated_leg(args):
    """The converged variable-density solve (Method III weights) on 128^3:
    FP64 solves against FP32 solves inside the same loop, to the same
    summed residual."""
    import torch
    import paper_2005_11806_amd as psv
    import workloads as W
    case = W.converged_128()
    spec = case.grid
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    out = {"workload": "128^3 two-phase (20 spheres, rho_l 10, rho_g 1-5), converged solve "
                       "D(rho_f^-1 G p) = f iterated with Method III weights to eps <= 1e-10 eps(0)"}
    for prec in ("fp64", "mixed"):
        plan = psv.Plan(psv.Grid.from_spec(spec), precision=prec, autotune=args.autotune)
        f = plan.divergence(*(to(u) for u in case.faces))
        rho = plan.density_from_colour(to(case.phi), to(case.rho_gas), case.rho_liq)
        p = torch.empty(spec.nz, spec.ny, spec.nx, dtype=torch.float64, device=dev)
        _, i0 = plan.solve_converged(f, rho, iteration="method3", max_iter=1, out=p)
        eps_t = 1e-10 * i0.eps_start
        _, info = plan.solve_converged(f, rho, iteration="method3", eps_t=eps_t, max_iter=500, out=p)
        t = _timed(lambda: plan.solve_converged(f, rho, iteration="method3", eps_t=eps_t,
                                                max_iter=500, out=p), max(1, args.steps // 4), 1)
        out[prec] = {"ms": 1e3 * t, "pts_per_s": spec.n / t, "iterations": info.iterations,
                     "eps_over_eps0": info.eps / i0.eps_start}
    out["mixed_speedup_vs_fp64"] = out["fp64"]["ms"] / out["mixed"]["ms"]
    return out


def bench_headline(args):
    """The default line: the 256x256x512 FP64 solve, its dominant kernel's
    roofline, the oracle on the host, and the mixed / batched / iterated
    comparisons."""
    import numpy as np
    import torch
    import oracle as O
    import paper_2005_11806_amd as psv
    import workloads as W
    case = W.mixed_tanh()
    spec = case.grid
    n = spec.n
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    plan = psv.Plan(psv.Grid.from_spec(spec), precision="fp64", autotune=args.autotune)
    f = plan.divergence(*(to(u) for u in case.faces))
    rho = plan.density_from_colour(to(case.phi), to(case.rho_gas), case.rho_liq)
    pp = to(case.p_prev)
    out = torch.empty(spec.nz, spec.ny, spec.nx, dtype=torch.float64, device=dev)

    def step():
        plan.solve(f, rho=rho, p_prev=pp, out=out)

    _, info = plan.solve(f, rho=rho, p_prev=pp, out=out, info=True)
    t = _timed(_graphed(step), args.steps, args.warmup)
    ms = 1e3 * t
    p64 = out.cpu().numpy()

    # per-kernel event timing over an eager pass of the same K steps, after the
    # settle phase and one discarded pass that fills the trace's event pool
    settle(step)
    plan.trace(True)
    for rep in range(2):
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        summary = plan.trace_summary()
    plan.trace(False)
    dom = dominant_kernel(summary)
    launches, total_ms = summary[dom]
    avg_s = total_ms / launches * 1e-3
    kc = plan.launch_shape()[1]
    alg = kernel_bytes(dom, spec.nx, spec.ny, spec.nz, kc)
    achieved = alg / avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, "c3_fp64"),
                "kernel": dom, "avg_launch_us": avg_s * 1e6, "algorithmic_bytes": alg,
                "chunk_rows": kc,
                "kernels": {k: kernel_row(k, v, spec, kc) for k, v in
                            sorted(summary.items(), key=lambda kv: -kv[1][1])}}

    if args.legs == "headline":
        args.no_cpu_baseline = True
        tm = float("nan")
    # mixed precision on the same problem
    pm = None if args.legs == "headline" else psv.Plan(psv.Grid.from_spec(spec), precision="mixed", autotune=args.autotune)
    if pm is not None:
        outm = torch.empty_like(out)
        _, minfo = pm.solve(f, rho=rho, p_prev=pp, out=outm, info=True)
        # without info the refinement checks run on the device: graph-replayed
        tm = _timed(_graphed(lambda: pm.solve(f, rho=rho, p_prev=pp, out=outm)), args.steps,
                    args.warmup)
        pmix = outm.cpu().numpy()
        pm.close()

    # the oracle on the host: the same solve, timed, and the reference for both
    g = O.Grid.from_spec(spec)
    fo = O.divergence_of_faces(*case.faces, g)
    ro = O.mixture_density(case.phi, case.rho_gas, case.rho_liq)
    cpu = None
    err64 = errm = None
    if not args.no_cpu_baseline:
        po, t_cpu, nsolves = oracle_solves(fo, g, ro, case.p_prev)
        scale = np.abs(po).max()
        err64 = float(np.abs(p64 - po).max() / scale)
        errm = float(np.abs(pmix - po).max() / scale)
        hi = host_info()
        cpu = {"value": n / t_cpu, "unit": "grid_pts/s",
               "cores": (hi["blas"] or {}).get("threads") or hi["nproc"], "kind": "oracle",
               "sample": f"{nsolves} full Method-I solve(s) of the same 256x256x512 grid and inputs "
                         f"(matrix-form DFT + textbook Thomas), {t_cpu:.2f} s each",
               "host": hi}

    comparisons = None if args.legs == "headline" else {
        "mixed_c3": {"workload": "same grid and inputs, FP32 transforms and tridiagonal sweeps, "
                                 "FP64 residual refinement to relres 1e-10",
                     "ms": 1e3 * tm, "pts_per_s": n / tm, "relres": minfo.relres,
                     "refine_steps": minfo.refine_steps,
                     "relres_per_sweep": list(minfo.relres_sweep), "err_vs_oracle": errm,
                     "speedup_vs_fp64": t / tm},
        "batched_c4": _batch_leg(args),
        "iterated_128": _iterated_leg(args),
    }
    line = {
        "metric": METRIC, "value": n / t, "unit": "grid_pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generators in workloads/)",
        "config": {"workload": "c3_fp64: 256x256x512, z tanh-stretched (alpha 1.5), Method I "
                               "(rho0 = min rho on the device), 200 spheres, rho_l 1000, "
                               "rho_g 1-5, FP64, one solve per step, graph-replayed",
                   "grid": [spec.nx, spec.ny, spec.nz], "precision": "fp64",
                   "relres": info.relres, "err_vs_oracle": err64,
                   "whole_step": {"algorithmic_bytes": 32 * n,
                                  "alg_gbs": 32 * n / t / 1e9,
                                  "frac_of_peak": 32 * n / t / 1e9 / HBM_PEAK_GBS,
                                  "note": "32 B/pt: f, rho, p_prev in and p out, FP64"},
                   "comparisons": comparisons},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3_fp64",
                    choices=["c3_fp64"] + sorted(WORKLOADS) + sorted(BATCH_WORKLOADS) + sorted(METHOD3_WORKLOADS)
                    + sorted(GRAD_WORKLOADS) + sorted(CONVERGED_WORKLOADS)
                    + sorted(METHODS2D_WORKLOADS))
    ap.add_argument("--mode", default="graph", choices=["graph", "eager"])
    ap.add_argument("--autotune", type=int, default=2, choices=[0, 1, 2],
                    help="launch shapes: 0 built-in, 1 from the cache, 2 tuned at plan creation "
                         "when the cache has none (outside the timed region)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="all", choices=["all", "headline"],
                    help="c3_fp64: 'headline' runs the FP64 solve alone (for counter runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run 3 plain device copies of 256 MiB (counter calibration)")
    ap.add_argument("--ingest-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_<workload>.json from two counter runs and exit")
    ap.add_argument("--pmc-command", default="", help="command recorded with --ingest-pmc")
    args = ap.parse_args()
    if args.ingest_pmc:
        ingest_pmc(args.ingest_pmc[0], args.ingest_pmc[1], args.workload, args.pmc_command)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solver has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2005_11806_amd as psv

    if args.copy_probe:
        a = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.workload == "c3_fp64":
        bench_headline(args)
        return
    if args.workload in BATCH_WORKLOADS:
        bench_batch(args)
        return
    if args.workload in METHOD3_WORKLOADS:
        bench_method3(args)
        return
    if args.workload in GRAD_WORKLOADS:
        bench_grad(args)
        return
    if args.workload in CONVERGED_WORKLOADS:
        bench_converged(args)
        return
    if args.workload in METHODS2D_WORKLOADS:
        bench_methods2d(args)
        return

    wl = WORKLOADS[args.workload]
    case = make_case(args.workload)
    spec = case.grid
    dev = torch.device("cuda:0")
    to = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    const = case.phi is None
    plan = psv.Plan(psv.Grid.from_spec(spec), precision=wl["precision"],
                    method="const" if const else "method1", autotune=args.autotune)
    f = plan.divergence(*(to(u) for u in case.faces))
    if case.extra_rhs is not None:
        f += to(case.extra_rhs)
    rho = None if const else plan.density_from_colour(to(case.phi), to(case.rho_gas), case.rho_liq)
    pp = None if const else to(case.p_prev)
    out = torch.empty(spec.nz, spec.ny, spec.nx, dtype=torch.float64, device=dev)
    n_steps = wl["n_steps"]

    def step():
        plan.solve(f, rho=rho, p_prev=pp, n_steps=n_steps, out=out)

    # accuracy of the timed configuration (outside the timed region)
    _, info = plan.solve(f, rho=rho, p_prev=pp, n_steps=n_steps, out=out, info=True)
    mode = args.mode
    graph = None
    if mode == "graph":
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        run = graph.replay
    else:
        run = step

    settle(run)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / args.steps
    value = spec.n * n_steps * args.steps / elapsed

    # per-kernel event timing over an eager pass of the same K steps, after the
    # settle phase and one discarded pass that fills the trace's event pool
    settle(step)
    plan.trace(True)
    for rep in range(2):
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        summary = plan.trace_summary()
    plan.trace(False)
    dom = dominant_kernel(summary)
    launches, total_ms = summary[dom]
    avg_s = total_ms / launches * 1e-3
    kc = plan.launch_shape()[1]
    alg = kernel_bytes(dom, spec.nx, spec.ny, spec.nz, kc)
    achieved = alg / avg_s / 1e9 if alg else None
    traffic = measured_traffic(dom, args.workload)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
                "kernel": dom, "avg_launch_us": avg_s * 1e6, "algorithmic_bytes": alg,
                "chunk_rows": kc,
                "kernels": {k: kernel_row(k, v, spec, kc) for k, v in
                            sorted(summary.items(), key=lambda kv: -kv[1][1])}}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(case, n_steps)

    line = {
        "metric": METRIC, "value": value, "unit": "grid_pts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if wl["precision"] == "fp64" else "f32+f64",
        "data": "synthetic (seeded generators in workloads/)",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "grid": [spec.nx, spec.ny, spec.nz],
                   "solves_per_step": n_steps, "precision": wl["precision"], "mode": mode,
                   "relres_last_solve": info.relres, "refine_steps": info.refine_steps},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
