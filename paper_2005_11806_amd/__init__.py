"""MI355X-native eigenexpansion pressure solve for variable-density two-phase
flow (Dalla Barba et al., arXiv:2005.11806, Sec. 3.3.1).

Thin Python binding over libpsv.so (include/psv.h): every step of the solve
runs in the library's HIP kernels; this module only checks tensors and passes
their device pointers. PyTorch provides device memory and streams.

    import paper_2005_11806_amd as psv
    plan = psv.Plan(psv.Grid(128, 128, 128, 1.0, 1.0, 1.0))
    p = plan.solve(f, rho=rho, p_prev=p_prev, n_steps=10)
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np

from . import _abi
from ._abi import PsvError, check

__all__ = ["Grid", "Plan", "Batch", "SolveInfo", "Method3Info", "PsvError", "lib",
           "PressureSolve", "pressure_solve", "ConvergedSolve", "converged_solve"]


def lib():
    return _abi.load()


@dataclasses.dataclass
class Grid:
    """Periodic x, y; walls in z. zf: nz+1 face positions (0 .. lz) or None (uniform)."""
    nx: int
    ny: int
    nz: int
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0
    zf: object = None

    @classmethod
    def from_spec(cls, spec):
        return cls(spec.nx, spec.ny, spec.nz, spec.lx, spec.ly, spec.lz, spec.zf)

    def _c(self):
        g = _abi.psv_grid()
        g.nx, g.ny, g.nz = int(self.nx), int(self.ny), int(self.nz)
        g.lx, g.ly, g.lz = float(self.lx), float(self.ly), float(self.lz)
        keep = None
        if self.zf is not None:
            keep = np.ascontiguousarray(np.asarray(self.zf, dtype=np.float64))
            g.zf = keep.ctypes.data_as(_abi.dptr)
        else:
            g.zf = None
        g.bc_z = _abi.PSV_BC_WALL_NEUMANN
        return g, keep

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def validate(self):
        g, _keep = self._c()
        check(lib().psv_grid_validate(C.byref(g)))


@dataclasses.dataclass
class SolveInfo:
    refine_steps: int
    relres: float
    rhs_mean_removed: float
    rho0_used: float
    relres_sweep: tuple = ()  # mixed: relres after the FP32 solve and after each sweep


def _info(x):
    hist = tuple(v for v in x.relres_sweep if v == v)  # drop the NaN tail
    return SolveInfo(x.refine_steps, x.relres, x.rhs_mean_removed, x.rho0_used, hist)


@dataclasses.dataclass
class Method3Info:
    iterations: int      # eigenexpansion solves performed
    converged: bool      # eps <= eps_t
    eps: float           # sum over cells of |div u - div_target| of the result
    eps_start: float     # the same for u* (nan when started from p_init)


_PREC = {"fp64": _abi.PSV_FP64, "mixed": _abi.PSV_MIXED}
_METH = {"const": _abi.PSV_CONST, "method1": _abi.PSV_SPLIT_RHO0}
_XSTENCIL = {"auto": 0, "staged": 1, "direct": 2}
_ITER = {"method1": _abi.PSV_ITER_METHOD1, "method2": _abi.PSV_ITER_METHOD2,
         "method3": _abi.PSV_ITER_METHOD3}


def _iteration(name):
    if name not in _ITER:
        raise ValueError(f"iteration must be one of {sorted(_ITER)}, got {name!r}")
    return _ITER[name]


def _ptr(t, shape=None, name="tensor"):
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Plan:
    """A solver plan: device tables and workspace for one grid.

    precision: "fp64" or "mixed" (FP32 transforms/tridiagonal + FP64 refinement);
    method: "method1" (Eq. poisson_me1 with rho0 = min rho) or "const".
    """

    def __init__(self, grid: Grid, precision="fp64", method="method1", tol=1e-10,
                 max_refine=4, check_inputs=False, autotune=0, chunk_rows=0, x_stencil="auto"):
        self.grid = grid
        self.precision = precision
        self.method = method
        o = _abi.psv_opts()
        lib().psv_opts_default(C.byref(o))
        o.precision = _PREC[precision]
        o.method = _METH[method]
        o.tol = float(tol)
        o.max_refine = int(max_refine)
        o.check_inputs = int(bool(check_inputs))
        o.autotune = int(autotune)
        o.chunk_rows = int(chunk_rows)
        o.x_stencil = _XSTENCIL[x_stencil]
        g, _keep = grid._c()
        h = C.c_void_p()
        check(lib().psv_plan_create(C.byref(g), C.byref(o), C.byref(h)))
        self._h = h

    @property
    def shape(self):
        return self.grid.shape

    def workspace_size(self) -> int:
        n = C.c_size_t()
        check(lib().psv_plan_workspace_size(self._h, C.byref(n)))
        return n.value

    def launch_shape(self):
        """(x lines per block, rows per chunk of the wall-normal partition)."""
        lx, kc = C.c_int(), C.c_int()
        check(lib().psv_plan_shape(self._h, C.byref(lx), C.byref(kc)))
        return lx.value, kc.value

    def get_shape(self) -> dict:
        """Every launch-shape field (psv_plan_get_shape)."""
        sh = _abi.psv_shape()
        check(lib().psv_plan_get_shape(self._h, C.byref(sh)))
        return {k: getattr(sh, k) for k, _ in _abi.psv_shape._fields_}

    def set_shape(self, **fields):
        """Replaces launch-shape fields (psv_plan_set_shape); unnamed ones keep
        their value."""
        cur = self.get_shape()
        unknown = set(fields) - set(cur)
        if unknown:
            raise ValueError(f"unknown shape fields {sorted(unknown)}")
        cur.update(fields)
        sh = _abi.psv_shape(**{k: int(v) for k, v in cur.items()})
        check(lib().psv_plan_set_shape(self._h, C.byref(sh)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            check(lib().psv_plan_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, f, rho=None, p_prev=None, rho0=None, n_steps=1, out=None, stream=None,
              info=False):
        import torch
        sh = self.shape
        if out is None:
            out = torch.empty(sh, dtype=torch.float64, device=f.device)
        inf = _abi.psv_info() if info else None
        st = lib().psv_solve(self._h, _ptr(f, sh, "f"), _ptr(rho, sh, "rho"),
                             0.0 if rho0 is None else float(rho0), _ptr(p_prev, sh, "p_prev"),
                             _ptr(out, sh, "out"), int(n_steps), _stream(stream),
                             C.byref(inf) if info else None)
        if info:
            si = _info(inf)
            if st == _abi.PSV_ERR_NOT_CONVERGED:
                raise PsvError(st, f"not converged: {si}")
            check(st)
            return out, si
        check(st)
        return out

    def adjoint(self, w, f=None, rho=None, p_prev=None, rho0=None, grad_f=True, grad_rho=True,
                grad_p_prev=False, grad_rho0=False, stream=None):
        """Gradients of sum(w * p) for one step; returns a dict of tensors
        (and 'rho0' as a float when grad_rho0)."""
        import torch
        sh = self.shape
        mk = lambda want: torch.empty(sh, dtype=torch.float64, device=w.device) if want else None  # noqa
        gf, gr, gp = mk(grad_f), mk(grad_rho), mk(grad_p_prev)
        r0 = C.c_double(0.0)
        check(lib().psv_solve_adjoint(self._h, _ptr(w, sh, "w"), _ptr(f, sh, "f"), _ptr(rho, sh, "rho"),
                                      0.0 if rho0 is None else float(rho0), _ptr(p_prev, sh, "p_prev"),
                                      _ptr(gf, sh), _ptr(gr, sh), _ptr(gp, sh),
                                      C.byref(r0) if grad_rho0 else None, _stream(stream)))
        out = {"f": gf, "rho": gr, "p_prev": gp}
        if grad_rho0:
            out["rho0"] = r0.value
        return out

    def solve_method3(self, u_star, div_target, rho, dt, eps_t=0.0, max_iter=50, p_init=None,
                      out=None, u_out=False, stream=None):
        """Method III with its loop (psv_solve_method3). u_star = (ux, uy, uz)
        face tensors ([nz][ny][nx] twice, [nz+1][ny][nx]). Returns
        (p, (ux, uy, uz) or None, Method3Info)."""
        import torch
        sh = self.shape
        nz, ny, nx = sh
        ux, uy, uz = u_star
        if out is None:
            out = torch.empty(sh, dtype=torch.float64, device=rho.device)
        uo = None
        if u_out:
            uo = (torch.empty(sh, dtype=torch.float64, device=rho.device),
                  torch.empty(sh, dtype=torch.float64, device=rho.device),
                  torch.empty((nz + 1, ny, nx), dtype=torch.float64, device=rho.device))
        inf = _abi.psv_m3_info()
        check(lib().psv_solve_method3(
            self._h, _ptr(ux, sh, "ux"), _ptr(uy, sh, "uy"), _ptr(uz, (nz + 1, ny, nx), "uz"),
            _ptr(div_target, sh, "div_target"), _ptr(rho, sh, "rho"), float(dt), float(eps_t),
            int(max_iter), _ptr(p_init, sh, "p_init"), _ptr(out, sh, "out"),
            _ptr(uo[0], sh) if uo else None, _ptr(uo[1], sh) if uo else None,
            _ptr(uo[2], (nz + 1, ny, nx)) if uo else None, _stream(stream), C.byref(inf)))
        return out, uo, Method3Info(inf.iterations, bool(inf.converged), inf.eps, inf.eps_start)

    def solve_converged(self, f, rho, iteration="method3", eps_t=0.0, max_iter=50, p_init=None,
                        out=None, stream=None):
        """Converged variable-density solve D(rho_f^-1 G p) = f - mean_V(f)
        (psv_solve_converged). iteration: "method1" (weight min rho),
        "method2" (harmonic mean of min and max rho) or "method3" (weight rho). Returns (p, Method3Info); eps is the summed
        absolute residual of that equation."""
        import torch
        sh = self.shape
        if out is None:
            out = torch.empty(sh, dtype=torch.float64, device=f.device)
        inf = _abi.psv_m3_info()
        check(lib().psv_solve_converged(
            self._h, _ptr(f, sh, "f"), _ptr(rho, sh, "rho"), _iteration(iteration), float(eps_t),
            int(max_iter), _ptr(p_init, sh, "p_init"), _ptr(out, sh, "out"), _stream(stream),
            C.byref(inf)))
        return out, Method3Info(inf.iterations, bool(inf.converged), inf.eps, inf.eps_start)

    def converged_adjoint(self, w, rho, p, iteration="method3", eps_t=0.0, max_iter=50,
                          grad_f=True, grad_rho=True, stream=None):
        """Implicit adjoint of solve_converged for loss = sum(w p)
        (psv_solve_converged_adjoint). Returns (grad_f or None, grad_rho or
        None, Method3Info of the adjoint solve)."""
        import torch
        sh = self.shape
        gf = torch.empty(sh, dtype=torch.float64, device=w.device) if grad_f else None
        gr = torch.empty(sh, dtype=torch.float64, device=w.device) if grad_rho else None
        inf = _abi.psv_m3_info()
        check(lib().psv_solve_converged_adjoint(
            self._h, _ptr(w, sh, "w"), _ptr(rho, sh, "rho"), _ptr(p, sh, "p"), _iteration(iteration),
            float(eps_t), int(max_iter), _ptr(gf, sh), _ptr(gr, sh), _stream(stream),
            C.byref(inf)))
        return gf, gr, Method3Info(inf.iterations, bool(inf.converged), inf.eps, inf.eps_start)

    def density_from_colour(self, phi, rho_gas, rho_liq, out=None, stream=None):
        import torch
        sh = self.shape
        if out is None:
            out = torch.empty(sh, dtype=torch.float64, device=phi.device)
        check(lib().psv_density_from_colour(self._h, _ptr(phi, sh, "phi"), _ptr(rho_gas, sh, "rho_gas"),
                                            float(rho_liq), _ptr(out, sh, "out"), _stream(stream)))
        return out

    def divergence(self, ux, uy, uz, out=None, stream=None):
        import torch
        nz, ny, nx = self.shape
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=ux.device)
        check(lib().psv_divergence(self._h, _ptr(ux, self.shape, "ux"), _ptr(uy, self.shape, "uy"),
                                   _ptr(uz, (nz + 1, ny, nx), "uz"), _ptr(out, self.shape, "out"),
                                   _stream(stream)))
        return out

    def trace(self, enable=True):
        """Per-kernel HIP-event timing of this plan's launches."""
        check(lib().psv_trace_enable(self._h, int(bool(enable))))

    def trace_summary(self) -> dict:
        """{kernel: (launches, total_ms)} since the last summary (synchronises)."""
        import json
        need = C.c_size_t()
        buf = C.create_string_buffer(1 << 16)
        check(lib().psv_trace_summary(self._h, buf, len(buf), C.byref(need)))
        if need.value > len(buf):
            raise RuntimeError("trace summary truncated")
        return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}

    def relres(self, r, p, stream=None) -> float:
        v = C.c_double()
        check(lib().psv_relres(self._h, _ptr(r, self.shape, "r"), _ptr(p, self.shape, "p"),
                               _stream(stream), C.byref(v)))
        return v.value


class Batch:
    """Uneven batch of independent problems solved together (psv_batch_*):
    one grid per problem, same options for all; replayed from a HIP graph.
    autotune (0, 1, 2) and x_stencil pick each problem's launch shapes as
    they do for a Plan."""

    _EXEC = {"default": 0, "passes": 1, "persistent": 2}

    def __init__(self, grids, precision="mixed", method="method1", tol=1e-10, max_refine=4,
                 executor="default", chunk_rows=0, autotune=0, x_stencil="auto"):
        self.grids = list(grids)
        n = len(self.grids)
        arr = (_abi.psv_grid * n)()
        self._keep = []
        for i, g in enumerate(self.grids):
            c, keep = g._c()
            arr[i] = c
            self._keep.append(keep)
        o = _abi.psv_opts()
        lib().psv_opts_default(C.byref(o))
        o.precision = _PREC[precision]
        o.method = _METH[method]
        o.tol = float(tol)
        o.max_refine = int(max_refine)
        o.batch_executor = self._EXEC[executor]
        o.chunk_rows = int(chunk_rows)
        o.autotune = int(autotune)
        o.x_stencil = _XSTENCIL[x_stencil]
        h = C.c_void_p()
        check(lib().psv_batch_create(n, arr, C.byref(o), C.byref(h)))
        self._h = h
        self.n = n
        self.method = method

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            check(lib().psv_batch_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, fs, rhos=None, p_prevs=None, outs=None, rho0s=None, stream=None, info=False):
        import torch
        n = self.n
        if outs is None:
            outs = [torch.empty(g.shape, dtype=torch.float64, device=fs[i].device)
                    for i, g in enumerate(self.grids)]
        P = C.c_void_p * n
        f_a = P(*[_ptr(fs[i], self.grids[i].shape, "f").value for i in range(n)])
        o_a = P(*[_ptr(outs[i], self.grids[i].shape, "out").value for i in range(n)])
        r_a = P(*[_ptr(rhos[i], self.grids[i].shape, "rho").value for i in range(n)]) if rhos else None
        p_a = P(*[_ptr(p_prevs[i], self.grids[i].shape, "p_prev").value for i in range(n)]) \
            if p_prevs else None
        r0 = (C.c_double * n)(*[0.0 if rho0s is None else float(rho0s[i]) for i in range(n)])
        infos = (_abi.psv_info * n)() if info else None
        st = lib().psv_batch_solve(self._h, f_a, r_a, r0, p_a, o_a, _stream(stream), infos)
        if info:
            out_infos = [_info(x) for x in infos]
            if st == _abi.PSV_ERR_NOT_CONVERGED:
                raise PsvError(st, f"not converged: {out_infos}")
            check(st)
            return outs, out_infos
        check(st)
        return outs


from .autograd import (PressureSolve, pressure_solve, ConvergedSolve,  # noqa: E402
                       converged_solve)
