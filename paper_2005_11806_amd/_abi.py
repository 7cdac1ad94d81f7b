"""ctypes declarations of include/psv.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsv.so")

PSV_OK, PSV_ERR_INVALID_ARG, PSV_ERR_UNSUPPORTED_SIZE, PSV_ERR_HIP, PSV_ERR_NONFINITE, \
    PSV_ERR_NOT_CONVERGED, PSV_ERR_OOM = range(7)
PSV_FP64, PSV_MIXED = 0, 1
PSV_CONST, PSV_SPLIT_RHO0 = 0, 1
PSV_ITER_METHOD1, PSV_ITER_METHOD2, PSV_ITER_METHOD3 = 1, 2, 3
PSV_BC_WALL_NEUMANN = 0

STATUS_NAMES = {0: "PSV_OK", 1: "PSV_ERR_INVALID_ARG", 2: "PSV_ERR_UNSUPPORTED_SIZE", 3: "PSV_ERR_HIP",
                4: "PSV_ERR_NONFINITE", 5: "PSV_ERR_NOT_CONVERGED", 6: "PSV_ERR_OOM"}

dptr = C.POINTER(C.c_double)


class psv_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("zf", dptr), ("bc_z", C.c_int)]


class psv_opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("method", C.c_int), ("tol", C.c_double),
                ("max_refine", C.c_int32), ("check_inputs", C.c_int32), ("autotune", C.c_int32),
                ("batch_executor", C.c_int32), ("chunk_rows", C.c_int32), ("x_stencil", C.c_int32)]


PSV_RELRES_HISTORY = 8


class psv_info(C.Structure):
    _fields_ = [("refine_steps", C.c_int32), ("relres", C.c_double),
                ("rhs_mean_removed", C.c_double), ("rho0_used", C.c_double),
                ("relres_sweep", C.c_double * PSV_RELRES_HISTORY)]


class psv_shape(C.Structure):
    _fields_ = [("lines_x", C.c_int32), ("lines_x_inv", C.c_int32), ("chunk_rows", C.c_int32),
                ("x_staged", C.c_int32), ("x_order", C.c_int32)]


class psv_m3_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("eps", C.c_double),
                ("eps_start", C.c_double)]


EXPORTS = {
    # name: (restype, argtypes)
    "psv_opts_default": (None, [C.POINTER(psv_opts)]),
    "psv_grid_validate": (C.c_int, [C.POINTER(psv_grid)]),
    "psv_plan_create": (C.c_int, [C.POINTER(psv_grid), C.POINTER(psv_opts), C.POINTER(C.c_void_p)]),
    "psv_plan_workspace_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "psv_plan_shape": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "psv_plan_get_shape": (C.c_int, [C.c_void_p, C.POINTER(psv_shape)]),
    "psv_plan_set_shape": (C.c_int, [C.c_void_p, C.POINTER(psv_shape)]),
    "psv_plan_destroy": (C.c_int, [C.c_void_p]),
    "psv_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                            C.c_int32, C.c_void_p, C.POINTER(psv_info)]),
    "psv_solve_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, dptr, C.c_void_p]),
    "psv_solve_method3": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_double, C.c_double, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.POINTER(psv_m3_info)]),
    "psv_solve_converged": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                                      C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(psv_m3_info)]),
    "psv_solve_converged_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.c_int32, C.c_double, C.c_int32, C.c_void_p,
                                              C.c_void_p, C.c_void_p, C.POINTER(psv_m3_info)]),
    "psv_solve_static": (C.c_int, [C.POINTER(psv_grid), C.POINTER(psv_opts), C.c_void_p, C.c_void_p,
                                   C.c_double, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "psv_density_from_colour": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                                          C.c_void_p]),
    "psv_divergence": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "psv_relres": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, dptr]),
    "psv_batch_create": (C.c_int, [C.c_int32, C.POINTER(psv_grid), C.POINTER(psv_opts),
                                   C.POINTER(C.c_void_p)]),
    "psv_batch_solve": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), dptr,
                                  C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p,
                                  C.POINTER(psv_info)]),
    "psv_batch_destroy": (C.c_int, [C.c_void_p]),
    "psv_trace_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "psv_trace_summary": (C.c_int, [C.c_void_p, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "psv_status_string": (C.c_char_p, [C.c_int]),
    "psv_last_error_message": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads libpsv.so (built by paper_2005_11806_amd.build). Raises if absent:
    there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpsv.so not found at {path}; build it with "
                           "`python -m paper_2005_11806_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PsvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int):
    if status != PSV_OK:
        raise PsvError(status, load().psv_last_error_message().decode(errors="replace"))
