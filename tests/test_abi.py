"""C-ABI checks that need no GPU: the library loads, exports every function
that include/psv.h declares, and rejects bad arguments on the host before any
device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2005_11806_amd import _abi
import paper_2005_11806_amd as psv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psv_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = _abi.load()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_abi.EXPORTS), set(names) ^ set(_abi.EXPORTS)


def test_struct_layouts_match_header():
    assert C.sizeof(_abi.psv_grid) == 3 * 4 + 4 + 3 * 8 + 8 + 8  # ints, pad, doubles, ptr, enum+pad
    assert C.sizeof(_abi.psv_opts) == 8 + 8 + 6 * 4  # precision, method, tol, 6 ints
    assert C.sizeof(_abi.psv_info) == 8 + 3 * 8 + _abi.PSV_RELRES_HISTORY * 8


def _status(g):
    c, _keep = g._c()
    return _abi.load().psv_grid_validate(C.byref(c))


@pytest.mark.parametrize("nx,ny,nz,code", [
    (32, 32, 32, _abi.PSV_OK), (96, 64, 128, _abi.PSV_OK), (6, 12, 2, _abi.PSV_OK),
    (100, 32, 32, _abi.PSV_ERR_UNSUPPORTED_SIZE),   # radix 5
    (33, 32, 32, _abi.PSV_ERR_UNSUPPORTED_SIZE),    # odd
    (2, 32, 32, _abi.PSV_ERR_UNSUPPORTED_SIZE),     # too small
    (2048, 32, 32, _abi.PSV_ERR_UNSUPPORTED_SIZE),  # too large
    (32, 32, 1, _abi.PSV_ERR_INVALID_ARG),          # nz < 2
    (32, 32, 4096, _abi.PSV_ERR_UNSUPPORTED_SIZE),
    (128, 1, 256, _abi.PSV_OK),                     # two-dimensional x-z problem
    (1, 32, 32, _abi.PSV_ERR_UNSUPPORTED_SIZE),     # only y may be a single cell
    (1, 1, 32, _abi.PSV_ERR_UNSUPPORTED_SIZE),
    (32, 2, 32, _abi.PSV_ERR_UNSUPPORTED_SIZE),
])
def test_grid_validation(nx, ny, nz, code):
    assert _status(psv.Grid(nx, ny, nz)) == code


def test_zf_validation():
    good = np.linspace(0.0, 2.0, 9)
    assert _status(psv.Grid(8, 8, 8, 1, 1, 2.0, good)) == _abi.PSV_OK
    bad = good.copy()
    bad[3] = bad[2]
    assert _status(psv.Grid(8, 8, 8, 1, 1, 2.0, bad)) == _abi.PSV_ERR_INVALID_ARG
    off = good.copy()
    off[0] = 0.1
    assert _status(psv.Grid(8, 8, 8, 1, 1, 2.0, off)) == _abi.PSV_ERR_INVALID_ARG
    end = good.copy()
    end[-1] = 2.5
    assert _status(psv.Grid(8, 8, 8, 1, 1, 2.0, end)) == _abi.PSV_ERR_INVALID_ARG
    assert _status(psv.Grid(8, 8, 8, -1, 1, 2.0)) == _abi.PSV_ERR_INVALID_ARG


def test_plan_create_rejects_before_device_work():
    lib = _abi.load()
    g, _keep = psv.Grid(100, 32, 32)._c()
    h = C.c_void_p()
    assert lib.psv_plan_create(C.byref(g), None, C.byref(h)) == _abi.PSV_ERR_UNSUPPORTED_SIZE
    assert h.value is None
    assert b"2^a 3^b" in lib.psv_last_error_message()
    g2, _k2 = psv.Grid(32, 32, 32)._c()
    o = _abi.psv_opts()
    lib.psv_opts_default(C.byref(o))
    o.precision = 7
    assert lib.psv_plan_create(C.byref(g2), C.byref(o), C.byref(h)) == _abi.PSV_ERR_INVALID_ARG
    lib.psv_opts_default(C.byref(o))
    assert o.chunk_rows == 0
    o.chunk_rows = 12  # only 4, 8 or 16
    assert lib.psv_plan_create(C.byref(g2), C.byref(o), C.byref(h)) == _abi.PSV_ERR_INVALID_ARG
    assert b"chunk_rows" in lib.psv_last_error_message()
    lib.psv_opts_default(C.byref(o))
    assert o.x_stencil == 0
    o.x_stencil = 3  # only 0, 1 or 2
    assert lib.psv_plan_create(C.byref(g2), C.byref(o), C.byref(h)) == _abi.PSV_ERR_INVALID_ARG
    assert b"x_stencil" in lib.psv_last_error_message()
    for bad in (-1, 3):
        lib.psv_opts_default(C.byref(o))
        o.autotune = bad  # 0 built-in, 1 cache only, 2 tune
        assert lib.psv_plan_create(C.byref(g2), C.byref(o), C.byref(h)) == _abi.PSV_ERR_INVALID_ARG
        assert b"autotune" in lib.psv_last_error_message()
    assert lib.psv_plan_create(C.byref(g2), None, None) == _abi.PSV_ERR_INVALID_ARG
    assert lib.psv_plan_shape(None, None, None) == _abi.PSV_ERR_INVALID_ARG


def test_null_plan_and_pointer_errors():
    lib = _abi.load()
    assert lib.psv_solve(None, None, None, 0.0, None, None, 1, None, None) == _abi.PSV_ERR_INVALID_ARG
    assert lib.psv_solve_adjoint(None, None, None, None, 0.0, None, None, None, None, None, None) \
        == _abi.PSV_ERR_INVALID_ARG
    assert lib.psv_density_from_colour(None, None, None, 1.0, None, None) == _abi.PSV_ERR_INVALID_ARG
    assert lib.psv_divergence(None, None, None, None, None, None) == _abi.PSV_ERR_INVALID_ARG
    assert lib.psv_solve_converged(None, None, None, _abi.PSV_ITER_METHOD3, 0.0, 1, None, None,
                                   None, None) == _abi.PSV_ERR_INVALID_ARG
    assert lib.psv_solve_converged_adjoint(None, None, None, None, _abi.PSV_ITER_METHOD1, 0.0, 1,
                                           None, None, None, None) == _abi.PSV_ERR_INVALID_ARG
    n = C.c_size_t()
    assert lib.psv_plan_workspace_size(None, C.byref(n)) == _abi.PSV_ERR_INVALID_ARG
    assert lib.psv_plan_destroy(None) == _abi.PSV_OK


def test_defaults_and_status_strings():
    lib = _abi.load()
    o = _abi.psv_opts()
    lib.psv_opts_default(C.byref(o))
    assert o.precision == _abi.PSV_FP64 and o.method == _abi.PSV_SPLIT_RHO0
    assert o.tol == 1e-10 and o.max_refine == 4
    for code, name in _abi.STATUS_NAMES.items():
        assert lib.psv_status_string(code).decode() == name


def test_static_solve_rejects_on_the_host():
    """The plan-free, allocation-free solve checks its arguments and the size
    of the static array before any device work."""
    lib = _abi.load()
    o = _abi.psv_opts()
    lib.psv_opts_default(C.byref(o))
    big, _k = psv.Grid(256, 256, 256)._c()  # spectrum alone exceeds the array
    x = C.c_void_p(4096)  # never dereferenced: rejected first
    assert lib.psv_solve_static(C.byref(big), C.byref(o), x, x, 0.0, None, x, 1, None) \
        == _abi.PSV_ERR_UNSUPPORTED_SIZE
    assert b"static scratch" in lib.psv_last_error_message()
    small, _k2 = psv.Grid(16, 16, 8)._c()
    o.precision = _abi.PSV_MIXED
    assert lib.psv_solve_static(C.byref(small), C.byref(o), x, x, 0.0, None, x, 1, None) \
        == _abi.PSV_ERR_INVALID_ARG
    lib.psv_opts_default(C.byref(o))
    assert lib.psv_solve_static(C.byref(small), C.byref(o), None, x, 0.0, None, x, 1, None) \
        == _abi.PSV_ERR_INVALID_ARG
    assert lib.psv_solve_static(C.byref(small), C.byref(o), x, x, 0.0, None, x, 0, None) \
        == _abi.PSV_ERR_INVALID_ARG
