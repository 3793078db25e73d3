"""Host half of the C ABI, checked without a GPU: the library loads, exports
every entry point include/fe_abi.h declares, and rejects bad arguments before
touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2104_12282_amd import fe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "fe_abi.h")).read()
    return sorted(set(re.findall(r"^FE_API\s+[\w\s\*]*?\b(\w+)\s*\(", src, re.M)))


def test_header_symbols_match_binding():
    assert _header_symbols() == sorted(fe.ABI_SYMBOLS)


def test_library_exports_every_symbol():
    lib = fe.load_library()
    for name in _header_symbols():
        assert hasattr(lib, name), name


def test_workspace_size_validation():
    lib = fe.load_library()
    good = fe.make_config(24, 12, 12)
    n = lib.fe_workspace_size(C.byref(good))
    assert n > 0 and n % 256 == 0
    bigger = fe.make_config(48, 24, 24)
    assert lib.fe_workspace_size(C.byref(bigger)) > n
    gmg = fe.make_config(24, 12, 12, precond="gmg", mg_levels=3)
    assert lib.fe_workspace_size(C.byref(gmg)) > n
    for kw in ({"nu": 0.5}, {"nu": -1.0}, {"Emin": 0.0}, {"Emin": 2.0}, {"penal": 0.5},
               {"filter_r": 0.0}, {"filter_r": 8.01}, {"h": -1.0}):
        cfg = fe.make_config(24, 12, 12, **kw)
        assert lib.fe_workspace_size(C.byref(cfg)) == 0, kw
    assert lib.fe_workspace_size(C.byref(fe.make_config(0, 12, 12))) == 0
    assert lib.fe_workspace_size(C.byref(fe.make_config(24, 12, 12, filter_r=8.0))) > 0
    # multigrid takes any dimensions (levels of ceil(n / 2) elements per axis)
    # and 2-6 levels
    odd = fe.make_config(25, 13, 7, precond="gmg", mg_levels=3)
    assert lib.fe_workspace_size(C.byref(odd)) > lib.fe_workspace_size(C.byref(fe.make_config(25, 13, 7)))
    for lv in (1, 7):
        assert lib.fe_workspace_size(C.byref(fe.make_config(24, 12, 12, precond="gmg", mg_levels=lv))) == 0


def test_setup_rejects_bad_arguments_without_gpu():
    lib = fe.load_library()
    out = C.c_void_p()
    cfg = fe.make_config(8, 4, 4)
    fake = C.c_void_p(256)  # never dereferenced: validation fails first
    assert lib.fe_setup(C.byref(cfg), None, fake, fake, 16, None, C.byref(out)) == fe.FE_ENOMEM
    assert b"workspace too small" in lib.fe_last_error()
    bad = fe.make_config(8, 4, 4, nu=0.7)
    assert lib.fe_setup(C.byref(bad), None, fake, fake, 1 << 30, None, C.byref(out)) == fe.FE_EINVAL
    assert b"nu" in lib.fe_last_error()
    assert lib.fe_setup(C.byref(cfg), None, None, fake, 1 << 30, None, C.byref(out)) == fe.FE_EINVAL
    assert lib.fe_setup(C.byref(cfg), None, fake, C.c_void_p(257), 1 << 30, None,
                        C.byref(out)) == fe.FE_EINVAL
    assert b"aligned" in lib.fe_last_error()
    assert lib.fe_setup(C.byref(cfg), None, fake, fake, 1 << 30, None, None) == fe.FE_EINVAL


def test_calls_on_null_handle_fail_cleanly():
    lib = fe.load_library()
    x = C.c_void_p(256)
    assert lib.fe_solve(None, x, x, 1e-8, 10, None) == fe.FE_EINVAL
    assert lib.fe_sensitivity(None, x, x, x, None) == fe.FE_EINVAL
    assert lib.fe_filter(None, x, x, 0) == fe.FE_EINVAL
    assert lib.oc_update(None, x, x, x, 0.1, 0.2, x, None) == fe.FE_EINVAL
    assert lib.fe_block_mean(None, x, 2, x) == fe.FE_EINVAL
    assert lib.fe_sensitivity_adjoint(None, x, x, x, x) == fe.FE_EINVAL
    assert lib.fe_set_load(None, x) == fe.FE_EINVAL
    assert lib.fe_get_mg_params(None, None, None, None, None) == fe.FE_EINVAL
    assert lib.fe_set_float32_levels(None, 1) == fe.FE_EINVAL
    assert lib.fe_apply_K(None, x, x, x, 0) == fe.FE_EINVAL
    lib.fe_destroy(None)


def test_serving_footprint_grows_with_grid():
    from paper_2104_12282_amd import serve, synth
    sizes = [serve.request_footprint(*g, precision="fp32_ir", precond="gmg", mg_levels=3)
             for g in synth.SERVING_GRIDS]
    assert all(a < b for a, b in zip(sizes, sizes[1:]))
    assert sizes[-1] < 1 << 30  # the largest request fits easily in HBM


def test_batch_workspace_and_argument_validation_without_gpu():
    lib = fe.load_library()
    cfg = fe.make_config(16, 8, 8, precision="fp32_ir", precond="gmg", mg_levels=3)
    one = lib.fe_workspace_size(C.byref(cfg))
    n4 = lib.fe_batch_workspace_size(C.byref(cfg), 4)
    # four slots, each at least a lone problem's workspace, plus the idle slots' zero load
    assert n4 >= 4 * one and n4 % 256 == 0
    assert lib.fe_batch_workspace_size(C.byref(cfg), 8) > n4
    assert lib.fe_batch_workspace_size(C.byref(cfg), 0) == 0
    assert lib.fe_batch_workspace_size(C.byref(cfg), 2000) == 0
    jac = fe.make_config(16, 8, 8, precision="fp32_ir", precond="jacobi")
    assert lib.fe_batch_workspace_size(C.byref(jac), 4) == 0   # batches are multigrid only
    bf = fe.make_config(16, 8, 8, precision="bf16_ir", precond="gmg", mg_levels=3)
    assert lib.fe_batch_workspace_size(C.byref(bf), 4) == 0    # not on matrix cores
    out = C.c_void_p()
    fake = C.c_void_p(256)
    assert lib.fe_batch_create(C.byref(cfg), 4, fake, 16, None, C.byref(out)) == fe.FE_ENOMEM
    assert lib.fe_batch_create(C.byref(jac), 4, fake, 1 << 30, None, C.byref(out)) == fe.FE_EINVAL
    assert lib.fe_batch_create(C.byref(cfg), 4, C.c_void_p(257), 1 << 30, None, C.byref(out)) == fe.FE_EINVAL
    assert lib.fe_batch_round_begin(None) == fe.FE_EINVAL
    assert lib.fe_batch_round_end(None, None) == fe.FE_EINVAL
    assert lib.fe_batch_setup_slot(None, 0, None, None, C.byref(out)) == fe.FE_EINVAL
    lib.fe_batch_destroy(None)
