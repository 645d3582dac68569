"""The C ABI library loads on a machine without a GPU, exports every entry
point that include/dm.h declares, and rejects bad arguments before touching
the HIP runtime."""
import ctypes
import os
import re

import pytest

import paper_2108_13478_amd as dmlib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dmlib.LIB_PATH):
        from paper_2108_13478_amd import build
        build.build()
    return dmlib.load()


def header_functions():
    text = open(os.path.join(ROOT, "include", "dm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dm_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(dmlib.EXPORTED) == names


def test_default_options(lib):
    opt = dmlib.dm_options()
    lib.dm_default_options(ctypes.byref(opt))
    assert opt.device == 0 and opt.precision == dmlib.DM_FP64
    assert opt.spin == 2.0 and opt.lanczos_steps == 100 and opt.bound_margin == 0.01


def test_null_arguments_rejected_without_hip(lib):
    assert lib.dm_init(None, None) == dmlib.DM_E_ARG
    assert b"NULL" in lib.dm_last_error(None)
    assert lib.dm_set_fock(None, 4, None, None, None, None, None, None, 1) == dmlib.DM_E_ARG
    assert lib.dm_chebyshev_block(None, None, 0, 10, 0.0, 1.0, None) == dmlib.DM_E_ARG
    assert lib.dm_trace(None, 0.0, 1.0, None, None) == dmlib.DM_E_ARG
    assert lib.dm_solve_mu(None, 1.0, 1.0, 1e-6, None) == dmlib.DM_E_ARG
    assert lib.dm_stoch_moments(None, 4, 1, None, None) == dmlib.DM_E_ARG
    lib.dm_destroy(None)


def test_invalid_options_rejected_before_device_query(lib):
    opt = dmlib.dm_options()
    lib.dm_default_options(ctypes.byref(opt))
    opt.precision = 7
    h = ctypes.c_void_p()
    assert lib.dm_init(ctypes.byref(h), ctypes.byref(opt)) == dmlib.DM_E_ARG
    assert not h.value
    opt.precision = 0
    opt.spin = -1.0
    assert lib.dm_init(ctypes.byref(h), ctypes.byref(opt)) == dmlib.DM_E_ARG


def test_tile_shape_table_without_hip(lib):
    shapes = dmlib.tile_shapes()
    assert len(shapes) == lib.dm_num_tile_shapes() >= 13
    for rows, cols, split in shapes:
        assert rows % 16 == 0 and cols % 16 == 0 and split in (1, 8, 16)
    assert any(s > 1 for _, _, s in shapes)  # split-reduction shapes for narrow passes
    assert lib.dm_tile_shape(len(shapes), None, None, None) == dmlib.DM_E_ARG
    assert lib.dm_tile_shape(-1, None, None, None) == dmlib.DM_E_ARG
    assert lib.dm_set_pass_shape(None, 32, 0) == dmlib.DM_E_ARG


def test_multi_and_dos_reject_null_context(lib):
    assert lib.dm_chebyshev_block_multi(None, None, 0, 10, 1, None, None, None) == dmlib.DM_E_ARG
    assert lib.dm_dos(None, 0, 0, None, 1.0, None) == dmlib.DM_E_ARG
