"""CPU checks of the C ABI: the library loads, exports every entry point that
include/mhar.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2104_07097_amd import mhar

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "mhar.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mhar_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = mhar.load()
    names = _declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    assert set(_declared_functions()) == set(mhar.SIGNATURES)


def test_options_and_strings():
    o = mhar.options("bf16x3", 7, 3)
    assert (o.precision, o.recompute_every, o.steps_per_launch) == (mhar.BF16X3, 7, 3)
    lib = mhar.load()
    assert lib.mhar_version() >= 100
    assert lib.mhar_status_string(mhar.E_NOT_INTERIOR).decode() == "start point not strictly interior"


@pytest.mark.parametrize("n,m,m_eq,code", [(0, 10, 0, mhar.E_SHAPE), (5, 0, 0, mhar.E_SHAPE),
                                           (9000, 10, 0, mhar.E_SHAPE), (5, 10, 5, mhar.E_SHAPE),
                                           (100, 10, 65, mhar.E_SHAPE)])
def test_workspace_size_rejects_bad_shapes(n, m, m_eq, code):
    lib = mhar.load()
    o = mhar.options()
    sz = ctypes.c_size_t()
    assert lib.mhar_problem_workspace_size(n, m, m_eq, ctypes.byref(o), ctypes.byref(sz)) == code
    assert lib.mhar_last_error().decode()


def test_workspace_size_and_bad_options():
    lib = mhar.load()
    sz = ctypes.c_size_t()
    assert lib.mhar_problem_workspace_size(100, 2000, 0, None, ctypes.byref(sz)) == mhar.OK
    # FP32 default: FP64 + FP32 copies of the padded A dominate
    assert sz.value >= 2048 * 128 * 12
    o = mhar.options()
    o.recompute_every = 0
    assert lib.mhar_problem_workspace_size(10, 20, 0, ctypes.byref(o), ctypes.byref(sz)) == mhar.E_INVALID_ARG
    o = mhar.options()
    o.precision = 9
    assert lib.mhar_problem_workspace_size(10, 20, 0, ctypes.byref(o), ctypes.byref(sz)) == mhar.E_INVALID_ARG


def test_create_rejects_null_and_misaligned():
    lib = mhar.load()
    h = ctypes.c_void_p()
    assert lib.mhar_problem_create(10, 20, None, None, 0, None, None, None, None, 0, None,
                                   ctypes.byref(h)) == mhar.E_INVALID_ARG
    # misaligned workspace pointer is refused before any device work
    assert lib.mhar_problem_create(10, 20, 256, 512, 0, None, None, None, 1025, 1 << 20, None,
                                   ctypes.byref(h)) == mhar.E_WORKSPACE
    assert lib.mhar_step(None, 1, None) == mhar.E_INVALID_ARG
    assert lib.mhar_chains_destroy(None) == mhar.OK


@pytest.mark.parametrize("prec,path,code", [("fp32", 5, mhar.E_INVALID_ARG), ("fp32", -1, mhar.E_INVALID_ARG),
                                            ("fp64", "tiled", mhar.E_UNSUPPORTED),
                                            ("bf16x3", "tiled", mhar.OK), ("fp64", "general", mhar.OK),
                                            ("fp64", "lane", mhar.OK), ("bf16x3", "lane", mhar.OK)])
def test_path_option_checked(prec, path, code):
    lib = mhar.load()
    o = mhar.options(prec, path=path)
    sz = ctypes.c_size_t()
    assert lib.mhar_problem_workspace_size(50, 100, 0, ctypes.byref(o), ctypes.byref(sz)) == code


@pytest.mark.parametrize("n,prec,path,code", [(2000, "bf16x3", "auto", mhar.OK), (8192, "fp32", "tiled", mhar.OK),
                                              (2000, "fp64", "auto", mhar.E_SHAPE),
                                              (2000, "fp32", "general", mhar.E_SHAPE),
                                              (2000, "fp32", "resident", mhar.E_SHAPE),
                                              (8193, "bf16x3", "tiled", mhar.E_SHAPE)])
def test_large_n_only_on_the_tiled_path(n, prec, path, code):
    lib = mhar.load()
    o = mhar.options(prec, path=path)
    sz = ctypes.c_size_t()
    assert lib.mhar_problem_workspace_size(n, 3 * n, 1, ctypes.byref(o), ctypes.byref(sz)) == code


def test_checkpoint_arguments_checked():
    lib = mhar.load()
    sz = ctypes.c_size_t()
    assert lib.mhar_checkpoint(None, None, ctypes.byref(sz), None) == mhar.E_INVALID_ARG
    assert lib.mhar_restore(None, None, 0, None) == mhar.E_INVALID_ARG
    assert lib.mhar_trace_read(None, None, None) == mhar.E_INVALID_ARG
    assert lib.mhar_precond_set_complement(None, 0.5) == mhar.E_INVALID_ARG


def test_packed_batch_sizes_and_arguments():
    lib = mhar.load()
    arr = lambda *v: (ctypes.c_int64 * len(v))(*v)
    sz = ctypes.c_size_t()
    o = mhar.options("fp32")
    assert lib.mhar_batch_packed_workspace_size(2, arr(20, 40), arr(100, 300), arr(64, 64),
                                                ctypes.byref(o), ctypes.byref(sz)) == mhar.OK
    small = sz.value
    assert lib.mhar_batch_packed_workspace_size(2, arr(20, 40), arr(100, 300), arr(64, 640),
                                                ctypes.byref(o), ctypes.byref(sz)) == mhar.OK
    assert sz.value > small > 0
    # each problem's handles and the batch tables: at least both problem workspaces
    p1, p2 = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.mhar_problem_workspace_size(20, 100, 0, ctypes.byref(o), ctypes.byref(p1)) == mhar.OK
    assert lib.mhar_problem_workspace_size(40, 300, 0, ctypes.byref(o), ctypes.byref(p2)) == mhar.OK
    assert small > p1.value + p2.value
    for count, n, code in [(0, (20,), mhar.E_INVALID_ARG), (1, (0,), mhar.E_SHAPE),
                           (1, (2000,), mhar.E_UNSUPPORTED)]:
        assert lib.mhar_batch_packed_workspace_size(count, arr(*n), arr(100), arr(16), ctypes.byref(o),
                                                    ctypes.byref(sz)) == code, (count, n)
    assert lib.mhar_batch_packed_workspace_size(1, arr(20), arr(100), arr(0), ctypes.byref(o),
                                                ctypes.byref(sz)) == mhar.E_SHAPE
    h = ctypes.c_void_p()
    offs = arr(0)
    assert lib.mhar_batch_create_packed(1, arr(20), arr(100), arr(16), None, offs, None, offs, None, offs, 0,
                                        ctypes.byref(o), None, 0, None, ctypes.byref(h)) == mhar.E_INVALID_ARG
    assert lib.mhar_batch_get_chains(None, 0, ctypes.byref(h)) == mhar.E_INVALID_ARG
