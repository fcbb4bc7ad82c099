"""The C-ABI library loads and exports what include/ddhf.h declares.

CPU only: loading the library and the pure host entry points (parameter
checks, sizes, argument errors) touch no GPU.
"""
import ctypes
import os
import re

import pytest

from conftest import ROOT
from paper_1803_11449_amd import ddhf

HEADER = os.path.join(ROOT, "include", "ddhf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sketch_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ddhf.LIB_PATH):
        pytest.fail("libddhf.so is not built (run __graft_entry__.build())")
    return ddhf.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(ddhf.EXPORTS)


def test_struct_layouts_match_header():
    assert ctypes.sizeof(ddhf.sketch_params_t) == 32
    assert ctypes.sizeof(ddhf.sketch_sp_t) == 16
    assert ctypes.sizeof(ddhf.sketch_info_t) == 216
    assert ctypes.sizeof(ddhf.sketch_update_job_t) == 24
    assert ctypes.sizeof(ddhf.sketch_restore_job_t) == 56
    assert ctypes.sizeof(ddhf.sketch_plan_job_t) == 32
    assert ctypes.sizeof(ddhf.sketch_timings_t) == 72


def test_params_default_check_and_bytes(L):
    p = ddhf.sketch_params_default()
    assert (p.g, p.k, p.r, p.alpha) == (1024, 14, 5, 6)
    assert ddhf.sketch_params_check(p) == ddhf.SKETCH_OK
    assert ddhf.sketch_bytes(p) == 5 * 2**14 * 128
    p2 = ddhf.sketch_params_t(1024, 18, 5, 5, 1, 0)
    assert ddhf.sketch_bytes(p2) == 5 * 2**18 * 128


@pytest.mark.parametrize("g,k,r,alpha", [
    (1024, 14, 5, 5), (1024, 14, 5, 15), (1000, 14, 5, 6), (16, 14, 5, 6),
    (1024, 4, 8, 4), (1024, 25, 5, 6), (1024, 14, 9, 6), (1024, 24, 3, 2)])
def test_invalid_params_rejected(L, g, k, r, alpha):
    p = ddhf.sketch_params_t(g, k, r, alpha, 1, 0)
    assert ddhf.sketch_params_check(p) == ddhf.SKETCH_E_INVAL
    assert ddhf.sketch_bytes(p) == 0
    h = ctypes.c_void_p()
    assert L.sketch_create(ctypes.byref(p), ctypes.byref(h)) == ddhf.SKETCH_E_INVAL
    assert h.value is None
    assert ddhf.last_error()


def test_null_handle_errors(L):
    n = ctypes.c_size_t(0)
    assert L.sketch_update(None, None, 0, None) == ddhf.SKETCH_E_INVAL
    assert L.sketch_reset(None, None) == ddhf.SKETCH_E_INVAL
    assert L.sketch_restore(None, 1024.0, None, 0, ctypes.byref(n), None,
                            None) == ddhf.SKETCH_E_INVAL
    assert L.sketch_download(None, None, 0, None) == ddhf.SKETCH_E_INVAL
    assert L.sketch_candidates(None, 1.0, None, 0, ctypes.byref(n), None) == ddhf.SKETCH_E_INVAL
    assert L.sketch_update_batch(None, 1, None) == ddhf.SKETCH_E_INVAL
    assert L.sketch_update_batch(None, 0, None) == ddhf.SKETCH_OK
    assert L.sketch_restore_batch(None, 1, None) == ddhf.SKETCH_E_INVAL
    assert L.sketch_merge(None, None, None) == ddhf.SKETCH_E_INVAL
    assert L.sketch_set_option(None, 1, 0) == ddhf.SKETCH_E_INVAL
    L.sketch_destroy(None)
    assert "NULL" in ddhf.last_error()
    out = ctypes.c_void_p()
    assert L.sketch_plan_create(None, 0, 3, ctypes.byref(out)) == ddhf.SKETCH_E_INVAL
    assert L.sketch_plan_create(None, 1, 3, None) == ddhf.SKETCH_E_INVAL
    assert L.sketch_plan_run(None, None) == ddhf.SKETCH_E_INVAL
    assert L.sketch_plan_results(None, None, 0, None) == ddhf.SKETCH_E_INVAL
    assert L.sketch_plan_launches(None) == 0
    L.sketch_plan_destroy(None)
