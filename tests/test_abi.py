"""The C-ABI library loads on the CPU and exports every declared entry point."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "podcg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(podcg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_sequence_calls():
    names = declared_functions()
    for must in ("podcg_set_matrix", "podcg_push_snapshot", "podcg_build_pod", "podcg_solve"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1512_05820_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpodcg.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_lib.EXPORTED) == declared_functions()


def test_strerror_and_defaults_without_gpu():
    from paper_1512_05820_amd import _lib
    L = _lib.load()
    assert L.podcg_strerror(-4) == b"matrix is not symmetric positive definite"
    o = _lib.Options()
    L.podcg_default_options(ctypes.byref(o))
    assert (o.omega, o.rank_max, o.check_every) == (20, 10, 16)
    assert o.rank_rtol == 1e-12


def test_create_rejects_bad_arguments_before_touching_the_gpu():
    from paper_1512_05820_amd import _lib
    L = _lib.load()
    h = ctypes.c_void_p()
    o = _lib.Options()
    L.podcg_default_options(ctypes.byref(o))
    assert L.podcg_create(ctypes.byref(h), 0, ctypes.byref(o), None) == _lib.ERR_INVALID_ARG
    o.omega = 33
    assert L.podcg_create(ctypes.byref(h), 10, ctypes.byref(o), None) == _lib.ERR_INVALID_ARG
    assert L.podcg_destroy(None) == 0


def test_batch_defaults_and_argument_checks_without_gpu():
    from paper_1512_05820_amd import _lib
    L = _lib.load()
    o = _lib.BatchOptions()
    L.podcg_batch_default_options(ctypes.byref(o))
    assert o.as_dict() == {"slices_per_item": 8, "rows_per_item": 2048, "grid": 1024,
                           "graph_iters": 16, "check_every": 16}
    h = ctypes.c_void_p()
    assert L.podcg_batch_create(ctypes.byref(h), 0, None, None) == _lib.ERR_INVALID_ARG
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.podcg_batch_create(ctypes.byref(h), 2, arr, None) == _lib.ERR_INVALID_ARG
    assert L.podcg_batch_destroy(None) == 0
