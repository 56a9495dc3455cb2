"""The C-ABI library loads and exports every symbol the header declares;
host-side argument checks work without a GPU (no compute calls here)."""
import ctypes
import os

import pytest

from paper_2405_12871_amd import binding


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2405_12871_amd import build
        build.build()
    return binding.load()


def test_header_declares_the_boundary():
    names = binding.header_functions()
    for required in ("imin_graph_create", "imin_graph_destroy", "imin_graph_info", "imin_solve",
                     "imin_solve_workspace_size", "imin_evaluate", "imin_status_string", "imin_last_device_flags"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in binding.header_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in range(7):
        s = lib.imin_status_string(code)
        assert s and s.decode() != "unknown status"
    assert lib.imin_status_string(99).decode() == "unknown status"


def test_host_argument_checks(lib):
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: rejected before use
    # n out of range, negative m, NULL outputs
    assert lib.imin_graph_create(0, 0, dummy, None, None, None, ctypes.byref(h)) == 1
    assert lib.imin_graph_create(1 << 24, 0, dummy, None, None, None, ctypes.byref(h)) == 1
    assert lib.imin_graph_create(5, -1, dummy, None, None, None, ctypes.byref(h)) == 1
    assert lib.imin_graph_create(5, 3, dummy, None, None, None, ctypes.byref(h)) == 1
    assert lib.imin_graph_create(5, 0, None, None, None, None, ctypes.byref(h)) == 1
    assert lib.imin_graph_create(5, 0, dummy, None, None, None, None) == 1
    # NULL graph handles
    assert lib.imin_solve(None, dummy, 1, 1, 10, 0, None, 0, None, dummy, dummy, dummy, dummy, None) == 1
    assert lib.imin_solve(None, dummy, 1, 1, 10, 0, dummy, 1 << 20, None, dummy, dummy, dummy, dummy, dummy) == 1
    nbytes = ctypes.c_size_t()
    assert lib.imin_solve_workspace_size(None, 1, 1, 10, ctypes.byref(nbytes)) == 1
    assert lib.imin_evaluate(None, dummy, 1, None, 0, 0, 10, 0, None, dummy, dummy, None, None, None) == 1
    assert lib.imin_graph_info(None, None, None) == 1
    # imin_evaluate_batch: NULL graph, negative count, NULL queries; an empty
    # batch does nothing
    eq = (binding.EvalQuery * 1)()
    assert lib.imin_evaluate_batch(None, eq, 1, None) == 1
    assert lib.imin_evaluate_batch(dummy, eq, -1, None) == 1
    assert lib.imin_evaluate_batch(dummy, None, 1, None) == 1
    assert lib.imin_evaluate_batch(dummy, None, 0, None) == 0
    # imin_solve_many: NULL graph, no stream, a stream named twice, bad counts
    q = (binding.Query * 1)()
    s1 = (ctypes.c_void_p * 2)(0x10, 0x20)
    s2 = (ctypes.c_void_p * 2)(0x10, 0x10)
    assert lib.imin_solve_many(None, q, 1, s1, 2, 0) == 1
    assert lib.imin_solve_many(dummy, q, 1, s1, 0, 0) == 1
    assert lib.imin_solve_many(dummy, q, 1, None, 1, 0) == 1
    assert lib.imin_solve_many(dummy, q, 1, s2, 2, 0) == 1
    assert lib.imin_solve_many(dummy, q, -1, s1, 2, 0) == 1
    assert lib.imin_solve_many(dummy, None, 1, s1, 2, 0) == 1
    # server: NULL graph / streams / output, no stream, a stream named twice;
    # NULL server handles
    hs = ctypes.c_void_p()
    assert lib.imin_server_create(None, s1, 2, 0, ctypes.byref(hs)) == 1
    assert lib.imin_server_create(dummy, None, 2, 0, ctypes.byref(hs)) == 1
    assert lib.imin_server_create(dummy, s1, 0, 0, ctypes.byref(hs)) == 1
    assert lib.imin_server_create(dummy, s2, 2, 0, ctypes.byref(hs)) == 1
    assert lib.imin_server_create(dummy, s1, 2, 0, None) == 1
    assert lib.imin_server_submit(None, q) == 1
    assert lib.imin_server_next(None, ctypes.byref(ctypes.POINTER(binding.Query)())) == 1
    assert lib.imin_server_destroy(None) == 0
    assert lib.imin_graph_destroy(None) == 0
