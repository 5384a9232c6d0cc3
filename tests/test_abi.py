"""The C ABI: every function declared in include/rqrcp.h is exported by the
built library, and argument errors are reported without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rqrcp.h")
LIB = os.path.join(ROOT, "paper_1804_05138_amd", "librqrcp.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:rqrcp|srqr)_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("rqrcp_factor", "rqrcp_sketch", "rqrcp_gaussian", "rqrcp_form_q",
              "rqrcp_workspace_size", "rqrcp_create", "rqrcp_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_every_declared_symbol():
    import paper_1804_05138_amd as rq
    assert sorted(rq.EXPORTS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_argument_checks_without_gpu():
    import paper_1804_05138_amd as rq
    lib = rq.load_library()
    out = ctypes.c_size_t()
    prm = rq.Params(32, 8, 0, rq.F64, rq.F64, 0)
    assert lib.rqrcp_workspace_size(100, 80, 20, ctypes.byref(prm), ctypes.byref(out)) == 0
    assert out.value > 0
    assert lib.rqrcp_workspace_size(0, 80, 20, ctypes.byref(prm), ctypes.byref(out)) == -1
    assert lib.rqrcp_workspace_size(100, 0, 20, ctypes.byref(prm), ctypes.byref(out)) == -2
    assert lib.rqrcp_workspace_size(100, 80, 81, ctypes.byref(prm), ctypes.byref(out)) == -3
    assert lib.rqrcp_workspace_size(100, 80, 0, ctypes.byref(prm), ctypes.byref(out)) == -3
    bad = rq.Params(0, 8, 0, rq.F64, rq.F64, 0)
    assert lib.rqrcp_workspace_size(100, 80, 20, ctypes.byref(bad), ctypes.byref(out)) == -4
    assert lib.rqrcp_factor(None, 10, 10, 5, ctypes.byref(prm), None, 10, None, None, None, 40,
                            None, None, 0) == -1
    for bad_types in ((7, rq.F64), (rq.F64, rq.F32), (rq.F32, 9)):
        bp = rq.Params(32, 8, 0, bad_types[0], bad_types[1], 0)
        assert lib.rqrcp_workspace_size(100, 80, 20, ctypes.byref(bp), ctypes.byref(out)) == -4
    for good in ((rq.F32, rq.F64), (rq.F32, rq.BF16), (rq.F32, rq.F8E4M3), (rq.F64, rq.BF16)):
        gp = rq.Params(32, 8, 0, good[0], good[1], 0)
        assert lib.rqrcp_workspace_size(100, 80, 20, ctypes.byref(gp), ctypes.byref(out)) == 0
    sw = ctypes.c_size_t()
    assert lib.srqr_workspace_size(100, 80, 20, ctypes.byref(prm), 16, 0, ctypes.byref(sw)) == 0
    assert sw.value > 0
    assert lib.srqr_workspace_size(100, 80, 80, ctypes.byref(prm), 16, 0, ctypes.byref(sw)) == -3
    assert lib.srqr_workspace_size(100, 80, 20, ctypes.byref(prm), 0, 0, ctypes.byref(sw)) == -5
    assert lib.srqr_workspace_size(100, 80, 20, ctypes.byref(prm), 0, rq.SRQR_EXACT,
                                   ctypes.byref(sw)) == 0
    assert lib.rqrcp_status_string(1002) == b"workspace too small"
    assert lib.rqrcp_status_string(-3) == b"invalid argument"


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_workspace_grows_with_the_problem():
    import paper_1804_05138_amd as rq
    small = rq.workspace_bytes(1024, 1024, 64, 32, 8)
    big = rq.workspace_bytes(16384, 16384, 1024, 64, 8)
    assert big > small
    assert rq.workspace_bytes(300, 200, 50, 16, 8, rq.FROZEN_PIVOTS) > rq.workspace_bytes(300, 200, 50, 16, 8)
