"""Host-side checks of the C ABI (no GPU needed, no device compute).

The library must load, export every function include/bfc.h declares, and
answer the pure host queries (status strings, sizes, argument errors).
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bfc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1801_00338_amd import _lib
    return _lib.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "bfc_exact" in names and "bfc_graph_build" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_1801_00338_amd import _lib
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def test_status_strings(lib):
    assert lib.bfc_status_str(0) == b"ok"
    assert b"duplicate" in lib.bfc_status_str(-4)
    assert lib.bfc_status_str(12345) == b"unknown status"


def test_size_queries_and_limits(lib):
    sz = C.c_size_t()
    assert lib.bfc_graph_storage_size(10, 20, 30, C.byref(sz)) == 0
    # 4 * (11 + 3*30 + 2*10 + 21 + 3*30 + 2*20) bytes at least
    assert sz.value >= 4 * (11 + 90 + 20 + 21 + 90 + 40)
    assert lib.bfc_graph_storage_size(10, 20, 30, None) == -1
    assert lib.bfc_graph_storage_size(2, 2, 5, C.byref(sz)) == -4      # m > |L||R|
    assert lib.bfc_graph_storage_size(0xFFFFFFFF, 2, 5, C.byref(sz)) == -5
    assert lib.bfc_graph_build_ws_size(1000, 1000, 5000, C.byref(sz)) == 0
    assert sz.value > 0


def test_null_arguments_rejected(lib):
    from paper_1801_00338_amd import _lib
    g = _lib.bfc_graph()
    assert lib.bfc_exact(None, 0, None, None, 0, None) == -1
    assert lib.bfc_side_used(C.byref(g), 9) == -2
    assert lib.bfc_local(C.byref(g), None, None, None, None, 0, None) == -1
