"""The C-ABI library loads on the CPU and exports every entry point that
include/ftree.h declares (no compute call: that needs a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ftree.h")
LIB = os.path.join(ROOT, "paper_1910_04126_amd", "libftree.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ft_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libftree.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_four_calls():
    names = declared()
    for n in ("ft_build_tree", "ft_quadtree_knn", "ft_flowtree_knn", "ft_flowtree_cost_grad"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (ft_[a-z_]+)", out))
    assert set(declared()) <= exported


def test_last_error_is_empty_string(lib):
    lib.ft_last_error.restype = ctypes.c_char_p
    assert lib.ft_last_error() == b""


def test_null_arguments_fail_cleanly(lib):
    """Argument checks that run before any device call."""
    lib.ft_build_tree.restype = ctypes.c_int
    out = ctypes.c_void_p()
    rc = lib.ft_build_tree(None, ctypes.c_int64(10), ctypes.c_int32(2), None, ctypes.c_int32(30),
                           None, None, None, ctypes.c_int64(1), ctypes.c_int32(24), None, ctypes.byref(out))
    assert rc == -1
    lib.ft_last_error.restype = ctypes.c_char_p
    assert b"NULL" in lib.ft_last_error()
    lib.ft_index_info.restype = ctypes.c_int
    assert lib.ft_index_info(None, None) == -1
    lib.ft_act_pairs.restype = ctypes.c_int
    assert lib.ft_act_pairs(None, None, None, None, ctypes.c_int64(0), None, None, ctypes.c_int64(0),
                            ctypes.c_int32(1), None, None) == -1
    lib.ft_act_knn.restype = ctypes.c_int
    assert lib.ft_act_knn(None, None, None, None, ctypes.c_int64(0), None, ctypes.c_int32(0), ctypes.c_int32(1),
                          ctypes.c_int32(1), None, None, None) == -1
    lib.ft_free(None)


def test_python_binding_imports_without_gpu():
    import paper_1910_04126_amd as ft
    ft.load()
    assert callable(ft.flowtree_knn) and callable(ft.build_tree)
