"""The C-ABI library loads and exports every entry point include/tnmh.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tnmh.h")
LIB = os.path.join(ROOT, "paper_2104_13264_amd", "libtnmh.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tn_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["tn_create", "tn_destroy", "tn_last_error", "tn_build_env", "tn_sample",
              "tn_eval_logq", "tn_mh_step", "tn_grad", "tn_stats", "tn_set_env",
              "tn_get_env", "tn_set_precision", "tn_set_instance"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libtnmh.so not built")
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert missing == []


def test_binding_lists_the_same_symbols():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "tnmh_binding", os.path.join(ROOT, "paper_2104_13264_amd", "tnmh.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert sorted(mod.exported_symbols()) == declared()


def test_null_context_is_rejected_without_a_device():
    if not os.path.exists(LIB):
        pytest.skip("libtnmh.so not built")
    L = ctypes.CDLL(LIB)
    L.tn_destroy.argtypes = [ctypes.c_void_p]
    L.tn_last_error.restype = ctypes.c_char_p
    L.tn_last_error.argtypes = [ctypes.c_void_p]
    L.tn_sample.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                            ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert L.tn_destroy(None) == 0
    assert L.tn_last_error(None) == b"NULL context"
    assert L.tn_sample(None, 1, 0, 0, 0, None, None, None) == -1
