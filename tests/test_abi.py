"""The C-ABI library loads and exports every entry point include/mf.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mf.h")
LIB = os.path.join(ROOT, "paper_1810_02821_amd", "libmf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(mf_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("mf_plan_create", "mf_plan_destroy", "mf_wiener", "mf_sample",
                     "mf_wiener_backward", "mf_status_string", "mf_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmf.so not built")
def test_status_strings_and_error_paths_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.mf_status_string.restype = ctypes.c_char_p
    lib.mf_last_error.restype = ctypes.c_char_p
    assert lib.mf_status_string(0) == b"ok"
    assert lib.mf_status_string(5) == b"not converged"
    # invalid arguments are rejected before any device call
    assert lib.mf_plan_create(None, 1, None, 0, None) == 1
    assert b"NULL" in lib.mf_last_error()
    h = ctypes.c_void_p()
    assert lib.mf_plan_create(ctypes.byref(h), 0, None, 0, None) == 1
    assert lib.mf_plan_destroy(None) == 0


def test_binding_exposes_the_same_names():
    from paper_1810_02821_amd import _binding
    for name in declared_functions():
        assert name in _binding.EXPORTS or name in ("mf_status_string", "mf_last_error")
