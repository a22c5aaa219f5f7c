"""The C-ABI library loads and exports every function include/gss.h declares (CPU only:
no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gss.h")
LIB = os.path.join(ROOT, "paper_2508_20403_amd", "libgss.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gss_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("gss_ctx_create", "gss_tree_prep", "gss_recover", "gss_tree_free", "gss_ctx_destroy"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgss.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgss.so not built")
def test_binding_lists_the_header():
    from paper_2508_20403_amd import gss
    assert sorted(gss.EXPORTS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgss.so not built")
def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.gss_status_str.restype = ctypes.c_char_p
    lib.gss_status_str.argtypes = [ctypes.c_int32]
    assert lib.gss_status_str(0) == b"GSS_OK"
    assert lib.gss_status_str(-7) == b"GSS_ERR_RANGE"
