"""CPU checks of the C ABI: the library loads and exports every entry point
declared in include/gcp.h (no compute call is made without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gcp.h")
LIB = os.path.join(ROOT, "paper_2208_05740_amd", "libgcp.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gcp_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["gcp_net_create", "gcp_net_destroy", "gcp_cuts_create", "gcp_splits_create",
              "gcp_bound", "gcp_optimize", "gcp_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n
    lib.gcp_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.gcp_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_arguments_are_rejected_without_a_device():
    lib = ctypes.CDLL(LIB)
    lib.gcp_last_error.restype = ctypes.c_char_p
    assert lib.gcp_net_create(None, None) == -1
    assert lib.gcp_net_get_info(None, None) == -1
    assert lib.gcp_last_error()
