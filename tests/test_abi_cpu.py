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
    # the variant and intermediate-bound entry points check their handles first
    vp = ctypes.c_void_p
    lib.gcp_bound_pi.argtypes = [vp, vp, ctypes.c_double, vp, ctypes.c_int32] + [vp] * 6 + [ctypes.c_int32] + \
        [vp] * 7
    assert lib.gcp_bound_pi(None, None, 0.0, None, 1, *([None] * 6), 0, *([None] * 7)) == -1
    lib.gcp_crown_bounds_domain.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int32, vp, vp, vp, vp, vp,
                                            ctypes.c_int32, vp]
    assert lib.gcp_crown_bounds_domain(None, None, 0.1, 0, None, None, None, None, None, 0, None) == -1
    assert b"network" in lib.gcp_last_error()


def test_shipped_tile_choices_are_well_formed():
    # bench.py starts from these autotuner choices; each line is
    # "<family>.k<epilogue>.b<bf16>.s<sign>.M<m>.N<n>.K<k> <config>" with a
    # config index the family's launcher accepts (8 dense tiles, 6 conv shapes,
    # and 6 = the direct kernel for the concretisation's transposed conv, k2)
    import re
    path = os.path.join(os.path.dirname(LIB), "tuned_tiles_gfx950.txt")
    pat = re.compile(r"^(gemm|conv|convT)\.k([0-4])\.b([01])\.s([01])\.M(\d+)\.N(\d+)\.K(\d+) (\d+)$")
    n = 0
    with open(path) as f:
        for line in f:
            m = pat.match(line.strip())
            assert m, line
            cfg = int(m.group(8))
            direct = m.group(1) == "convT" and m.group(2) == "2" and cfg == 6
            assert direct or 0 <= cfg < (8 if m.group(1) == "gemm" else 6), line
            n += 1
    assert n > 0
