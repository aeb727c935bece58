"""The C-ABI library loads and exports every symbol include/mcd.h declares;
the Python binding names the same calls.  No compute calls (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcd.h")
LIB = os.path.join(ROOT, "paper_2404_17542_amd", "libmcd.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcd_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    syms = declared_symbols()
    for name in ("mcd_build_stencils", "mcd_apply", "mcd_solve_ppe", "mcd_update_dps", "mcd_create",
                 "mcd_destroy", "mcd_sync", "mcd_last_error"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2404_17542_amd import mcd
    assert sorted(mcd.EXPORTED) == declared_symbols()


def test_struct_layouts_match_header_sizes():
    """Field order/size of the ctypes mirrors (checked against sizeof in C)."""
    from paper_2404_17542_amd import mcd
    assert ctypes.sizeof(mcd.MeshDesc) == 4 + 12 + 4 + 24 + 8 + 12 + 4 + 4
    assert ctypes.sizeof(mcd.WideInfo) == 3 * 4 + 4 + 3 * 8             # padding before the doubles
    assert ctypes.sizeof(mcd.Body) == 8 + 24 + 8 + 4 * 24 + 8 + 24 + 8 + 16 + 24 + 8   # sdf_n[3] padded to 16
    assert ctypes.sizeof(mcd.BcTable) == 4 * 17
    assert ctypes.sizeof(mcd.Params) == 8 + 7 * 8          # weight_kind padded to 8, then 7 doubles
    assert ctypes.sizeof(mcd.Tuning) == 4 + 4 * 32 + 4 * 32 + 4 + 8 * 32 + 4 + 4   # padding before the doubles and at the end
    assert ctypes.sizeof(mcd.SolveOpts) == 8 + 3 * 4 + 4 + 8 + 3 * 4 + 4 + 8 + 4 + 4  # with the alignment pads
