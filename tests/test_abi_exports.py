"""The C ABI library loads and exports every function include/iim.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iim.h")
LIB = os.path.join(ROOT, "paper_2503_22455_amd", "libiim.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(iim_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_abi():
    names = declared_functions()
    for must in ("iim_create", "iim_destroy", "iim_solve", "iim_apply", "iim_vcycle", "iim_set_rhs",
                 "iim_set_boundary_data", "iim_control_points", "iim_last_error"):
        assert must in names


def test_library_exports_every_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libiim.so not built in this checkout")
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
