"""The C ABI library loads and exports every function include/alphacx.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "alphacx.h")
SO = os.path.join(ROOT, "paper_1908_05944_amd", "libalphacx.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ac_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ac_alpha_complex", "ac_alpha_complex_device", "ac_count", "ac_simplices", "ac_sizes",
                 "ac_free", "ac_status_str", "ac_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(SO):
        pytest.fail("libalphacx.so is not built; run __graft_entry__.build()")
    import torch  # noqa: F401  (shares the HIP runtime soname with the library)
    lib = ctypes.CDLL(SO)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_without_device():
    import paper_1908_05944_amd as acx
    lib = acx.library()
    for st in range(7):
        assert lib.ac_status_str(st)
    assert lib.ac_count(None, 0) == -1
    assert lib.ac_count(None, 9) == -1
