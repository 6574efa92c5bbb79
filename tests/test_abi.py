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
    for must in ("ac_alpha_complex", "ac_alpha_complex_device", "ac_alpha_sweep_device", "ac_count", "ac_simplices",
                 "ac_sizes", "ac_free", "ac_status_str", "ac_last_error"):
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


def test_sweep_argument_checks_without_device():
    """Argument errors of the sweep are reported before any device work."""
    import paper_1908_05944_amd as acx
    lib = acx.library()
    outs = (ctypes.c_void_p * 4)()
    alphas = (ctypes.c_double * 4)(0.0, 1.0, 2.0, 3.0)
    # no value, too many values, NULL inputs, NULL output array
    assert lib.ac_alpha_sweep_device(None, None, 10, alphas, 0, None, None, outs) == 1
    assert lib.ac_alpha_sweep_device(None, None, 10, alphas, 1025, None, None, outs) == 1
    assert lib.ac_alpha_sweep_device(None, None, 10, alphas, 4, None, None, outs) == 1
    assert all(h is None for h in outs)
    assert lib.ac_alpha_sweep_device(None, None, 10, alphas, 4, None, None, None) == 1
    assert b"NULL" in lib.ac_last_error() or b"null" in lib.ac_last_error().lower()
