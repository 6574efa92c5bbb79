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


def _opt(acx, **kw):
    o = acx.Options()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


@pytest.mark.parametrize("field,value", [
    ("reserved", 1), ("wave_tile", 64), ("capacity_hint", 8), ("profile", -1), ("profile", 99),
    ("cell_mA", -5), ("force_exact", 2), ("vertex_shortcut", -1), ("cell_order", 2),
])
def test_options_out_of_range_are_rejected_before_device_work(field, value):
    """Every ac_options field outside its documented range is AC_E_INVALID,
    reported before any device call (so this runs without a GPU), on every
    entry point that takes options."""
    import paper_1908_05944_amd as acx
    lib = acx.library()
    o = _opt(acx, **{field: value})
    out = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)  # never dereferenced: the options are checked first
    xyz = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    rad = (ctypes.c_double * 1)(1.5)
    off = (ctypes.c_int64 * 2)(0, 1)
    alphas = (ctypes.c_double * 1)(0.0)
    outs = (ctypes.c_void_p * 1)()
    cells = (ctypes.c_int32 * 1)()
    calls = [
        lambda: lib.ac_alpha_complex(xyz, rad, 1, 0.0, ctypes.byref(o), ctypes.byref(out)),
        lambda: lib.ac_alpha_complex_device(dummy, dummy, 1, 0.0, ctypes.byref(o), None, ctypes.byref(out)),
        lambda: lib.ac_alpha_complex_partitioned(dummy, dummy, 1, 0.0, 2, ctypes.byref(o), None, ctypes.byref(out)),
        lambda: lib.ac_alpha_complex_partitioned_host(xyz, rad, 1, 0.0, 2, ctypes.byref(o), ctypes.byref(out)),
        lambda: lib.ac_alpha_sweep_device(dummy, dummy, 1, alphas, 1, ctypes.byref(o), None, outs),
        lambda: lib.ac_alpha_complex_batch(dummy, dummy, off, 1, 0.0, ctypes.byref(o), None, None, ctypes.byref(out)),
        lambda: lib.ac_tune_cells(dummy, dummy, off, 1, 0.0, ctypes.byref(o), None, cells, None),
    ]
    for k, call in enumerate(calls):
        assert call() == 1, (field, value, k)
        assert b"ac_options." + field.encode() in lib.ac_last_error(), (k, lib.ac_last_error())
    assert not out.value


def test_options_layout_matches_the_header():
    """The binding's ac_options has the header's fields, in order."""
    import paper_1908_05944_amd as acx
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = text[text.index("typedef struct {"):text.index("} ac_options;")]
    fields = re.findall(r"\b(?:int32_t|int64_t)\s+([A-Za-z_]+)\s*;", body)
    assert fields == [f for f, _ in acx.Options._fields_]


def test_host_streamed_input_checks_without_device():
    """The host-streamed build checks its x coordinates, radii, slab count and
    alpha on the host before any device work."""
    import paper_1908_05944_amd as acx
    lib = acx.library()
    out = ctypes.c_void_p()
    xyz = (ctypes.c_double * 6)(0.0, 0.0, 0.0, float("nan"), 1.0, 1.0)
    rad = (ctypes.c_double * 2)(1.5, 1.5)
    assert lib.ac_alpha_complex_partitioned_host(xyz, rad, 2, 0.0, 2, None, ctypes.byref(out)) == 1
    xyz[3] = 600.0
    assert lib.ac_alpha_complex_partitioned_host(xyz, rad, 2, 0.0, 2, None, ctypes.byref(out)) == 3
    xyz[3] = 2.0
    for parts in (0, 1025):
        assert lib.ac_alpha_complex_partitioned_host(xyz, rad, 2, 0.0, parts, None, ctypes.byref(out)) == 1
    assert lib.ac_alpha_complex_partitioned_host(xyz, rad, 2, float("inf"), 2, None, ctypes.byref(out)) == 1
    rad[1] = 0.0
    assert lib.ac_alpha_complex_partitioned_host(xyz, rad, 2, 0.0, 2, None, ctypes.byref(out)) == 1
    assert not out.value


def test_molecule_accessors_without_a_result():
    import paper_1908_05944_amd as acx
    lib = acx.library()
    assert not lib.ac_molecule(None, 0)
    assert not lib.ac_molecule_rows(None, 0)
    assert lib.ac_molecule_count(None) == -1


def test_measure_rejects_null_complex_without_device():
    import paper_1908_05944_amd as acx
    lib = acx.library()
    V, A = ctypes.c_double(), ctypes.c_double()
    dummy = ctypes.c_void_p(16)
    assert lib.ac_union_measure(None, dummy, dummy, 1, ctypes.byref(V), ctypes.byref(A), None) == 1


def test_noalloc_argument_checks_without_device():
    """Argument errors of the build without allocation are reported before
    any device work (and before its scratch is touched)."""
    import paper_1908_05944_amd as acx
    lib = acx.library()
    caps = (ctypes.c_int64 * 4)(10, 10, 10, 10)
    ptrs = (ctypes.c_void_p * 4)(8, 8, 8, 8)  # never dereferenced: every call below fails its checks first
    counts = (ctypes.c_int64 * 4)()
    fake = ctypes.c_void_p(8)
    assert lib.ac_alpha_complex_noalloc(fake, fake, 10, 0.0, None, None, None, ptrs, caps, counts) == 1
    assert lib.ac_alpha_complex_noalloc(fake, fake, 10, 0.0, None, None, ptrs, ptrs, caps, None) == 1
    assert lib.ac_alpha_complex_noalloc(None, None, 10, 0.0, None, None, ptrs, ptrs, caps, counts) == 1
    assert list(counts) == [-1] * 4
    o = acx.Options()
    o.profile = 1
    assert lib.ac_alpha_complex_noalloc(fake, fake, 10, 0.0, ctypes.byref(o), None, ptrs, ptrs, caps, counts) == 1
    bad = (ctypes.c_int64 * 4)(10, -1, 10, 10)
    assert lib.ac_alpha_complex_noalloc(fake, fake, 10, 0.0, None, None, ptrs, ptrs, bad, counts) == 1
    nulls = (ctypes.c_void_p * 4)(8, None, 8, 8)
    assert lib.ac_alpha_complex_noalloc(fake, fake, 10, 0.0, None, None, nulls, ptrs, caps, counts) == 1
    assert lib.ac_alpha_complex_noalloc(fake, fake, 0, 0.0, None, None, ptrs, ptrs, caps, counts) == 1
    # more balls than the fixed scratch can hold: refused up front
    too_many = (256 << 20) // 128 + 1
    assert lib.ac_alpha_complex_noalloc(fake, fake, too_many, 0.0, None, None, ptrs, ptrs, caps, counts) == 6
    assert b"scratch" in lib.ac_last_error()


def test_plan_argument_checks_without_device():
    """Argument errors of the recorded batch build are reported before any
    device work; the plan accessors take NULL."""
    import paper_1908_05944_amd as acx
    lib = acx.library()
    fake = ctypes.c_void_p(8)
    off = (ctypes.c_int64 * 3)(0, 5, 10)
    h = ctypes.c_void_p()
    assert lib.ac_plan_create(fake, fake, off, 2, 0.0, None, None, 1.25, None, None) == 1
    assert lib.ac_plan_create(None, None, off, 2, 0.0, None, None, 1.25, None, ctypes.byref(h)) == 1
    assert lib.ac_plan_create(fake, fake, off, 2, 0.0, None, None, 0.5, None, ctypes.byref(h)) == 1
    assert lib.ac_plan_create(fake, fake, off, 2, 0.0, None, None, 17.0, None, ctypes.byref(h)) == 1
    assert lib.ac_plan_create(fake, fake, off, 2, float("inf"), None, None, 1.25, None, ctypes.byref(h)) == 1
    bad = (ctypes.c_int64 * 3)(0, 5, 5)
    assert lib.ac_plan_create(fake, fake, bad, 2, 0.0, None, None, 1.25, None, ctypes.byref(h)) == 1
    o = acx.Options()
    o.profile = 1
    assert lib.ac_plan_create(fake, fake, off, 2, 0.0, ctypes.byref(o), None, 1.25, None, ctypes.byref(h)) == 1
    assert not h
    assert lib.ac_plan_launch(None, None) == 1
    assert lib.ac_plan_result(None, None, ctypes.byref(h)) == 1
    assert lib.ac_plan_stopped(None) == -1
    assert lib.ac_plan_ordinary_builds(None) == -1
    lib.ac_plan_free(None)
