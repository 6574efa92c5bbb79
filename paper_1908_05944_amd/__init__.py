"""alphacx for MI355X: Python binding of libalphacx.so (argument marshalling only).

Every step of the computation runs in the HIP kernels of libalphacx.so; this
module only converts arguments and results. It fails loudly when the library
is missing: there is no CPU fallback.

Names follow the C ABI in include/alphacx.h:
    ac_alpha_complex(xyz, radii, alpha, options=None)          host arrays in, host arrays out
    ac_alpha_complex_device(xyz, radii, alpha, options=None,   torch device tensors in,
                            stream=None)                        results kept on the device
Both return an `AlphaComplex` owning the library's result handle.

    ac_alpha_complex_batch(xyz, radii, offsets, alpha,        many molecules in one call (device
                           options=None, cell_mA=None)          tensors, host offsets)
    ac_tune_cells(xyz, radii, offsets, alpha)                   per-molecule cell sides (autotuner)
    ac_union_measure(c, xyz, radii)                   V, A of the union of the balls (host floats)
    ac_union_measure_device(c, xyz, radii)            the same as a device tensor [V, A]
    ac_union_measure_backward(c, xyz, radii, grad)    d(gV V + gA A)/d(xyz, radii), device tensors
    UnionMeasure.apply(xyz, radii, c)                 torch.autograd.Function over the two
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
_SO = os.path.join(_HERE, "libalphacx.so")
_SRC = os.path.join(_HERE, "csrc", "alphacx.hip")
_INC = os.path.join(_ROOT, "include")
_lib = None

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

STATUS = {0: "ok", 1: "invalid argument", 2: "duplicate centres", 3: "out of range", 4: "out of memory",
          5: "HIP device error", 6: "capacity exceeded"}


class AlphaCxError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        super().__init__(f"alphacx: {STATUS.get(status, status)}" + (f" ({detail})" if detail else ""))
        self.status = status
        self.detail = detail


def build() -> str:
    """Compile libalphacx.so for gfx950 with hipcc (always rebuilds)."""
    tmp = _SO + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, f"-I{_INC}", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class Options(ctypes.Structure):
    """ac_options: zero fields select the defaults; none changes the result."""
    _fields_ = [
        ("cell_mA", ctypes.c_int32),
        ("wave_tile", ctypes.c_int32),
        ("force_exact", ctypes.c_int32),
        ("vertex_shortcut", ctypes.c_int32),
        ("capacity_hint", ctypes.c_int64),
        ("profile", ctypes.c_int32),
        ("cell_order", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # The HIP runtime must be the one torch already uses (same soname), so
    # torch is imported first.
    import torch  # noqa: F401
    if not os.path.exists(_SO):
        raise RuntimeError(f"libalphacx.so is not built ({_SO}); run __graft_entry__.build()")
    lib = ctypes.CDLL(_SO)
    c_p, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    lib.ac_alpha_complex.argtypes = [c_p, c_p, i64, dbl, ctypes.POINTER(Options), ctypes.POINTER(c_p)]
    lib.ac_alpha_complex.restype = ctypes.c_int
    lib.ac_alpha_complex_device.argtypes = [c_p, c_p, i64, dbl, ctypes.POINTER(Options), c_p, ctypes.POINTER(c_p)]
    lib.ac_alpha_complex_device.restype = ctypes.c_int
    lib.ac_alpha_complex_noalloc.argtypes = [c_p, c_p, i64, dbl, ctypes.POINTER(Options), c_p, c_p, c_p, c_p, c_p]
    lib.ac_alpha_complex_noalloc.restype = ctypes.c_int
    lib.ac_plan_create.argtypes = [c_p, c_p, c_p, i64, dbl, ctypes.POINTER(Options), c_p, dbl, c_p,
                                   ctypes.POINTER(c_p)]
    lib.ac_plan_create.restype = ctypes.c_int
    lib.ac_plan_launch.argtypes = [c_p, c_p]
    lib.ac_plan_launch.restype = ctypes.c_int
    lib.ac_plan_result.argtypes = [c_p, c_p, ctypes.POINTER(c_p)]
    lib.ac_plan_result.restype = ctypes.c_int
    lib.ac_plan_stopped.argtypes = [c_p]
    lib.ac_plan_stopped.restype = ctypes.c_int32
    lib.ac_plan_ordinary_builds.argtypes = [c_p]
    lib.ac_plan_ordinary_builds.restype = i64
    lib.ac_plan_free.argtypes = [c_p]
    lib.ac_plan_free.restype = None
    lib.ac_alpha_sweep_device.argtypes = [c_p, c_p, i64, ctypes.POINTER(dbl), i64, ctypes.POINTER(Options), c_p,
                                          ctypes.POINTER(c_p)]
    lib.ac_alpha_sweep_device.restype = ctypes.c_int
    lib.ac_alpha_complex_partitioned.argtypes = [c_p, c_p, i64, dbl, ctypes.c_int32, ctypes.POINTER(Options), c_p,
                                                 ctypes.POINTER(c_p)]
    lib.ac_alpha_complex_partitioned.restype = ctypes.c_int
    lib.ac_alpha_complex_partitioned_host.argtypes = [c_p, c_p, i64, dbl, ctypes.c_int32, ctypes.POINTER(Options),
                                                      ctypes.POINTER(c_p)]
    lib.ac_alpha_complex_partitioned_host.restype = ctypes.c_int
    lib.ac_count.argtypes = [c_p, ctypes.c_int]
    lib.ac_count.restype = i64
    lib.ac_simplices.argtypes = [c_p, ctypes.c_int]
    lib.ac_simplices.restype = ctypes.POINTER(ctypes.c_int32)
    lib.ac_sizes.argtypes = [c_p, ctypes.c_int]
    lib.ac_sizes.restype = ctypes.POINTER(ctypes.c_double)
    lib.ac_simplices_device.argtypes = [c_p, ctypes.c_int]
    lib.ac_simplices_device.restype = c_p
    lib.ac_sizes_device.argtypes = [c_p, ctypes.c_int]
    lib.ac_sizes_device.restype = c_p
    lib.ac_candidate_count.argtypes = [c_p, ctypes.c_int]
    lib.ac_candidate_count.restype = i64
    lib.ac_exact_fallbacks.argtypes = [c_p]
    lib.ac_exact_fallbacks.restype = i64
    lib.ac_work_count.argtypes = [c_p, ctypes.c_int]
    lib.ac_work_count.restype = i64
    lib.ac_stage_count.argtypes = []
    lib.ac_stage_count.restype = ctypes.c_int
    lib.ac_stage_name.argtypes = [ctypes.c_int]
    lib.ac_stage_name.restype = ctypes.c_char_p
    lib.ac_stage_ms.argtypes = [c_p, ctypes.c_int]
    lib.ac_stage_ms.restype = ctypes.c_double
    lib.ac_free.argtypes = [c_p]
    lib.ac_free.restype = None
    lib.ac_release_workspace.argtypes = []
    lib.ac_release_workspace.restype = ctypes.c_int
    lib.ac_status_str.argtypes = [ctypes.c_int]
    lib.ac_status_str.restype = ctypes.c_char_p
    lib.ac_last_error.argtypes = []
    lib.ac_last_error.restype = ctypes.c_char_p
    lib.ac_alpha_complex_batch.argtypes = [c_p, c_p, c_p, i64, dbl, ctypes.POINTER(Options), c_p, c_p,
                                           ctypes.POINTER(c_p)]
    lib.ac_alpha_complex_batch.restype = ctypes.c_int
    lib.ac_molecule_count.argtypes = [c_p]
    lib.ac_molecule_count.restype = i64
    lib.ac_molecule_rows.argtypes = [c_p, ctypes.c_int]
    lib.ac_molecule_rows.restype = ctypes.POINTER(i64)
    lib.ac_molecule.argtypes = [c_p, ctypes.c_int]
    lib.ac_molecule.restype = ctypes.POINTER(ctypes.c_int32)
    lib.ac_tune_cells.argtypes = [c_p, c_p, c_p, i64, dbl, ctypes.POINTER(Options), c_p, c_p, c_p]
    lib.ac_tune_cells.restype = ctypes.c_int
    lib.ac_union_measure.argtypes = [c_p, c_p, c_p, i64, ctypes.POINTER(dbl), ctypes.POINTER(dbl), c_p]
    lib.ac_union_measure.restype = ctypes.c_int
    lib.ac_union_measure_device.argtypes = [c_p, c_p, c_p, i64, c_p, c_p]
    lib.ac_union_measure_device.restype = ctypes.c_int
    lib.ac_union_measure_backward.argtypes = [c_p, c_p, c_p, i64, c_p, c_p, c_p, c_p]
    lib.ac_union_measure_backward.restype = ctypes.c_int
    lib.ac_union_measure_fused.argtypes = [c_p, c_p, c_p, i64, c_p, c_p, c_p, c_p, c_p]
    lib.ac_union_measure_fused.restype = ctypes.c_int
    _lib = lib
    return lib


def library():
    """The loaded ctypes handle of libalphacx.so."""
    return _load()


def stage_names() -> list:
    """Names of the pipeline stages, in order: stage i of options profile=2+i."""
    lib = _load()
    return [lib.ac_stage_name(i).decode() for i in range(lib.ac_stage_count())]


def _check(st: int):
    if st != 0:
        raise AlphaCxError(st, _load().ac_last_error().decode(errors="replace"))


class AlphaComplex:
    """Owns an ac_complex handle; released on close() or garbage collection."""

    def __init__(self, handle):
        self._h = handle

    def close(self):
        if self._h:
            _load().ac_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def count(self, dim: int) -> int:
        return int(_load().ac_count(self._h, dim))

    def counts(self):
        return [self.count(d) for d in range(4)]

    def simplices(self, dim: int) -> np.ndarray:
        lib = _load()
        m = self.count(dim)
        p = lib.ac_simplices(self._h, dim)
        if not p:
            _check(5)
        if m == 0:
            return np.zeros((0, dim + 1), dtype=np.int32)
        return np.ctypeslib.as_array(p, shape=(m * (dim + 1),)).reshape(m, dim + 1).copy()

    def sizes(self, dim: int) -> np.ndarray:
        lib = _load()
        m = self.count(dim)
        p = lib.ac_sizes(self._h, dim)
        if not p:
            _check(5)
        if m == 0:
            return np.zeros((0,), dtype=np.float64)
        return np.ctypeslib.as_array(p, shape=(m,)).copy()

    def device_pointers(self, dim: int):
        lib = _load()
        return lib.ac_simplices_device(self._h, dim), lib.ac_sizes_device(self._h, dim)

    def stage_ms(self) -> dict:
        """Per-stage device milliseconds of a profiled call (options profile=1:
        every stage; profile=2+i: stage i only, the others -1)."""
        lib = _load()
        return {lib.ac_stage_name(i).decode(): lib.ac_stage_ms(self._h, i) for i in range(lib.ac_stage_count())}

    def candidate_count(self, dim: int) -> int:
        return int(_load().ac_candidate_count(self._h, dim))

    def exact_fallbacks(self) -> int:
        return int(_load().ac_exact_fallbacks(self._h))

    def work_count(self, which: int) -> int:
        return int(_load().ac_work_count(self._h, which))

    def molecule_count(self) -> int:
        return int(_load().ac_molecule_count(self._h))

    def molecule(self, dim: int) -> np.ndarray:
        """Molecule of every dim-simplex of a batch result (ac_molecule)."""
        p = _load().ac_molecule(self._h, dim)
        if not p:
            _check(1)
        m = self.count(dim)
        if m == 0:
            return np.zeros((0,), dtype=np.int32)
        return np.ctypeslib.as_array(p, shape=(m,)).copy()

    def molecule_rows(self, dim: int) -> np.ndarray:
        """Rows [r[m], r[m+1]) of the dim-simplex array belong to molecule m."""
        lib = _load()
        p = lib.ac_molecule_rows(self._h, dim)
        if not p:
            _check(1)
        return np.ctypeslib.as_array(p, shape=(self.molecule_count() + 1,)).copy()


def _opts(options):
    if options is None:
        return None
    if isinstance(options, Options):
        return ctypes.byref(options)
    o = Options()
    for k, v in dict(options).items():
        setattr(o, k, int(v))
    return ctypes.byref(o)


def ac_alpha_complex(xyz, radii, alpha: float, options=None) -> AlphaComplex:
    """Host arrays (n x 3 and n float64, angstrom) -> alpha complex (host results)."""
    lib = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    radii = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    if xyz.shape[0] != radii.shape[0]:
        raise ValueError("xyz and radii disagree in length")
    h = ctypes.c_void_p()
    st = lib.ac_alpha_complex(xyz.ctypes.data, radii.ctypes.data, xyz.shape[0], float(alpha), _opts(options),
                              ctypes.byref(h))
    _check(st)
    return AlphaComplex(h)


def ac_alpha_complex_device(xyz, radii, alpha: float, options=None, stream=None) -> AlphaComplex:
    """torch float64 device tensors (n x 3, n) -> alpha complex kept on the device.

    Runs on `stream` (a torch.cuda.Stream; default: the current stream)."""
    import torch
    lib = _load()
    if not (xyz.is_cuda and radii.is_cuda):
        raise ValueError("ac_alpha_complex_device needs device tensors")
    if xyz.dtype != torch.float64 or radii.dtype != torch.float64:
        raise ValueError("float64 tensors expected")
    xyz = xyz.contiguous()
    radii = radii.contiguous()
    if xyz.dim() != 2 or xyz.shape[1] != 3 or radii.shape[0] != xyz.shape[0]:
        raise ValueError("xyz must be n x 3 and radii n")
    s = stream if stream is not None else torch.cuda.current_stream(xyz.device)
    h = ctypes.c_void_p()
    st = lib.ac_alpha_complex_device(xyz.data_ptr(), radii.data_ptr(), xyz.shape[0], float(alpha), _opts(options),
                                     ctypes.c_void_p(s.cuda_stream), ctypes.byref(h))
    _check(st)
    return AlphaComplex(h)


class CapacityError(AlphaCxError):
    """An output buffer of ac_alpha_complex_noalloc is smaller than the
    result; `counts` holds the rows needed per dimension."""

    def __init__(self, detail: str, counts):
        super().__init__(6, detail)
        self.counts = counts


def ac_alpha_complex_noalloc(xyz, radii, alpha: float, simp_out, size_out, options=None, stream=None) -> list:
    """As ac_alpha_complex_device, with no allocation by the library: its
    buffers come from a fixed device scratch array, and the result goes into
    the caller's tensors. simp_out[d]: contiguous int32 device tensor of shape
    (capacity, d + 1); size_out[d]: contiguous float64 device tensor of
    (capacity,) (d = 0..3). Returns the row counts [m0, m1, m2, m3]; rows
    [:m_d] of the outputs hold the result. Nothing is copied or allocated
    here: non-contiguous or mistyped tensors are refused. Raises
    CapacityError (with .counts) when an output is too small."""
    import torch
    lib = _load()
    for t in (xyz, radii, *simp_out, *size_out):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("contiguous device tensors expected (no copy is made)")
    if xyz.dtype != torch.float64 or radii.dtype != torch.float64:
        raise ValueError("float64 inputs expected")
    if xyz.dim() != 2 or xyz.shape[1] != 3 or radii.dim() != 1 or radii.shape[0] != xyz.shape[0]:
        raise ValueError("xyz must be n x 3 and radii n")
    if len(simp_out) != 4 or len(size_out) != 4:
        raise ValueError("one output tensor per dimension 0..3")
    cap = (ctypes.c_int64 * 4)()
    sp = (ctypes.c_void_p * 4)()
    zp = (ctypes.c_void_p * 4)()
    for d in range(4):
        a, z = simp_out[d], size_out[d]
        if a.dtype != torch.int32 or a.dim() != 2 or a.shape[1] != d + 1:
            raise ValueError(f"simp_out[{d}] must be int32 of shape (capacity, {d + 1})")
        if z.dtype != torch.float64 or z.dim() != 1 or z.shape[0] != a.shape[0]:
            raise ValueError(f"size_out[{d}] must be float64 of shape ({a.shape[0]},)")
        cap[d] = a.shape[0]
        sp[d] = a.data_ptr() if a.shape[0] else None
        zp[d] = z.data_ptr() if a.shape[0] else None
    counts = (ctypes.c_int64 * 4)()
    st = lib.ac_alpha_complex_noalloc(xyz.data_ptr(), radii.data_ptr(), xyz.shape[0], float(alpha), _opts(options),
                                      _stream(xyz.device, stream), sp, zp, cap, counts)
    if st == 6 and min(counts) >= 0:
        raise CapacityError(lib.ac_last_error().decode(errors="replace"), list(counts))
    _check(st)
    return list(counts)


def ac_alpha_complex_partitioned(xyz, radii, alpha: float, parts: int, options=None, stream=None) -> AlphaComplex:
    """As ac_alpha_complex_device, built slab by slab (`parts` slabs along x,
    each with a halo) and merged; equal to the single build bit for bit."""
    import torch
    lib = _load()
    if not (xyz.is_cuda and radii.is_cuda):
        raise ValueError("ac_alpha_complex_partitioned needs device tensors")
    if xyz.dtype != torch.float64 or radii.dtype != torch.float64:
        raise ValueError("float64 tensors expected")
    xyz = xyz.contiguous()
    radii = radii.contiguous()
    if xyz.dim() != 2 or xyz.shape[1] != 3 or radii.shape[0] != xyz.shape[0]:
        raise ValueError("xyz must be n x 3 and radii n")
    s = stream if stream is not None else torch.cuda.current_stream(xyz.device)
    h = ctypes.c_void_p()
    st = lib.ac_alpha_complex_partitioned(xyz.data_ptr(), radii.data_ptr(), xyz.shape[0], float(alpha), int(parts),
                                          _opts(options), ctypes.c_void_p(s.cuda_stream), ctypes.byref(h))
    _check(st)
    return AlphaComplex(h)


def ac_alpha_complex_partitioned_host(xyz, radii, alpha: float, parts: int, options=None) -> AlphaComplex:
    """Host arrays (n x 3, n float64) -> alpha complex with host results, built
    slab by slab with only one slab on the device at a time (out of core);
    equal to ac_alpha_complex bit for bit."""
    lib = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    radii = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    if xyz.shape[0] != radii.shape[0]:
        raise ValueError("xyz and radii disagree in length")
    h = ctypes.c_void_p()
    st = lib.ac_alpha_complex_partitioned_host(xyz.ctypes.data, radii.ctypes.data, xyz.shape[0], float(alpha),
                                               int(parts), _opts(options), ctypes.byref(h))
    _check(st)
    return AlphaComplex(h)


def ac_alpha_sweep_device(xyz, radii, alphas, options=None, stream=None) -> list:
    """torch float64 device tensors (n x 3, n) -> one AlphaComplex per value of
    `alphas` (in that order), all from a single candidate search at the
    largest; each equals ac_alpha_complex_device at its alpha bit for bit."""
    import torch
    lib = _load()
    if not (xyz.is_cuda and radii.is_cuda):
        raise ValueError("ac_alpha_sweep_device needs device tensors")
    if xyz.dtype != torch.float64 or radii.dtype != torch.float64:
        raise ValueError("float64 tensors expected")
    xyz = xyz.contiguous()
    radii = radii.contiguous()
    if xyz.dim() != 2 or xyz.shape[1] != 3 or radii.shape[0] != xyz.shape[0]:
        raise ValueError("xyz must be n x 3 and radii n")
    a = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64).ravel())
    s = stream if stream is not None else torch.cuda.current_stream(xyz.device)
    hs = (ctypes.c_void_p * max(len(a), 1))()
    st = lib.ac_alpha_sweep_device(xyz.data_ptr(), radii.data_ptr(), xyz.shape[0],
                                   a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(a), _opts(options),
                                   ctypes.c_void_p(s.cuda_stream), hs)
    _check(st)
    return [AlphaComplex(ctypes.c_void_p(h)) for h in hs[:len(a)]]


def _batch_args(xyz, radii, offsets):
    import torch
    if not (xyz.is_cuda and radii.is_cuda):
        raise ValueError("device tensors expected")
    if xyz.dtype != torch.float64 or radii.dtype != torch.float64:
        raise ValueError("float64 tensors expected")
    xyz = xyz.contiguous()
    radii = radii.contiguous()
    off = np.ascontiguousarray(offsets, dtype=np.int64).reshape(-1)
    if xyz.dim() != 2 or xyz.shape[1] != 3 or radii.shape[0] != xyz.shape[0]:
        raise ValueError("xyz must be n x 3 and radii n")
    if len(off) < 2 or off[-1] != xyz.shape[0]:
        raise ValueError("offsets must end at the number of balls")
    return xyz, radii, off


def ac_alpha_complex_batch(xyz, radii, offsets, alpha: float, options=None, cell_mA=None, stream=None) -> AlphaComplex:
    """Molecules [offsets[m], offsets[m+1]) of the concatenated device tensors
    in one call; ids of the result index the concatenated arrays."""
    xyz, radii, off = _batch_args(xyz, radii, offsets)
    cells = None
    if cell_mA is not None:
        cells = np.ascontiguousarray(cell_mA, dtype=np.int32).reshape(-1)
        if len(cells) != len(off) - 1:
            raise ValueError("cell_mA needs one side per molecule")
    h = ctypes.c_void_p()
    st = _load().ac_alpha_complex_batch(xyz.data_ptr(), radii.data_ptr(), off.ctypes.data, len(off) - 1, float(alpha),
                                        _opts(options), None if cells is None else cells.ctypes.data,
                                        _stream(xyz.device, stream), ctypes.byref(h))
    _check(st)
    return AlphaComplex(h)


class Plan:
    """A recorded batch build (ac_plan_create): the pipeline captured once in
    a HIP graph on the given device tensors; launch() replays it on whatever
    coordinates and radii those tensors hold then, result() returns the
    complex (an ordinary batch build instead when the input no longer fits
    what was recorded). Keep xyz and radii alive (and at the same storage)
    for the plan's lifetime."""

    def __init__(self, xyz, radii, offsets, alpha: float, options=None, cell_mA=None, headroom: float = 1.25,
                 stream=None):
        xyz_c, radii_c, off = _batch_args(xyz, radii, offsets)
        if xyz_c.data_ptr() != xyz.data_ptr() or radii_c.data_ptr() != radii.data_ptr():
            raise ValueError("contiguous tensors expected: the plan records their storage")
        self._xyz, self._radii = xyz, radii
        cells = None
        if cell_mA is not None:
            cells = np.ascontiguousarray(cell_mA, dtype=np.int32).reshape(-1)
            if len(cells) != len(off) - 1:
                raise ValueError("cell_mA needs one side per molecule")
        self._device = xyz.device
        h = ctypes.c_void_p()
        st = _load().ac_plan_create(xyz.data_ptr(), radii.data_ptr(), off.ctypes.data, len(off) - 1, float(alpha),
                                    _opts(options), None if cells is None else cells.ctypes.data, float(headroom),
                                    _stream(xyz.device, stream), ctypes.byref(h))
        _check(st)
        self._h = h

    def launch(self, stream=None):
        _check(_load().ac_plan_launch(self._h, _stream(self._device, stream)))

    def result(self, stream=None) -> AlphaComplex:
        h = ctypes.c_void_p()
        _check(_load().ac_plan_result(self._h, _stream(self._device, stream), ctypes.byref(h)))
        return AlphaComplex(h)

    def stopped(self) -> int:
        return int(_load().ac_plan_stopped(self._h))

    def ordinary_builds(self) -> int:
        return int(_load().ac_plan_ordinary_builds(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _load().ac_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ac_plan_create(xyz, radii, offsets, alpha: float, options=None, cell_mA=None, headroom: float = 1.25,
                   stream=None) -> Plan:
    return Plan(xyz, radii, offsets, alpha, options=options, cell_mA=cell_mA, headroom=headroom, stream=stream)


def ac_tune_cells(xyz, radii, offsets, alpha: float, options=None, stream=None):
    """Autotuned cell side (mA) per molecule, and each molecule's size bucket."""
    xyz, radii, off = _batch_args(xyz, radii, offsets)
    n_mol = len(off) - 1
    cells = np.zeros(n_mol, dtype=np.int32)
    buckets = np.zeros(n_mol, dtype=np.int32)
    _check(_load().ac_tune_cells(xyz.data_ptr(), radii.data_ptr(), off.ctypes.data, n_mol, float(alpha),
                                 _opts(options), _stream(xyz.device, stream), cells.ctypes.data, buckets.ctypes.data))
    return cells, buckets


def ac_release_workspace():
    _check(_load().ac_release_workspace())


def _balls(xyz, radii):
    import torch
    if not (xyz.is_cuda and radii.is_cuda):
        raise ValueError("device tensors expected")
    if xyz.dtype != torch.float64 or radii.dtype != torch.float64:
        raise ValueError("float64 tensors expected")
    xyz = xyz.detach().contiguous()
    radii = radii.detach().contiguous()
    if xyz.dim() != 2 or xyz.shape[1] != 3 or radii.dim() != 1 or radii.shape[0] != xyz.shape[0]:
        raise ValueError("xyz must be n x 3 and radii n")
    return xyz, radii


def _stream(dev, stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    return ctypes.c_void_p(s.cuda_stream)


def ac_union_measure(c: AlphaComplex, xyz, radii, stream=None):
    """(V, A) of the union of the balls from the complex at alpha = 0 (host floats)."""
    xyz, radii = _balls(xyz, radii)
    V, A = ctypes.c_double(), ctypes.c_double()
    _check(_load().ac_union_measure(c._h, xyz.data_ptr(), radii.data_ptr(), xyz.shape[0], ctypes.byref(V),
                                    ctypes.byref(A), _stream(xyz.device, stream)))
    return V.value, A.value


def ac_union_measure_device(c: AlphaComplex, xyz, radii, stream=None):
    """Device float64 tensor [V, A]; no host synchronisation."""
    import torch
    xyz, radii = _balls(xyz, radii)
    out = torch.empty(2, dtype=torch.float64, device=xyz.device)
    _check(_load().ac_union_measure_device(c._h, xyz.data_ptr(), radii.data_ptr(), xyz.shape[0], out.data_ptr(),
                                           _stream(xyz.device, stream)))
    return out


def ac_union_measure_backward(c: AlphaComplex, xyz, radii, grad, stream=None):
    """Gradient of grad[0] * V + grad[1] * A (grad: device float64 tensor of 2)
    with respect to xyz (n x 3) and radii (n), the complex held fixed."""
    import torch
    xyz, radii = _balls(xyz, radii)
    grad = grad.detach().to(device=xyz.device, dtype=torch.float64).contiguous()
    if grad.numel() != 2:
        raise ValueError("grad must hold (gV, gA)")
    dx = torch.empty_like(xyz)
    dr = torch.empty_like(radii)
    _check(_load().ac_union_measure_backward(c._h, xyz.data_ptr(), radii.data_ptr(), xyz.shape[0], grad.data_ptr(),
                                             dx.data_ptr(), dr.data_ptr(), _stream(xyz.device, stream)))
    return dx, dr


def ac_union_measure_fused(c: AlphaComplex, xyz, radii, grad, stream=None):
    """V, A (device tensor of 2) and the gradient of grad[0] * V + grad[1] * A
    with respect to xyz and radii, in one pass."""
    import torch
    xyz, radii = _balls(xyz, radii)
    grad = grad.detach().to(device=xyz.device, dtype=torch.float64).contiguous()
    if grad.numel() != 2:
        raise ValueError("grad must hold (gV, gA)")
    out = torch.empty(2, dtype=torch.float64, device=xyz.device)
    dx = torch.empty_like(xyz)
    dr = torch.empty_like(radii)
    _check(_load().ac_union_measure_fused(c._h, xyz.data_ptr(), radii.data_ptr(), xyz.shape[0], grad.data_ptr(),
                                          out.data_ptr(), dx.data_ptr(), dr.data_ptr(), _stream(xyz.device, stream)))
    return out, dx, dr


def _autograd_function():
    import torch

    class UnionMeasure(torch.autograd.Function):
        """[V, A] = UnionMeasure.apply(xyz, radii, complex): volume and boundary
        area of the union of the balls, differentiable in xyz and radii with
        the complex (built at alpha = 0) held fixed."""

        @staticmethod
        def forward(ctx, xyz, radii, c):
            ctx.save_for_backward(xyz, radii)
            ctx.complex = c
            return ac_union_measure_device(c, xyz, radii)

        @staticmethod
        def backward(ctx, g):
            xyz, radii = ctx.saved_tensors
            dx, dr = ac_union_measure_backward(ctx.complex, xyz, radii, g)
            return dx, dr, None

    return UnionMeasure


def __getattr__(name):
    if name == "UnionMeasure":
        fn = _autograd_function()
        globals()["UnionMeasure"] = fn
        return fn
    raise AttributeError(name)
