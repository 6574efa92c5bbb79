"""alphacx for MI355X: Python binding of libalphacx.so (argument marshalling only).

Every step of the computation runs in the HIP kernels of libalphacx.so; this
module only converts arguments and results. It fails loudly when the library
is missing: there is no CPU fallback.

Names follow the C ABI in include/alphacx.h:
    ac_alpha_complex(xyz, radii, alpha, options=None)          host arrays in, host arrays out
    ac_alpha_complex_device(xyz, radii, alpha, options=None,   torch device tensors in,
                            stream=None)                        results kept on the device
Both return an `AlphaComplex` owning the library's result handle.
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
    _lib = lib
    return lib


def library():
    """The loaded ctypes handle of libalphacx.so."""
    return _load()


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
        """Per-stage device milliseconds of a profiled call (options profile=1)."""
        lib = _load()
        return {lib.ac_stage_name(i).decode(): lib.ac_stage_ms(self._h, i) for i in range(lib.ac_stage_count())}

    def candidate_count(self, dim: int) -> int:
        return int(_load().ac_candidate_count(self._h, dim))

    def exact_fallbacks(self) -> int:
        return int(_load().ac_exact_fallbacks(self._h))


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


def ac_release_workspace():
    _check(_load().ac_release_workspace())
