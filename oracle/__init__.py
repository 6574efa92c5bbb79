"""CPU oracle for the alpha complex of weighted points: test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package. It shares no code with the HIP path (see oracle.c for the
method: the weighted Delaunay triangulation, Size of every simplex, then the
alpha filter, all in exact integer arithmetic).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

STATUS = {0: "ok", 1: "invalid", 2: "duplicate", 3: "range", 4: "nomem", 7: "degenerate"}


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"oracle failed: {STATUS.get(status, status)}")
        self.status = status


class _Result(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int64 * 4),
        ("simp", ctypes.POINTER(ctypes.c_int32) * 4),
        ("size", ctypes.POINTER(ctypes.c_double) * 4),
        ("n_hidden", ctypes.c_int64),
        ("d_count", ctypes.c_int64 * 4),
    ]


def build() -> str:
    """Compile oracle.c with gcc into oracle/liboracle.so (always rebuilds)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-o", _SO + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    lib.oracle_alpha_complex.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                         ctypes.c_uint64, ctypes.POINTER(_Result)]
    lib.oracle_alpha_complex.restype = ctypes.c_int
    lib.oracle_free.argtypes = [ctypes.POINTER(_Result)]
    _lib = lib
    return lib


class Complex:
    """K_alpha as four sorted simplex arrays (input ids) with Sizes in square angstrom."""

    def __init__(self, simplices, sizes, n_hidden, d_count):
        self.simplices = simplices
        self.sizes = sizes
        self.n_hidden = n_hidden
        self.d_count = d_count

    def counts(self):
        return [int(s.shape[0]) for s in self.simplices]

    def euler(self) -> int:
        c = self.counts()
        return c[0] - c[1] + c[2] - c[3]


def alpha_complex(xyz, radii, alpha: float, order_seed: int = 0) -> Complex:
    """Alpha complex of balls (centres xyz [n,3] and radii [n], angstrom) at alpha (square angstrom)."""
    lib = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    radii = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    if radii.shape[0] != xyz.shape[0]:
        raise ValueError("xyz and radii disagree in length")
    res = _Result()
    st = lib.oracle_alpha_complex(xyz.shape[0], xyz.ctypes.data, radii.ctypes.data, float(alpha), order_seed,
                                  ctypes.byref(res))
    if st != 0:
        raise OracleError(st)
    try:
        simplices, sizes = [], []
        for d in range(4):
            m = res.count[d]
            if m:
                s = np.ctypeslib.as_array(res.simp[d], shape=(m * (d + 1),)).reshape(m, d + 1).copy()
                z = np.ctypeslib.as_array(res.size[d], shape=(m,)).copy()
            else:
                s = np.zeros((0, d + 1), dtype=np.int32)
                z = np.zeros((0,), dtype=np.float64)
            simplices.append(s)
            sizes.append(z)
        return Complex(simplices, sizes, int(res.n_hidden), [int(x) for x in res.d_count])
    finally:
        lib.oracle_free(ctypes.byref(res))
