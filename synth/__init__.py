"""Seeded synthetic molecules shared by the tests, the benchmark and the oracle runs.

Input generation only: nothing here computes any part of the alpha complex.

Recipe (one molecule): centres by random sequential adsorption on the integer
milli-angstrom lattice (minimum centre separation 2.4 A) inside a ball, or a
shell with inner radius 0.7 R_out, at 0.05 centres per cubic angstrom; then one
element per centre in acceptance order (C 1.70 A p=.62, N 1.55 .17, O 1.52 .19,
S 1.80 .02). Solvent-accessible radii add 1.4 A. Coordinates and radii are
multiples of 0.001 A, handed over as float64 angstrom values.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None

DENSITY = 0.05        # centres per cubic angstrom
MIN_SEP_MA = 2400     # minimum centre separation, milli-angstrom
PROBE_MA = 1400       # solvent probe added for solvent-accessible radii


def build() -> str:
    """Compile the generator with gcc into synth/libsynth.so (always rebuilds)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", _SO + ".tmp", _SRC, "-lm"]
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
    i64, u64, p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
    lib.synth_rsa.argtypes = [i64, u64, i64, i64, i64, p, p]
    lib.synth_rsa.restype = ctypes.c_int
    lib.synth_radii.argtypes = [i64, u64, p]
    lib.synth_normal.argtypes = [i64, u64, p]
    lib.synth_uniform.argtypes = [i64, u64, p]
    lib.synth_below.argtypes = [i64, u64, u64, p]
    _lib = lib
    return lib


def ball_radius_A(n: int, density: float = DENSITY) -> float:
    return (3.0 * n / (4.0 * math.pi * density)) ** (1.0 / 3.0)


def shell_radius_A(n: int, inner_frac: float = 0.7, density: float = DENSITY) -> float:
    return (3.0 * n / (4.0 * math.pi * density * (1.0 - inner_frac ** 3))) ** (1.0 / 3.0)


def rsa_centres(n: int, seed: int, r_out_mA: int, r_in_mA: int = 0, min_sep_mA: int = MIN_SEP_MA) -> np.ndarray:
    """int32 [n,3] lattice centres (mA) in acceptance order."""
    lib = _load()
    out = np.empty((n, 3), dtype=np.int32)
    darts = ctypes.c_int64(0)
    rc = lib.synth_rsa(n, seed, r_in_mA, r_out_mA, min_sep_mA, out.ctypes.data, ctypes.byref(darts))
    if rc != 0:
        raise RuntimeError(f"synth_rsa failed (rc={rc}) for n={n}, seed={seed}")
    return out


def element_radii_mA(n: int, seed: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, dtype=np.int32)
    lib.synth_radii(n, seed, out.ctypes.data)
    return out


def normals(n: int, seed: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, dtype=np.float64)
    lib.synth_normal(n, seed, out.ctypes.data)
    return out


def uniforms(n: int, seed: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, dtype=np.float64)
    lib.synth_uniform(n, seed, out.ctypes.data)
    return out


def integers_below(n: int, seed: int, m: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, dtype=np.int64)
    lib.synth_below(n, seed, m, out.ctypes.data)
    return out


class Molecule:
    """Lattice centres and radii (mA, int32) plus their float64 angstrom views."""

    def __init__(self, X_mA: np.ndarray, R_mA: np.ndarray, name: str = ""):
        self.X_mA = np.ascontiguousarray(X_mA, dtype=np.int32)
        self.R_mA = np.ascontiguousarray(R_mA, dtype=np.int32)
        self.name = name

    @property
    def n(self) -> int:
        return int(self.R_mA.shape[0])

    @property
    def xyz(self) -> np.ndarray:
        return self.X_mA.astype(np.float64) / 1000.0

    @property
    def radii(self) -> np.ndarray:
        return self.R_mA.astype(np.float64) / 1000.0

    def with_sas(self, probe_mA: int = PROBE_MA) -> "Molecule":
        return Molecule(self.X_mA, self.R_mA + probe_mA, self.name + "+sas")


def molecule(n: int, seed: int, shell: bool = False, sas: bool = False) -> Molecule:
    """One synthetic molecule: a ball (or a shell with inner radius 0.7 R_out) at 0.05/A^3."""
    if shell:
        r_out = shell_radius_A(n)
        r_in = 0.7 * r_out
    else:
        r_out, r_in = ball_radius_A(n), 0.0
    X = rsa_centres(n, seed, int(round(r_out * 1000)), int(round(r_in * 1000)))
    R = element_radii_mA(n, seed + (1 << 32))
    m = Molecule(X, R, f"{'shell' if shell else 'ball'}{n}_s{seed}")
    return m.with_sas() if sas else m


def batch_sizes(n_mol: int = 512, seed: int = 999, lo: int = 500, hi: int = 50000) -> np.ndarray:
    """Log-uniform molecule sizes in [lo, hi]."""
    u = uniforms(n_mol, seed)
    return np.rint(np.exp(math.log(lo) + u * math.log(hi / lo))).astype(np.int64)


def jittered(mol: Molecule, sigma_A: float, seed: int) -> Molecule:
    """Gaussian jitter on every coordinate, re-quantised to the mA lattice; radii unchanged."""
    g = normals(mol.n * 3, seed).reshape(mol.n, 3)
    X = np.rint(mol.X_mA.astype(np.float64) + g * sigma_A * 1000.0).astype(np.int32)
    return Molecule(X, mol.R_mA, mol.name + f"_j{seed}")


# Named workloads (seeds recorded here so tests and the benchmark agree).
def config_small() -> Molecule:
    """1,000 atoms in a ball, vdW radii (alpha = 0)."""
    return molecule(1000, 1)


def config_100k(sas: bool = False) -> Molecule:
    """100,000 atoms in a ball; vdW radii, or solvent-accessible radii (+1.4 A)."""
    return molecule(100_000, 2, sas=sas)


def config_shell_3m(cache_dir: str | None = None) -> Molecule:
    """3,000,000 atoms in a shell (inner radius 0.7 R_out). With cache_dir, the
    lattice arrays are kept there as .npy files (generation takes ~30-70 s)."""
    if cache_dir:
        fx = os.path.join(cache_dir, "shell3m_s3_X.npy")
        fr = os.path.join(cache_dir, "shell3m_s3_R.npy")
        if os.path.exists(fx) and os.path.exists(fr):
            return Molecule(np.load(fx), np.load(fr), "shell3000000_s3")
    m = molecule(3_000_000, 3, shell=True)
    if cache_dir:
        os.makedirs(cache_dir, exist_ok=True)
        np.save(fx, m.X_mA)
        np.save(fr, m.R_mA)
    return m
