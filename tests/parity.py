"""Comparison helpers shared by the GPU parity tests (no arithmetic of the method)."""
import numpy as np

SIZE_ABS_TOL = 1e-9   # square angstrom
SIZE_REL_TOL = 1e-12


def assert_same_complex(got, want, label=""):
    """got: paper_1908_05944_amd.AlphaComplex; want: oracle.Complex.
    Simplex lists must be identical; Sizes within the float64 tolerance."""
    for d in range(4):
        s = got.simplices(d)
        w = want.simplices[d]
        if not np.array_equal(s, w):
            a = set(map(tuple, s.tolist()))
            b = set(map(tuple, w.tolist()))
            raise AssertionError(f"{label} dim {d}: {len(s)} vs {len(w)} simplices; gpu-only {sorted(a - b)[:5]} "
                                 f"oracle-only {sorted(b - a)[:5]}")
        z = got.sizes(d)
        err = np.abs(z - want.sizes[d])
        tol = SIZE_ABS_TOL + SIZE_REL_TOL * np.abs(want.sizes[d])
        bad = np.nonzero(err > tol)[0]
        if bad.size:
            i = bad[0]
            raise AssertionError(f"{label} dim {d}: Size of {w[i].tolist()} is {z[i]!r}, oracle {want.sizes[d][i]!r}")
