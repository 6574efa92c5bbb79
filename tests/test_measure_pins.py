"""Pins of the oracle's union volume / area and their gradients (oracle/measure.py).

Independent of the inclusion-exclusion formulas: textbook closed forms for one
and two balls, quadrature by slicing (tests/slicing.py) for up to a dozen
balls, Monte Carlo within its error bound on the 1,000-atom molecule, central
finite differences of V and A for the gradients, and the invariances that any
correct gradient obeys (translation, rotation, homogeneity of degree 3 and 2).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import measure
from slicing import union_volume_area

EPS = np.finfo(np.float64).eps


def _measure(xyz, rad, grad=False):
    xyz = np.asarray(xyz, dtype=float)
    rad = np.asarray(rad, dtype=float)
    c = oracle.alpha_complex(xyz, rad, 0.0)
    return c, measure.union_measure(c.simplices, xyz, rad, with_grad=grad)


def test_one_ball():
    _, (V, A) = _measure([[1.0, -2.0, 0.5]], [1.7])
    assert V == pytest.approx(4 / 3 * math.pi * 1.7 ** 3, rel=1e-15)
    assert A == pytest.approx(4 * math.pi * 1.7 ** 2, rel=1e-15)


@pytest.mark.parametrize("d", [0.4, 1.0, 2.2, 3.1])
def test_two_balls_lens(d):
    r1, r2 = 1.7, 1.5
    xyz = np.array([[0.0, 0.0, 0.0], [d * 0.6, d * 0.8, 0.0]])
    _, (V, A) = _measure(xyz, [r1, r2])
    # textbook lens volume of two intersecting balls
    lens = math.pi * (r1 + r2 - d) ** 2 * (d * d + 2 * d * (r1 + r2) - 3 * (r1 - r2) ** 2) / (12 * d)
    assert V == pytest.approx(4 / 3 * math.pi * (r1 ** 3 + r2 ** 3) - lens, rel=1e-13)
    # Archimedes: a cap of height h on a sphere of radius r has area 2 pi r h
    h1 = r1 - (d * d + r1 * r1 - r2 * r2) / (2 * d)
    h2 = r2 - (d * d + r2 * r2 - r1 * r1) / (2 * d)
    assert A == pytest.approx(4 * math.pi * (r1 * r1 + r2 * r2) - 2 * math.pi * (r1 * h1 + r2 * h2), rel=1e-13)


def test_disjoint_balls_add_up():
    xyz = np.array([[0.0, 0, 0], [5.0, 0, 0], [0, 6.0, 0]])
    rad = np.array([1.2, 1.9, 1.5])
    c, (V, A) = _measure(xyz, rad)
    assert c.counts() == [3, 0, 0, 0]
    assert V == pytest.approx(4 / 3 * math.pi * np.sum(rad ** 3), rel=1e-15)
    assert A == pytest.approx(4 * math.pi * np.sum(rad ** 2), rel=1e-15)


CASES = {
    "three": ([[0, 0, 0], [2.0, 0.3, 0.1], [0.8, 1.6, 0.4]], [1.5, 1.2, 1.4]),
    "four": ([[0, 0, 0], [2.0, 0.3, 0.1], [0.8, 1.6, 0.4], [0.9, 0.7, 1.5]], [1.5, 1.2, 1.4, 1.3]),
    # one ball much smaller, deep in the lens of two others: large faces
    "small_in_lens": ([[0, 0, 0], [2.2, 0, 0], [1.1, 0.4, 0.2]], [1.8, 1.8, 0.6]),
    # the orthocentre of the tetrahedron outside its convex hull
    "obtuse_tet": ([[0, 0, 0], [2.6, 0, 0], [1.3, 2.0, 0], [1.3, 0.5, 0.35]], [1.6, 1.6, 1.6, 0.9]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_small_configurations_match_slicing(name):
    xyz, rad = CASES[name]
    c, (V, A) = _measure(xyz, rad)
    Vs, As = union_volume_area(xyz, rad)
    assert abs(V - Vs) <= 1e-11 * Vs, (c.counts(), V, Vs)
    assert abs(A - As) <= 1e-11 * As, (c.counts(), A, As)


# Near-degenerate four-ball sets (found by a seeded search, kept as data):
# a common intersection of four balls that is tiny (tetrahedron OrthoSize
# -0.011 and -0.012 A^2), centres almost coplanar (tetrahedra of 0.029 and
# 0.018 A^3), and a small ball near the triple region of three large ones.
DEGENERATE4 = {
    "tiny_a": ([[1.55, -0.622, -0.522], [0.004, 0.484, -0.661], [0.411, 0.036, 1.11], [-0.622, -0.955, -0.077]],
               [1.373, 1.712, 1.344, 1.084]),
    "tiny_b": ([[-0.585, 1.018, -1.017], [-0.291, -0.253, 1.396], [0.406, -0.468, -1.192], [-1.061, -1.515, -0.911]],
               [1.692, 1.424, 1.316, 1.797]),
    "flat_a": ([[-0.479, 1.412, 0.244], [1.294, 1.173, 0.242], [0.615, 1.424, -0.807], [1.024, 1.172, -0.123]],
               [1.402, 1.604, 1.343, 1.393]),
    "flat_b": ([[0.64, -0.228, -0.319], [-0.093, -0.197, -1.019], [-0.544, -0.575, 1.536], [-1.425, -0.503, 0.065]],
               [1.006, 1.417, 1.406, 1.521]),
    "inner_a": ([[1.1, -1.332, -0.634], [0.13, -0.154, -0.938], [0.947, 0.012, -1.057], [0.407, -1.009, 0.485]],
                [1.26, 1.316, 1.608, 0.536]),
    "inner_b": ([[-1.557, -0.53, 0.8], [-0.569, -0.676, -0.507], [-0.558, -1.217, 1.341], [-0.205, -0.135, 0.722]],
                [1.469, 1.158, 1.633, 0.516]),
}


@pytest.mark.parametrize("name", sorted(DEGENERATE4))
def test_near_degenerate_four_balls_match_slicing(name):
    """Each set is one tetrahedron with all its faces in K_0; the slicing
    quadrature at 96 nodes per panel converges to about 1e-15 on them."""
    xyz, rad = DEGENERATE4[name]
    c, (V, A) = _measure(xyz, rad)
    assert c.counts() == [4, 6, 4, 1]
    Vs, As = union_volume_area(xyz, rad, nodes=96)
    assert abs(V - Vs) <= 1e-13 * Vs, (V, Vs)
    assert abs(A - As) <= 1e-13 * As, (A, As)


def test_random_sets_match_slicing():
    rng = np.random.RandomState(5)
    dims = np.zeros(4)
    for t in range(6):
        n = 12
        xyz = np.round(rng.uniform(-2.5, 2.5, (n, 3)), 3)
        rad = np.round(rng.uniform(1.0, 1.8, n), 3)
        c, (V, A) = _measure(xyz, rad)
        dims += np.array(c.counts()) > 0
        Vs, As = union_volume_area(xyz, rad)
        assert abs(V - Vs) <= 1e-11 * Vs, (t, V, Vs)
        assert abs(A - As) <= 1e-11 * As, (t, A, As)
    assert dims[3] >= 3  # tetrahedra were exercised


def test_monte_carlo_1k_molecule():
    from scipy.spatial import cKDTree
    m = synth.config_small()
    _, (V, A) = _measure(m.xyz, m.radii)
    lo = m.xyz.min(0) - m.radii.max()
    hi = m.xyz.max(0) + m.radii.max()
    rng = np.random.RandomState(17)
    tree = cKDTree(m.xyz)
    inside = 0
    total = 0
    for _ in range(8):
        pts = lo + (hi - lo) * rng.random_sample((500_000, 3))
        d, j = tree.query(pts, k=8, distance_upper_bound=m.radii.max())
        ok = np.isfinite(d)
        rr = np.zeros_like(d)
        rr[ok] = m.radii[j[ok]]
        inside += int(np.sum(np.any(ok & (d < rr), axis=1)))
        total += len(pts)
    box = float(np.prod(hi - lo))
    p = inside / total
    Vmc = box * p
    sigma = box * math.sqrt(p * (1 - p) / total)
    assert abs(V - Vmc) < 5 * sigma, (V, Vmc, sigma)
    assert 0.3 * V < A < 3 * V  # sanity: area of a fused set of ~1.6 A balls


def _star(simplices, i):
    """The simplices of the complex that contain ball i: the only terms of V
    and A that move with it."""
    return [s[np.any(s == i, axis=1)] if len(s) else s for s in simplices]


def _abs_terms(star, xyz, rad):
    """Sums of |term| of V and of A over a set of simplices: what bounds the
    rounding error of their signed sums."""
    sv = sa = 0.0
    for s in star:
        if len(s):
            vol, area = measure.intersection_terms(xyz[s], rad[s])[:2]
            sv += np.abs(vol).sum()
            sa += np.abs(area).sum()
    return sv, sa


def _fd_check(xyz, rad, atoms, h=1e-5):
    """Central differences of V and A over the terms incident to the moved
    ball (differencing the whole sum would lose the 1e-6 tolerance to
    cancellation). For a buried ball the star's terms cancel to zero, so the
    tolerance also admits the rounding of the star's sums, 8 eps sum|term| / h."""
    c, (V, A, gVx, gVr, gAx, gAr) = _measure(xyz, rad, grad=True)
    med_V = np.median(np.abs(np.concatenate([gVx.ravel(), gVr])))
    med_A = np.median(np.abs(np.concatenate([gAx.ravel(), gAr])))
    for i in atoms:
        star = _star(c.simplices, i)
        sv, sa = _abs_terms(star, xyz, rad)
        for k in range(4):
            xp, xm, rp, rm = xyz.copy(), xyz.copy(), rad.copy(), rad.copy()
            if k < 3:
                xp[i, k] += h
                xm[i, k] -= h
            else:
                rp[i] += h
                rm[i] -= h
            Vp, Ap = measure.union_measure(star, xp, rp)
            Vm, Am = measure.union_measure(star, xm, rm)
            gv = gVx[i, k] if k < 3 else gVr[i]
            ga = gAx[i, k] if k < 3 else gAr[i]
            tol_v = 1e-6 * max(abs(gv), 1e-3 * med_V) + 8 * EPS * sv / h
            tol_a = 1e-6 * max(abs(ga), 1e-3 * med_A) + 8 * EPS * sa / h
            assert abs((Vp - Vm) / (2 * h) - gv) <= tol_v, (i, k, (Vp - Vm) / (2 * h), gv)
            assert abs((Ap - Am) / (2 * h) - ga) <= tol_a, (i, k, (Ap - Am) / (2 * h), ga)
    return V, A, gVx, gVr, gAx, gAr


def test_gradients_finite_differences_random():
    rng = np.random.RandomState(7)
    for _ in range(3):
        n = 12
        xyz = np.round(rng.uniform(-2.5, 2.5, (n, 3)), 3)
        rad = np.round(rng.uniform(1.0, 1.8, n), 3)
        _fd_check(xyz, rad, range(n))


@pytest.mark.parametrize("sas", [False, True])
def test_gradients_finite_differences_molecule(sas):
    m = synth.molecule(400, 9)
    if sas:
        m = m.with_sas(1400)
    atoms = np.random.RandomState(3).choice(m.n, 40, replace=False)
    _fd_check(m.xyz.copy(), m.radii.copy(), atoms)


def test_gradient_invariances():
    m = synth.molecule(500, 4).with_sas(1400)
    c, (V, A, gVx, gVr, gAx, gAr) = _measure(m.xyz, m.radii, grad=True)
    for f, gx, gr, deg in ((V, gVx, gVr, 3), (A, gAx, gAr, 2)):
        scale = np.abs(gx).max()
        assert np.abs(gx.sum(0)).max() <= 1e-11 * scale * m.n          # translation
        assert np.abs(np.cross(m.xyz, gx).sum(0)).max() <= 1e-9 * scale * m.n  # rotation
        # Euler: f(lambda x, lambda r) = lambda^deg f
        assert np.sum(m.xyz * gx) + np.sum(m.radii * gr) == pytest.approx(deg * f, rel=1e-11)
    # dV/dr_i is the exposed area of sphere i, which sums to A and is never negative
    assert np.sum(gVr) == pytest.approx(A, rel=1e-12)
    assert gVr.min() > -1e-9
