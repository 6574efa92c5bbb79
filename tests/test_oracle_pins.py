"""Pins for the CPU oracle against what the paper and the mathematics fix.

- brute force from the definitions on tiny inputs (tests/bruteforce.py): every
  simplex set, every Size and the simplex counts of D itself, including
  degenerate lattices where simulation of simplicity decides;
- closed forms for two balls (the edge's OrthoSize is minus the squared
  radius of the spheres' intersection circle);
- topology: chi(K_alpha) equals chi of the union of grown balls, computed from
  the Cech nerve (tests/cech.py);
- invariants on synthetic molecules: insertion-order independence,
  translation / rotation / reflection / relabelling, closure under faces,
  monotonicity in alpha, Size monotone along cofaces, chi(D) = 1, and every atom
  a vertex with Size -r^2 for the molecule workloads.
"""
import itertools
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import bruteforce
import cech
import oracle
import synth


def _as_sets(c):
    return [set(map(tuple, s.tolist())) for s in c.simplices]


def _compare_bruteforce(xyz, rad, alpha):
    K, D = bruteforce.alpha_complex(xyz, rad, alpha)
    c = oracle.alpha_complex(xyz, rad, alpha)
    for d in range(4):
        got = [tuple(int(v) for v in row) for row in c.simplices[d]]
        want = [s for s, _ in K[d]]
        assert got == want, f"dim {d}: oracle-only {sorted(set(got) - set(want))[:4]} bf-only {sorted(set(want) - set(got))[:4]}"
        for (s, v), z in zip(K[d], c.sizes[d]):
            exact = float(v) / 1e6
            assert abs(exact - z) <= 1e-9 + 1e-12 * abs(exact), (d, s, exact, z)
    if c.d_count[0] >= 0:
        assert list(c.d_count) == D


def _random_case(rng):
    n = rng.choice([4, 5, 6, 8, 10, 12])
    box = rng.choice([3.0, 5.0, 8.0])
    xyz = np.array([[rng.randint(-int(box * 1000), int(box * 1000)) / 1000 for _ in range(3)] for _ in range(n)])
    rad = np.array([rng.choice([1.2, 1.5, 1.7, 2.0, 0.5]) for _ in range(n)])
    alpha = rng.choice([0.0, 1.0, -0.5, 4.0, 20.0])
    return xyz, rad, alpha


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_random(seed):
    rng = random.Random(100 + seed)
    for _ in range(8):
        _compare_bruteforce(*_random_case(rng))


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 2, 2), (2, 2, 3)])
@pytest.mark.parametrize("rad", [1.0, 1.5])
def test_bruteforce_cubic_lattice(dims, rad):
    """Eight co-spherical centres per cube: every tetrahedron is a tie that
    simulation of simplicity must resolve identically in both codes."""
    pts = np.array([[2.0 * i, 2.0 * j, 2.0 * k] for i in range(dims[0]) for j in range(dims[1]) for k in range(dims[2])])
    for perm in (None, 7):
        p = pts if perm is None else pts[np.random.RandomState(perm).permutation(len(pts))]
        # 0.75 and 2.0 are the exact OrthoSize of the cube-corner tetrahedra for
        # radii 1.5 and 1.0: the closed comparison Size <= alpha decides there.
        for alpha in (0.0, 0.75, 1.0, 2.0, 3.0, 10.0):
            _compare_bruteforce(p, np.full(len(p), rad), alpha)


def test_bruteforce_integer_grid_ties():
    rng = random.Random(3)
    for trial in range(20):
        n = rng.choice([6, 8, 10, 12])
        pts = np.array([[rng.randint(-3, 3) for _ in range(3)] for _ in range(n)], dtype=float)
        pts = np.unique(pts, axis=0)
        pts = pts[np.random.RandomState(trial).permutation(len(pts))]
        rad = np.array([rng.choice([1.0, 1.5]) for _ in range(len(pts))])
        _compare_bruteforce(pts, rad, rng.choice([0.0, 0.5, 2.0, 8.0]))


def test_bruteforce_hidden_ball():
    """A small ball near the centre of a large one has an empty power cell."""
    xyz = np.array([[0, 0, 0], [0.1, 0.05, 0.0], [3, 0, 0], [0, 3, 0], [0, 0, 3], [2, 2, 2]], dtype=float)
    rad = np.array([2.0, 0.4, 1.5, 1.5, 1.5, 1.5])
    for order_seed in range(8):  # the small ball arrives before and after the big one
        c = oracle.alpha_complex(xyz, rad, 50.0, order_seed=order_seed)
        assert c.n_hidden == 1
        assert 1 not in set(c.simplices[0][:, 0].tolist())
    _compare_bruteforce(xyz, rad, 50.0)
    _compare_bruteforce(xyz, rad, 0.0)


def test_bruteforce_planar_hull_face():
    """Many centres on one hull plane: insertions land coplanar with hull
    facets, inside and outside their ortho-circles."""
    rng = random.Random(17)
    for trial in range(4):
        base = [[2.0 * i + rng.randint(-300, 300) / 1000, 2.0 * j + rng.randint(-300, 300) / 1000, 0.0]
                for i in range(4) for j in range(3)]
        pts = np.array(base + [[3.0, 2.0, 2.5], [2.5, 1.5, 3.5]])
        rad = np.array([rng.choice([1.2, 1.5, 1.8]) for _ in range(len(pts))])
        for order_seed in range(3):
            c = oracle.alpha_complex(pts, rad, 4.0, order_seed=order_seed)
            assert c.d_count[0] - c.d_count[1] + c.d_count[2] - c.d_count[3] == 1
        _compare_bruteforce(pts, rad, 4.0)
        _compare_bruteforce(pts, rad, 0.0)


@pytest.mark.parametrize("pts", [
    [[0, 0, 0]],
    [[0, 0, 0], [2.5, 0, 0]],
    [[0, 0, 0], [2.5, 0, 0], [0.7, 2.2, 0]],
    [[0, 0, 0], [2.5, 0, 0], [5.1, 0, 0]],
    [[0, 0, 0], [2.5, 0, 0], [0.7, 2.2, 0], [2.9, 2.4, 0], [1.4, -2.0, 0]],
])
def test_bruteforce_low_dimensional(pts):
    """Fewer than four balls, collinear or coplanar centres: D is not 3-D."""
    xyz = np.array(pts, dtype=float)
    for alpha in (0.0, 1.0, 6.0):
        _compare_bruteforce(xyz, np.full(len(xyz), 1.6), alpha)


def test_two_ball_closed_form():
    """Two balls: the edge is in D with Size = OrthoSize = -(radius of the
    intersection circle)^2, the radical plane being at distance
    t = (d^2 + r0^2 - r1^2) / (2d) from p0; vertex i keeps Size -r_i^2 unless
    its own centre is closer in power to the other ball (d^2 < r_j^2 - r_i^2)."""
    rng = random.Random(9)
    for _ in range(40):
        d = rng.randint(500, 4000) / 1000.0
        r0, r1 = rng.randint(800, 2500) / 1000.0, rng.randint(800, 2500) / 1000.0
        xyz = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
        dq, w0, w1 = Fraction(int(round(d * 1000))), Fraction(int(round(r0 * 1000))) ** 2, Fraction(int(round(r1 * 1000))) ** 2
        t = (dq * dq + w0 - w1) / (2 * dq)
        edge = t * t - w0  # = -(r0^2 - t^2)
        v0 = -w0 if dq * dq >= w1 - w0 else edge
        v1 = -w1 if dq * dq >= w0 - w1 else edge
        for alpha in (0.0, 1.0, -1.0):
            c = oracle.alpha_complex(xyz, np.array([r0, r1]), alpha)
            aq = int(round(alpha * 1e6))
            want_edge = edge <= aq
            assert (len(c.simplices[1]) == 1) == want_edge
            if want_edge:
                assert abs(c.sizes[1][0] - float(edge) / 1e6) < 1e-9
            got_v = {int(s[0]): z for s, z in zip(c.simplices[0], c.sizes[0])}
            for i, v in ((0, v0), (1, v1)):
                assert (i in got_v) == (v <= aq)
                if i in got_v:
                    assert abs(got_v[i] - float(v) / 1e6) < 1e-9


def test_three_ball_triangle_closed_form():
    """Three balls: the triangle is in D and its Size is its OrthoSize, the
    power of the radical centre, found here as the point of the plane where
    the three radical planes meet (solved in the plane's own coordinates)."""
    rng = random.Random(21)
    for _ in range(20):
        pts = [(0, 0, 0), (rng.randint(2000, 3500), 0, 0), (rng.randint(-500, 2000), rng.randint(2000, 3500), 0)]
        R = [rng.randint(1400, 2200) for _ in range(3)]
        W = [Fraction(r * r) for r in R]
        # c = (x, y, 0): |c - p_k|^2 - W_k equal for k = 0, 1, 2
        (x1, _, _), (x2, y2, _) = pts[1], pts[2]
        # 2 x x1 = x1^2 - W1 + W0 ; 2 x x2 + 2 y y2 = x2^2 + y2^2 - W2 + W0
        x = (Fraction(x1 * x1) - W[1] + W[0]) / (2 * x1)
        y = (Fraction(x2 * x2 + y2 * y2) - W[2] + W[0] - 2 * x * x2) / (2 * y2)
        os_ = x * x + y * y - W[0]
        xyz = np.array(pts, dtype=float) / 1000.0
        c = oracle.alpha_complex(xyz, np.array(R) / 1000.0, 50.0)
        assert c.simplices[2].tolist() == [[0, 1, 2]]
        assert abs(c.sizes[2][0] - float(os_) / 1e6) < 1e-9


@pytest.mark.parametrize("seed", range(5))
def test_euler_matches_cech_nerve(seed):
    rng = random.Random(500 + seed)
    for _ in range(4):
        n = rng.choice([6, 8, 10])
        xyz = np.array([[rng.randint(-4000, 4000) / 1000 for _ in range(3)] for _ in range(n)])
        rad = np.array([rng.randint(1200, 2000) / 1000 for _ in range(n)])
        for alpha in (0.0, 1.5):
            c = oracle.alpha_complex(xyz, rad, alpha)
            assert c.euler() == cech.union_euler(xyz, rad, alpha)


@pytest.fixture(scope="module")
def small_mol():
    return synth.config_small()


def test_insertion_order_independent(small_mol):
    base = oracle.alpha_complex(small_mol.xyz, small_mol.radii, 0.0)
    for s in (1, 2):
        c = oracle.alpha_complex(small_mol.xyz, small_mol.radii, 0.0, order_seed=s)
        for d in range(4):
            assert np.array_equal(base.simplices[d], c.simplices[d])
            assert np.array_equal(base.sizes[d], c.sizes[d])


def test_delaunay_is_a_ball(small_mol):
    c = oracle.alpha_complex(small_mol.xyz, small_mol.radii, 0.0)
    v, e, f, t = c.d_count
    assert v - e + f - t == 1
    assert c.n_hidden == 0


def test_every_atom_is_a_vertex(small_mol):
    """No centre lies in another ball's power cell for these radii and the
    2.4 A separation, so K^0 holds every atom with Size -r^2."""
    c = oracle.alpha_complex(small_mol.xyz, small_mol.radii, 0.0)
    assert c.simplices[0][:, 0].tolist() == list(range(small_mol.n))
    assert np.allclose(c.sizes[0], -(small_mol.R_mA.astype(np.float64) ** 2) / 1e6, rtol=0, atol=1e-12)


def test_rigid_motions_and_relabelling(small_mol):
    base = oracle.alpha_complex(small_mol.xyz, small_mol.radii, 0.5)
    X = small_mol.X_mA.astype(np.int64)
    # translation by a lattice vector, axis permutation with reflections
    moved = (X[:, [2, 0, 1]] * np.array([-1, 1, -1]) + np.array([1234, -567, 89])) / 1000.0
    c = oracle.alpha_complex(moved, small_mol.radii, 0.5)
    for d in range(4):
        assert np.array_equal(base.simplices[d], c.simplices[d])
        assert np.allclose(base.sizes[d], c.sizes[d], rtol=1e-12, atol=1e-12)
    # relabelling (these inputs have no exact ties, so SoS never decides)
    perm = np.random.RandomState(4).permutation(small_mol.n)
    c = oracle.alpha_complex(small_mol.xyz[perm], small_mol.radii[perm], 0.5)
    for d in range(4):
        mapped = np.sort(perm[c.simplices[d]], axis=1)
        a = sorted(map(tuple, mapped.tolist()))
        assert a == list(map(tuple, base.simplices[d].tolist()))


def test_closure_monotonicity_and_sizes(small_mol):
    ks = [oracle.alpha_complex(small_mol.xyz, small_mol.radii, a) for a in (0.0, 1.0, 2.0)]
    for c, a in zip(ks, (0.0, 1.0, 2.0)):
        sets = _as_sets(c)
        size = [dict(zip(map(tuple, c.simplices[d].tolist()), c.sizes[d])) for d in range(4)]
        for d in range(1, 4):
            for s in sets[d]:
                for face in itertools.combinations(s, d):
                    assert face in sets[d - 1]
                    assert size[d - 1][face] <= size[d][s] + 1e-12
        for d in range(4):
            assert all(z <= a + 1e-12 for z in c.sizes[d])
    for lo, hi in zip(ks, ks[1:]):
        for d in range(4):
            assert _as_sets(lo)[d] <= _as_sets(hi)[d]


def test_filtration_by_size(small_mol):
    """K_alpha is the part of K_alpha_max with Size <= alpha, Sizes unchanged
    (Size is the least alpha at which a simplex enters, Sec. 2.4): the
    reading the alpha sweep rests on. Checked on the 1,000-atom molecule, its
    solvent-accessible form and the brute-force lattice sizes; none of these
    Sizes lies within rounding of the alpha values used."""
    cases = [(small_mol.xyz, small_mol.radii), (small_mol.with_sas().xyz, small_mol.with_sas().radii)]
    for xyz, rad in cases:
        top = oracle.alpha_complex(xyz, rad, 2.0)
        for alpha in (-1.0, 0.0, 0.35, 1.0, 2.0):
            c = oracle.alpha_complex(xyz, rad, alpha)
            for d in range(4):
                keep = top.sizes[d] <= alpha
                assert np.array_equal(top.simplices[d][keep], c.simplices[d]), (alpha, d)
                assert np.array_equal(top.sizes[d][keep], c.sizes[d]), (alpha, d)


def test_locality_of_regions():
    """Membership and Size of a simplex depend only on balls within a few
    grown radii of its vertices (AC2 violators meet its ortho-centre; its
    cofaces and their violators lie within 4 s_g): the oracle on the balls
    within 12 A of a cube of half-width 8 A agrees with the oracle on all
    100,000 balls on every simplex inside the cube. The full-size GPU test
    relies on this."""
    m = synth.config_100k()
    full = oracle.alpha_complex(m.xyz, m.radii, 0.0)
    rng = np.random.RandomState(7)
    for ca in rng.choice(m.n, 4, replace=False):
        dist = np.abs(m.xyz - m.xyz[ca]).max(axis=1)
        sel = np.nonzero(dist <= 20.0)[0]
        inner = dist <= 8.0
        part = oracle.alpha_complex(m.xyz[sel], m.radii[sel], 0.0)
        for d in range(4):
            g = full.simplices[d].astype(np.int64)
            keep = np.all(inner[g], axis=1)
            w = sel[part.simplices[d]]
            wk = np.all(inner[w], axis=1)
            assert keep.sum() > 0 or d == 3
            assert np.array_equal(g[keep], w[wk]), (ca, d)
            assert np.array_equal(full.sizes[d][keep], part.sizes[d][wk]), (ca, d)


def test_rejects_bad_input():
    good = np.zeros((2, 3)), np.ones(2)
    with pytest.raises(oracle.OracleError) as e:
        oracle.alpha_complex(np.zeros((2, 3)), np.ones(2), 0.0)
    assert e.value.status == 2
    with pytest.raises(oracle.OracleError) as e:
        oracle.alpha_complex(np.array([[0, 0, 0], [1, 1, 1.0]]), np.array([1.0, -1.0]), 0.0)
    assert e.value.status == 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.alpha_complex(np.array([[0, 0, 0], [600, 0, 0.0]]), np.ones(2), 0.0)
    assert e.value.status == 3
    with pytest.raises(oracle.OracleError) as e:
        oracle.alpha_complex(np.array([[0, 0, 0], [1, np.nan, 0.0]]), np.ones(2), 0.0)
    assert e.value.status == 1
    del good


@pytest.mark.slow
def test_oracle_100k_invariants():
    """100,000-atom ball: insertion order does not matter, D is a 3-ball, and
    every atom is a vertex of K_0 with Size -r^2 (vdW and solvent radii)."""
    m = synth.config_100k()
    for mol in (m, m.with_sas()):
        a = oracle.alpha_complex(mol.xyz, mol.radii, 0.0)
        b = oracle.alpha_complex(mol.xyz, mol.radii, 0.0, order_seed=5)
        for d in range(4):
            assert np.array_equal(a.simplices[d], b.simplices[d])
            assert np.array_equal(a.sizes[d], b.sizes[d])
        v, e, f, t = a.d_count
        assert v - e + f - t == 1 and a.n_hidden == 0
        assert a.counts()[0] == mol.n


def test_quantisation_rounds_half_to_even():
    """Coordinates and radii are rounded to integer milli-angstrom, half to
    even (the reading of the 0.001 A input lattice; the paper fixes no rule).
    Multiples of 1/16 A are exact binary values whose x 1000 ends in .5, so a
    half-away-from-zero rounding would change every value below.
    - one ball of radius 1.0625 A: R = 1062 mA (half-away: 1063), so its
      vertex Size is -1062^2 mA^2 = -1.127844 A^2; radius 1.1875 A: R = 1188,
      Size -1.411344 A^2 (ties go up as well as down);
    - two balls of radius 1.5 A at x = -0.0625 and x = 2.0625 A: centres -62
      and 2062 mA, d = 2124 mA; equal weights put the radical plane at d / 2,
      so the edge's Size is (d / 2)^2 - 1500^2 = 1127844 - 2250000 mA^2
      = -1.122156 A^2 (half-away: d = 2126, -1.120031)."""
    for r, want in ((1.0625, -1.127844), (1.1875, -1.411344), (0.0625 + 1.5, -(1562 ** 2) / 1e6)):
        c = oracle.alpha_complex(np.array([[0.0625, -0.1875, 0.3125]]), np.array([r]), 0.0)
        assert c.counts() == [1, 0, 0, 0]
        assert c.sizes[0][0] == want, (r, c.sizes[0][0], want)
    xyz = np.array([[-0.0625, 0.0625, -0.1875], [2.0625, 0.0625, -0.1875]])
    c = oracle.alpha_complex(xyz, np.array([1.5, 1.5]), 0.0)
    assert c.simplices[1].tolist() == [[0, 1]]
    assert abs(c.sizes[1][0] - (-1.122156)) <= 1e-12
    # the tie along y and z: 2.0625 A apart on y, the pair shifted on z by a tie
    xyz = np.array([[0.0, -0.0625, 0.1875], [0.0, 2.0625, 0.1875]])
    c = oracle.alpha_complex(xyz, np.array([1.5, 1.5]), 0.0)
    assert abs(c.sizes[1][0] - (-1.122156)) <= 1e-12


def _planar_molecule(n, seed, spacing=2.4):
    """n centres on the plane z = 0 (dart throwing with minimum separation
    `spacing` at 0.1 atoms per A^2 in a disk, on a background grid of cells
    of side spacing / sqrt(2): at most one centre per cell), vdW radii."""
    rng = np.random.RandomState(seed)
    R = math.sqrt(n / (math.pi * 0.1))
    h = spacing / math.sqrt(2.0)
    grid = {}
    pts = []
    while len(pts) < n:
        p = rng.uniform(-R, R, 2)
        if p @ p > R * R:
            continue
        cx, cy = int(math.floor(p[0] / h)), int(math.floor(p[1] / h))
        near = (grid.get((cx + i, cy + j)) for i in range(-2, 3) for j in range(-2, 3))
        if all(q is None or (p - q) @ (p - q) >= spacing * spacing for q in near):
            grid[(cx, cy)] = p
            pts.append(p)
    xyz = np.zeros((n, 3))
    xyz[:, :2] = np.round(np.array(pts) * 1000) / 1000
    rad = rng.choice([1.70, 1.55, 1.52, 1.80], size=n, p=[0.62, 0.17, 0.19, 0.02])
    return xyz, rad


def test_bruteforce_coplanar_molecule():
    """Twenty coplanar balls of a planar molecule: the low-dimensional route
    against the definition-level brute force."""
    xyz, rad = _planar_molecule(20, 31)
    for alpha in (0.0, 1.0, 4.0):
        _compare_bruteforce(xyz, rad, alpha)


@pytest.mark.parametrize("n", [150, 600, 3000])
def test_coplanar_route_against_lifted_apex(n):
    """All centres on one plane, more balls than a brute force can take. Adding
    one tiny ball 300 A off the plane makes the input three-dimensional (the
    incremental triangulation then builds it) without changing any simplex of
    Size <= alpha on the plane: the apex is farther in power than 300^2 A^2
    from every planar ortho-centre, so it violates none of them, and every
    simplex through it has OrthoSize above 150^2 A^2. The planar part of the
    lifted complex must therefore equal the low-dimensional route's result,
    simplex for simplex and Size for Size."""
    xyz, rad = _planar_molecule(n, 40 + n)
    apex = np.vstack([xyz, [[xyz[:, 0].mean(), xyz[:, 1].mean(), 300.0]]])
    arad = np.append(rad, 0.001)
    for alpha in (0.0, 1.0, 5.0):
        flat = oracle.alpha_complex(xyz, rad, alpha)
        assert flat.d_count[0] == -1  # the low-dimensional route ran
        lifted = oracle.alpha_complex(apex, arad, alpha)
        assert lifted.d_count[0] > 0  # the three-dimensional route ran
        for d in range(4):
            keep = np.all(lifted.simplices[d] < n, axis=1)
            assert np.array_equal(flat.simplices[d], lifted.simplices[d][keep]), (n, alpha, d)
            assert np.array_equal(flat.sizes[d], lifted.sizes[d][keep]), (n, alpha, d)
        assert flat.counts()[3] == 0
        if alpha == 5.0:
            assert flat.counts()[2] > n // 4


def test_coplanar_beyond_route_limit_is_reported():
    """More than 4096 coplanar balls: the oracle reports the input as
    degenerate instead of answering."""
    k = np.arange(4097)
    xyz = np.stack([(k % 64) * 2.5, (k // 64) * 2.5, np.zeros(4097)], axis=1)
    with pytest.raises(oracle.OracleError) as e:
        oracle.alpha_complex(xyz, np.full(4097, 1.5), 0.0)
    assert e.value.status == 7
