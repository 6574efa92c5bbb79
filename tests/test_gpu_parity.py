"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Simplex sets must be identical and Sizes within 1e-9 A^2 + 1e-12 relative
(every membership decision is exact on both sides; Sizes are float64 on the
GPU and exact rationals in the oracle).
"""
import random
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import assert_same_complex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def acx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_05944_amd as m
    return m


def _dev(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float64)).to("cuda:0")


def _run(acx, xyz, rad, alpha, **opt):
    print(f"[case] n={len(rad)} alpha={alpha} opt={opt}", flush=True)
    return acx.ac_alpha_complex_device(_dev(xyz), _dev(rad), alpha, options=opt or None)


def test_tiny_inputs(acx):
    cases = [
        ([[0, 0, 0]], [1.5]),
        ([[0, 0, 0], [2.5, 0, 0]], [1.5, 1.7]),
        ([[0, 0, 0], [2.5, 0, 0], [0.7, 2.2, 0]], [1.5, 1.7, 1.6]),
        ([[0, 0, 0], [2.5, 0, 0], [5.1, 0, 0]], [1.6, 1.6, 1.6]),
        ([[0, 0, 0], [2.5, 0, 0], [0.7, 2.2, 0], [2.9, 2.4, 0], [1.4, -2.0, 0]], [1.6] * 5),
        ([[0, 0, 0], [2.4, 0, 0], [0, 2.4, 0], [0, 0, 2.4], [2.0, 2.0, 2.0]], [1.7, 1.5, 1.6, 1.8, 1.5]),
    ]
    for xyz, rad in cases:
        xyz, rad = np.array(xyz, dtype=float), np.array(rad, dtype=float)
        for alpha in (0.0, 1.0, 6.0):
            assert_same_complex(_run(acx, xyz, rad, alpha), oracle.alpha_complex(xyz, rad, alpha), f"n={len(rad)}")


def test_dense_neighbourhoods(acx):
    """Balls with many neighbours (long neighbour rows, many candidates per
    ball), built twice in a row on reused device memory."""
    m = synth.molecule(4000, 21).with_sas(2200)  # radii ~3.9 A: ~60 neighbours per ball
    want = oracle.alpha_complex(m.xyz, m.radii, 0.0)
    for _ in range(2):
        assert_same_complex(_run(acx, m.xyz, m.radii, 0.0), want, "dense")


def test_hub_ball_beyond_emit_lds(acx):
    """A ball of radius 8 A at index 0 touched by 3,600 balls of radius
    0.45 A spread over a sphere of radius 8.2 A around it: the hub is the least
    id of more kept edges, triangles and tetrahedra than an emit block orders
    in LDS (2,048 rows for edges and triangles, 512 for tetrahedra), so its
    buckets are finished through global scratch."""
    n = 3600
    k = np.arange(n) + 0.5
    phi, th = np.arccos(1 - 2 * k / n), np.pi * (1 + 5 ** 0.5) * k
    shell = 8.2 * np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    xyz = np.vstack([[0.0, 0.0, 0.0], shell])
    rad = np.concatenate([[8.0], np.full(n, 0.45)])
    for alpha in (0.0, 1.0):
        want = oracle.alpha_complex(xyz, rad, alpha)
        hub_rows = [int((want.simplices[d][:, 0] == 0).sum()) for d in (1, 2, 3)]
        assert hub_rows[0] > 2048 and hub_rows[1] > 2048 and hub_rows[2] > 512, hub_rows
        assert_same_complex(_run(acx, xyz, rad, alpha), want, f"hub alpha={alpha}")


def test_random_small(acx):
    rng = random.Random(42)
    for trial in range(40):
        n = rng.choice([4, 6, 10, 20, 40])
        box = rng.choice([3.0, 5.0, 8.0])
        xyz = np.array([[rng.randint(-int(box * 1000), int(box * 1000)) / 1000 for _ in range(3)] for _ in range(n)])
        xyz = np.unique(xyz, axis=0)
        rad = np.array([rng.choice([1.2, 1.5, 1.7, 2.0, 0.5]) for _ in range(len(xyz))])
        alpha = rng.choice([0.0, 1.0, -0.5, 4.0, 20.0])
        assert_same_complex(_run(acx, xyz, rad, alpha), oracle.alpha_complex(xyz, rad, alpha), f"trial {trial}")


@pytest.mark.parametrize("rad", [1.0, 1.5])
def test_cubic_lattice_ties(acx, rad):
    """4x4x4 cubic lattice, equal radii: every cube has eight co-spherical
    centres; simulation of simplicity decides, and alpha = 2.0 / 0.75 hits the
    cube-corner tetrahedra's OrthoSize exactly."""
    pts = np.array([[2.0 * i, 2.0 * j, 2.0 * k] for i in range(4) for j in range(4) for k in range(4)])
    for perm_seed in (None, 3):
        p = pts if perm_seed is None else pts[np.random.RandomState(perm_seed).permutation(len(pts))]
        r = np.full(len(p), rad)
        for alpha in (0.0, 0.75, 1.0, 2.0, 3.0):
            assert_same_complex(_run(acx, p, r, alpha), oracle.alpha_complex(p, r, alpha), f"lattice a={alpha}")


def test_integer_grid_ties(acx):
    rng = random.Random(8)
    for trial in range(10):
        pts = np.unique(np.array([[rng.randint(-4, 4) for _ in range(3)] for _ in range(60)], dtype=float), axis=0)
        pts = pts[np.random.RandomState(trial).permutation(len(pts))]
        rad = np.array([rng.choice([1.0, 1.5]) for _ in range(len(pts))])
        alpha = rng.choice([0.0, 0.5, 2.0, 8.0])
        assert_same_complex(_run(acx, pts, rad, alpha), oracle.alpha_complex(pts, rad, alpha), f"grid {trial}")


def test_quantisation_ties(acx):
    """Coordinates and radii on multiples of 1/16 A: x 1000 ends in .5 for odd
    multiples, so every such value is a rounding tie (half to even on both
    sides). The hand-derived Sizes of the oracle's pins, then a molecule
    snapped to the 1/16 A lattice with tie radii, against the oracle."""
    c = _run(acx, [[0.0625, -0.1875, 0.3125]], [1.0625], 0.0)
    assert c.sizes(0).tolist() == [-1.127844]
    c = _run(acx, [[-0.0625, 0.0625, -0.1875], [2.0625, 0.0625, -0.1875]], [1.5, 1.5], 0.0)
    assert c.simplices(1).tolist() == [[0, 1]] and abs(c.sizes(1)[0] + 1.122156) <= 1e-12
    m = synth.molecule(2000, 12)
    snapped = np.round(m.xyz * 16.0) / 16.0
    rad = np.choose(np.arange(m.n) % 4, [1.5625, 1.6875, 1.5, 1.8125])  # 1562.5 1687.5 1500 1812.5 mA
    assert np.mean(np.abs(snapped * 1000 - np.round(snapped * 1000)) == 0.5) > 0.4  # mostly ties
    for alpha in (0.0, 1.0625):
        assert_same_complex(_run(acx, snapped, rad, alpha), oracle.alpha_complex(snapped, rad, alpha),
                            f"1/16 A lattice alpha={alpha}")


def test_planar_molecule(acx):
    """3,000 balls on one plane (a planar molecule: the complex has no
    tetrahedra), against the oracle's low-dimensional route."""
    rng = np.random.RandomState(77)
    pts = []
    grid = {}
    R = np.sqrt(3000 / (np.pi * 0.1))
    while len(pts) < 3000:
        p = rng.uniform(-R, R, 2)
        if p @ p > R * R:
            continue
        key = (int(np.floor(p[0] / 1.7)), int(np.floor(p[1] / 1.7)))
        near = [grid.get((key[0] + i, key[1] + j)) for i in range(-2, 3) for j in range(-2, 3)]
        if all(q is None or (p - q) @ (p - q) >= 2.4 ** 2 for q in near):
            grid[key] = p
            pts.append(p)
    xyz = np.zeros((3000, 3))
    xyz[:, 0], xyz[:, 2] = np.round(np.array(pts) * 1000).T / 1000
    xyz[:, 1] = -3.21
    rad = rng.choice([1.70, 1.55, 1.52, 1.80], size=3000, p=[0.62, 0.17, 0.19, 0.02])
    for alpha in (0.0, 2.0):
        c = _run(acx, xyz, rad, alpha)
        assert c.count(3) == 0
        assert_same_complex(c, oracle.alpha_complex(xyz, rad, alpha), f"plane alpha={alpha}")


def test_small_molecule_alphas(acx):
    m = synth.config_small()
    for alpha in (0.0, 0.5, 1.0, 2.0):
        assert_same_complex(_run(acx, m.xyz, m.radii, alpha), oracle.alpha_complex(m.xyz, m.radii, alpha),
                            f"1k a={alpha}")


def test_options_do_not_change_result(acx):
    """Exact-only predicates and other cell sizes give the same simplices and
    bit-identical Sizes (each OrthoSize is evaluated with the vertices in a
    canonical order of their centres)."""
    m = synth.molecule(2000, 11)
    want = oracle.alpha_complex(m.xyz, m.radii, 1.0)
    base = _run(acx, m.xyz, m.radii, 1.0)
    assert_same_complex(base, want, "default")
    for opt in ({"force_exact": 1}, {"cell_mA": 900}, {"cell_mA": 4000}, {"cell_mA": 2500, "force_exact": 1},
                {"cell_order": 1}, {"cell_order": 1, "cell_mA": 900}, {"cell_order": 1, "cell_mA": 4000}):
        got = _run(acx, m.xyz, m.radii, 1.0, **opt)
        assert_same_complex(got, want, str(opt))
        for d in range(4):
            assert np.array_equal(got.sizes(d), base.sizes(d)), (opt, d)


@pytest.mark.parametrize("sas,alpha,cells", [(False, 0.0, (3600, 4000, 5000)), (False, 0.2, (3800,)),
                                              (True, 0.0, (6400, 7000))])
def test_one_cell_reach(acx, sas, alpha, cells):
    """Cell sides of one-cell reach (the neighbour scan covers 3 x 3 x 3
    cells), including solvent-accessible radii at 6.4 and 7 A cells, whose
    rows outgrow the slot (counted fill). Every side gives the oracle's
    complex."""
    m = synth.molecule(6000, 17, sas=sas)
    want = oracle.alpha_complex(m.xyz, m.radii, alpha)
    for side in cells:
        print(f"[case] one-cell reach sas={sas} alpha={alpha} cell_mA={side}", flush=True)
        got = _run(acx, m.xyz, m.radii, alpha, cell_mA=side)
        assert_same_complex(got, want, f"sas={sas} alpha={alpha} cell_mA={side}")


@pytest.mark.parametrize("sas", [False, True])
def test_morton_order_100k(acx, sas):
    """The 100k-atom molecule with cells on a Morton curve: the same complex as
    with row-major cells, bit for bit (the solvent-accessible radii take the
    counted-fill neighbour path)."""
    m = synth.config_100k(sas=sas)
    a = _run(acx, m.xyz, m.radii, 0.0)
    b = _run(acx, m.xyz, m.radii, 0.0, cell_order=1)
    for d in range(4):
        assert np.array_equal(a.simplices(d), b.simplices(d)), d
        assert np.array_equal(a.sizes(d), b.sizes(d)), d


def test_stage_events(acx):
    """profile=1 times every stage of the build (the two AC2 stages of the
    per-step arrangement are not run: -1); profile=2+i only stage i (the others
    -1); profile=2+stage count runs the AC2 tests of edges and triangles as
    kernels of their own and times every stage. None changes the result."""
    m = synth.molecule(2000, 13)
    base = _run(acx, m.xyz, m.radii, 0.0)
    names = acx.stage_names()
    split_only = {"edges_ac2", "triangles_ac2"}
    full = _run(acx, m.xyz, m.radii, 0.0, profile=1)
    assert all((v >= 0) != (k in split_only) for k, v in full.stage_ms().items()), full.stage_ms()
    for i in (0, names.index("triangles_count"), names.index("emit")):
        one = _run(acx, m.xyz, m.radii, 0.0, profile=2 + i)
        ms = one.stage_ms()
        assert ms[names[i]] >= 0
        assert all(v == -1.0 for k, v in ms.items() if k != names[i])
        for d in range(4):
            assert np.array_equal(one.simplices(d), base.simplices(d))
            assert np.array_equal(one.sizes(d), base.sizes(d))
    for alpha in (0.0, 1.5):
        ref = _run(acx, m.xyz, m.radii, alpha)
        split = _run(acx, m.xyz, m.radii, alpha, profile=2 + len(names))
        assert all(v >= 0 for v in split.stage_ms().values()), split.stage_ms()
        for d in range(4):
            assert np.array_equal(split.simplices(d), ref.simplices(d))
            assert np.array_equal(split.sizes(d), ref.sizes(d))
    s = synth.config_100k(sas=True)  # counted-fill neighbour path, split arrangement
    ref = _run(acx, s.xyz, s.radii, 0.0)
    split = _run(acx, s.xyz, s.radii, 0.0, profile=2 + len(names))
    for d in range(4):
        assert np.array_equal(split.simplices(d), ref.simplices(d))


def test_host_path_matches(acx):
    m = synth.molecule(1500, 12)
    got = acx.ac_alpha_complex(m.xyz, m.radii, 0.0)
    assert_same_complex(got, oracle.alpha_complex(m.xyz, m.radii, 0.0), "host path")


def test_errors(acx):
    with pytest.raises(acx.AlphaCxError) as e:
        _run(acx, np.zeros((2, 3)), np.ones(2), 0.0)
    assert e.value.status == 2
    with pytest.raises(acx.AlphaCxError) as e:
        _run(acx, np.array([[0, 0, 0], [1, np.nan, 0.0]]), np.ones(2), 0.0)
    assert e.value.status == 1
    with pytest.raises(acx.AlphaCxError) as e:
        _run(acx, np.array([[0, 0, 0], [600, 0, 0.0]]), np.ones(2), 0.0)
    assert e.value.status == 3
    with pytest.raises(acx.AlphaCxError) as e:
        _run(acx, np.array([[0, 0, 0], [3, 0, 0.0]]), np.array([1.0, 0.0]), 0.0)
    assert e.value.status == 1
    # alpha so negative that no ball is left: an empty complex, not an error
    c = _run(acx, np.array([[0, 0, 0], [3, 0, 0.0]]), np.ones(2), -5.0)
    assert c.counts() == [0, 0, 0, 0]


@pytest.mark.parametrize("sas,alpha", [(False, 1.0), (False, 2.5), (True, 0.5)])
def test_100k_alpha_parity(acx, sas, alpha):
    """alpha > 0 at full 100k size: the wide neighbour slots (grown radius
    1.9-2.6 A) and, with SAS radii, the counted-fill path."""
    m = synth.config_100k(sas=sas)
    got = _run(acx, m.xyz, m.radii, alpha)
    assert_same_complex(got, oracle.alpha_complex(m.xyz, m.radii, alpha), f"100k sas={sas} alpha={alpha}")


@pytest.mark.parametrize("sas", [False, True])
def test_100k_full_parity(acx, sas):
    m = synth.config_100k(sas=sas)
    got = _run(acx, m.xyz, m.radii, 0.0)
    assert_same_complex(got, oracle.alpha_complex(m.xyz, m.radii, 0.0), f"100k sas={sas}")

