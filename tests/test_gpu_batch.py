"""GPU batches of molecules: one call over concatenated molecules must give,
molecule by molecule, exactly the single-molecule result (ids shifted by the
molecule's offset; Sizes bit for bit), and the oracle's complex.
"""
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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _concat(mols):
    xyz = np.concatenate([m.xyz for m in mols])
    rad = np.concatenate([m.radii for m in mols])
    off = np.concatenate([[0], np.cumsum([m.n for m in mols])]).astype(np.int64)
    return xyz, rad, off


class _Slice:
    """One molecule's part of a batch result, ids made local."""

    def __init__(self, c, m, off):
        self._s = []
        self._z = []
        for d in range(4):
            rows = c.molecule_rows(d)
            self._s.append(c.simplices(d)[rows[m]:rows[m + 1]] - off[m])
            self._z.append(c.sizes(d)[rows[m]:rows[m + 1]])

    def count(self, d):
        return len(self._s[d])

    def counts(self):
        return [self.count(d) for d in range(4)]

    def simplices(self, d):
        return self._s[d]

    def sizes(self, d):
        return self._z[d]


def _check_batch(acx, mols, alpha, cells=None, oracle_upto=0, options=None):
    xyz, rad, off = _concat(mols)
    print(f"[case] batch of {len(mols)} molecules, {len(rad)} balls, alpha={alpha} {options}", flush=True)
    c = acx.ac_alpha_complex_batch(_dev(xyz), _dev(rad), off, alpha, cell_mA=cells, options=options)
    assert c.molecule_count() == len(mols)
    for d in range(4):
        rows = c.molecule_rows(d)
        want = np.repeat(np.arange(len(mols), dtype=np.int32), np.diff(rows))
        assert np.array_equal(c.molecule(d), want), d
    for m, mol in enumerate(mols):
        got = _Slice(c, m, off)
        single = acx.ac_alpha_complex_device(_dev(mol.xyz), _dev(mol.radii), alpha)
        for d in range(4):
            assert np.array_equal(got.simplices(d), single.simplices(d)), (m, d)
            assert np.array_equal(got.sizes(d), single.sizes(d)), (m, d)
        if m < oracle_upto:
            assert_same_complex(got, oracle.alpha_complex(mol.xyz, mol.radii, alpha), f"molecule {m}")
    return c


def test_uneven_sizes(acx):
    sizes = [60, 500, 2500, 140, 7, 1200, 3000, 1, 400]
    mols = [synth.molecule(k, 100 + i) for i, k in enumerate(sizes)]
    _check_batch(acx, mols, 0.0, oracle_upto=len(mols))


def test_overlapping_coordinates(acx):
    # the same molecule three times at the same place, and once with SAS
    # radii: balls of different molecules must never interact
    m = synth.molecule(800, 41)
    _check_batch(acx, [m, m, m.with_sas(1400), m], 0.0, oracle_upto=3)


def test_alpha_and_cell_sides(acx):
    mols = [synth.molecule(k, 200 + i) for i, k in enumerate([300, 1500, 900])]
    for alpha in (0.0, 1.0):
        _check_batch(acx, mols, alpha)
    # per-molecule cell sides change nothing
    _check_batch(acx, mols, 0.0, cells=np.array([900, 4000, 1700], dtype=np.int32))


def test_tuner(acx):
    mols = [synth.molecule(k, 300 + i) for i, k in enumerate([600, 2500, 900, 9000])]
    xyz, rad, off = _concat(mols)
    cells, buckets = acx.ac_tune_cells(_dev(xyz), _dev(rad), off, 0.0)
    assert cells.min() >= 1
    assert list(buckets) == [0, 1, 0, 2]
    assert cells[0] == cells[2]  # one side per bucket
    _check_batch(acx, mols, 0.0, cells=cells)


def test_errors(acx):
    m = synth.molecule(100, 3)
    X, R = _dev(m.xyz), _dev(m.radii)
    for off in ([1, 100], [0, 50, 50, 100], [0, 60, 40, 100]):
        with pytest.raises(acx.AlphaCxError) as e:
            acx.ac_alpha_complex_batch(X, R, np.array(off), 0.0)
        assert e.value.status == 1
    # a duplicate inside one molecule is an error; across molecules it is not
    xyz = np.concatenate([m.xyz, m.xyz[:1]])
    rad = np.concatenate([m.radii, m.radii[:1]])
    with pytest.raises(acx.AlphaCxError) as e:
        acx.ac_alpha_complex_batch(_dev(xyz), _dev(rad), np.array([0, 101]), 0.0)
    assert e.value.status == 2
    c = acx.ac_alpha_complex_batch(_dev(xyz), _dev(rad), np.array([0, 100, 101]), 0.0)
    assert c.counts()[0] == 101


def test_batch_union_measure(acx):
    """V and A over a batch complex are the sums of the molecules' own."""
    mols = [synth.molecule(k, 400 + i) for i, k in enumerate([700, 1300])]
    xyz, rad, off = _concat(mols)
    X, R = _dev(xyz), _dev(rad)
    c = acx.ac_alpha_complex_batch(X, R, off, 0.0)
    V, A = acx.ac_union_measure(c, X, R)
    Vs = As = 0.0
    for mol in mols:
        Xm, Rm = _dev(mol.xyz), _dev(mol.radii)
        v, a = acx.ac_union_measure(acx.ac_alpha_complex_device(Xm, Rm, 0.0), Xm, Rm)
        Vs += v
        As += a
    assert V == pytest.approx(Vs, rel=1e-12)
    assert A == pytest.approx(As, rel=1e-12)


def test_morton_cells_in_a_batch(acx):
    """Per-molecule Morton grids (each padded to a cube of 2^L cells, numbered
    one after the other): molecule by molecule the single result and the oracle."""
    sizes = [700, 30, 2200, 5, 1300]
    mols = [synth.molecule(k, 300 + i) for i, k in enumerate(sizes)]
    _check_batch(acx, mols, 0.0, oracle_upto=len(mols), options={"cell_order": 1})
    _check_batch(acx, mols, 1.5, cells=np.array([900, 4000, 1800, 2500, 3100]), options={"cell_order": 1})


def test_molecule_of_rows_only_for_batches(acx):
    m = synth.molecule(200, 3)
    c = acx.ac_alpha_complex_device(_dev(m.xyz), _dev(m.radii), 0.0)
    assert not acx.library().ac_molecule(c._h, 1)
    cb = acx.ac_alpha_complex_batch(_dev(m.xyz), _dev(m.radii), np.array([0, m.n]), 0.0)
    assert np.array_equal(cb.molecule(1), np.zeros(cb.count(1), dtype=np.int32))


@pytest.mark.timeout(900)
def test_full_512_molecule_batch_against_oracle(acx):
    """The batching workload itself: 512 molecules with sizes log-uniform in
    [500, 50000] atoms (seed 999; molecule k from seed 1000 + k; 5.1M balls),
    one batched call with the autotuner's cell sides as bench.py makes it,
    every molecule compared with the oracle simplex for simplex and Size for
    Size. The oracle runs in 16 threads (its C call releases the interpreter
    lock and keeps no shared state)."""
    from concurrent.futures import ThreadPoolExecutor
    from parity import SIZE_ABS_TOL, SIZE_REL_TOL
    sizes = synth.batch_sizes()
    print(f"[case] 512-molecule batch: generating {int(np.sum(sizes))} balls", flush=True)
    mols = [synth.molecule(int(k), 1000 + i) for i, k in enumerate(sizes)]
    xyz, rad, off = _concat(mols)
    X, R = _dev(xyz), _dev(rad)
    cells, _ = acx.ac_tune_cells(X, R, off, 0.0)
    c = acx.ac_alpha_complex_batch(X, R, off, 0.0, cell_mA=cells)
    simp = [c.simplices(d) for d in range(4)]
    size = [c.sizes(d) for d in range(4)]
    rows = [c.molecule_rows(d) for d in range(4)]
    c.close()
    print("[case] 512-molecule batch: oracle per molecule", flush=True)

    def check(m):
        want = oracle.alpha_complex(mols[m].xyz, mols[m].radii, 0.0)
        for d in range(4):
            got = simp[d][rows[d][m]:rows[d][m + 1]] - off[m]
            if not np.array_equal(got, want.simplices[d]):
                return f"molecule {m} dim {d}: {len(got)} vs {len(want.simplices[d])} simplices"
            z = size[d][rows[d][m]:rows[d][m + 1]]
            if np.any(np.abs(z - want.sizes[d]) > SIZE_ABS_TOL + SIZE_REL_TOL * np.abs(want.sizes[d])):
                return f"molecule {m} dim {d}: Sizes differ"
        return None

    with ThreadPoolExecutor(16) as ex:
        bad = [r for r in ex.map(check, range(len(mols))) if r]
    assert not bad, bad[:5]
