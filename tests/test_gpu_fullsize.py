"""Full-size parity on the 3M-atom shell, built as bench.py builds it (cell
side 3.6 A, default options).

- Sampled regions: membership and Size of a simplex depend only on balls
  within a few grown radii of its vertices (AC2 violators meet its
  ortho-centre, cofaces share its vertices' neighbours, and their AC2 the
  same again: 4 s_g = 7.2 A at alpha = 0). For cubes of half-width 8 A
  around sampled balls, the oracle is run on the balls within 12 A more, and
  the simplices with every vertex in the cube must agree exactly (Sizes to
  the oracle tolerance).
- Properties that hold at any size, on the whole output: every ball a vertex
  with Size -r^2, every facet of every simplex present, Size never smaller
  on a coface than on its facets, every Size <= alpha, rows sorted.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from parity import SIZE_ABS_TOL, SIZE_REL_TOL

pytestmark = pytest.mark.gpu

HALF = 8.0     # A, half-width of a sampled cube
MARGIN = 12.0  # A, extra balls given to the oracle around it


@pytest.fixture(scope="module")
def built():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_05944_amd as acx
    print("[case] 3M shell: generating the input (about a minute without a cache)", flush=True)
    mol = synth.config_shell_3m(os.environ.get("ALPHACX_INPUT_CACHE") or None)
    X = torch.from_numpy(mol.xyz).cuda()
    R = torch.from_numpy(mol.radii).cuda()
    print("[case] 3M shell: building", flush=True)
    c = acx.ac_alpha_complex_device(X, R, 0.0, options={"cell_mA": 3600})
    simp = [c.simplices(d).astype(np.int64) for d in range(4)]
    size = [c.sizes(d) for d in range(4)]
    counts = c.counts()
    c.close()
    return mol, simp, size, counts


@pytest.mark.timeout(900)
def test_whole_output_against_oracle(built):
    """Every simplex and Size of the 3M-atom shell against the oracle run on
    all 3,000,000 balls (single-threaded, in this process)."""
    mol, simp, size, counts = built
    print("[case] 3M shell: oracle on all balls", flush=True)
    want = oracle.alpha_complex(mol.xyz, mol.radii, 0.0)
    assert want.counts() == counts, (want.counts(), counts)
    for d in range(4):
        assert np.array_equal(simp[d], want.simplices[d]), d
        err = np.abs(size[d] - want.sizes[d])
        bad = np.nonzero(err > SIZE_ABS_TOL + SIZE_REL_TOL * np.abs(want.sizes[d]))[0]
        assert bad.size == 0, (d, want.simplices[d][bad[:3]].tolist(), size[d][bad[:3]], want.sizes[d][bad[:3]])


def _rows_in(rows, inside):
    return rows[np.all(inside[rows], axis=1)]


def test_sampled_regions_against_oracle(built):
    mol, simp, size, _ = built
    xyz = mol.xyz
    rng = np.random.RandomState(7)
    for centre_atom in rng.choice(mol.n, 4, replace=False):
        c0 = xyz[centre_atom]
        dist = np.abs(xyz - c0).max(axis=1)
        sel = np.nonzero(dist <= HALF + MARGIN)[0]  # ascending: input order kept
        inner = dist <= HALF
        print(f"[case] region around ball {centre_atom}: {inner.sum()} inner, {len(sel)} given to the oracle",
              flush=True)
        want = oracle.alpha_complex(xyz[sel], mol.radii[sel], 0.0)
        for d in range(4):
            keep = np.all(inner[simp[d]], axis=1)
            got_rows, got_size = simp[d][keep], size[d][keep]
            w_rows = sel[want.simplices[d]]
            w_keep = np.all(inner[w_rows], axis=1)
            w_rows, w_size = w_rows[w_keep], want.sizes[d][w_keep]
            assert np.array_equal(got_rows, w_rows), (centre_atom, d, len(got_rows), len(w_rows))
            assert np.all(np.abs(got_size - w_size) <= SIZE_ABS_TOL + SIZE_REL_TOL * np.abs(w_size)), (centre_atom, d)


def _pair_key(rows, n):
    return rows[:, 0] * n + rows[:, 1]


def _find_rows(table, queries, n):
    """Whether each query row (K ids, ascending) is a row of `table` (rows
    sorted lexicographically), for K = 1, 2, 3."""
    k = table.shape[1]
    if k == 1:
        key, q = table[:, 0], queries[:, 0]
    elif k == 2:
        key, q = _pair_key(table, n), _pair_key(queries, n)
    else:
        ab = _pair_key(table, n)
        uab, inv = np.unique(ab, return_inverse=True)
        key = inv.astype(np.int64) * (1 << 26) + table[:, 2]
        qab = _pair_key(queries, n)
        idx = np.clip(np.searchsorted(uab, qab), 0, len(uab) - 1)
        ok = uab[idx] == qab
        q = np.where(ok, idx.astype(np.int64) * (1 << 26) + queries[:, 2], -1)
    pos = np.clip(np.searchsorted(key, q), 0, len(key) - 1)
    return key[pos] == q, pos


def test_whole_output_properties(built):
    mol, simp, size, counts = built
    n = mol.n
    assert counts[0] == n
    assert np.array_equal(simp[0][:, 0], np.arange(n))
    assert np.allclose(size[0], -(mol.R_mA.astype(np.float64) ** 2) / 1e6, rtol=0, atol=1e-12)
    for d in range(4):
        rows = simp[d]
        assert np.all(np.diff(rows, axis=1) > 0), d  # ascending ids inside a row
        if d >= 1 and len(rows) > 1:
            key = _pair_key(rows, n) if d >= 1 else rows[:, 0]
            if d == 1:
                assert np.all(np.diff(key) > 0)
            else:
                assert np.all(np.diff(key) >= 0)
        assert np.all(size[d] <= 1e-12), d
    for d in range(1, 4):
        rows, sz = simp[d], size[d]
        for drop in range(d + 1):
            face = np.delete(rows, drop, axis=1)
            found, pos = _find_rows(simp[d - 1], face, n)
            assert found.all(), (d, drop, int((~found).sum()))
            fs = size[d - 1][pos]
            assert np.all(fs <= sz + SIZE_ABS_TOL + SIZE_REL_TOL * np.abs(sz)), (d, drop)
