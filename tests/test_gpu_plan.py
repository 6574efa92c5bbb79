"""Recorded batch builds (ac_plan_*): the pipeline captured once in a HIP
graph and replayed on new coordinates, against ac_alpha_complex_batch on the
same arrays (bit for bit: rows, Sizes and molecule rows), with eager work and
synchronisations between the replays; inputs that no longer fit the recording
stop the replay, and the result is then the ordinary build's. One molecule of
the batch is also checked against the oracle.
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


def _same(a, b, what):
    assert a.counts() == b.counts(), (what, a.counts(), b.counts())
    for d in range(4):
        assert np.array_equal(a.simplices(d), b.simplices(d)), (what, d)
        assert np.array_equal(a.sizes(d).view(np.int64), b.sizes(d).view(np.int64)), (what, d)
        assert np.array_equal(a.molecule_rows(d), b.molecule_rows(d)), (what, d)


@pytest.fixture(scope="module")
def batch():
    sizes = np.exp(np.log(500) + np.linspace(0, 1, 24) * np.log(16)).astype(int)
    mols = [synth.molecule(int(k), 4100 + i) for i, k in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum([m.n for m in mols])]).astype(np.int64)
    return mols, off


def test_replays_against_batch_builds(acx, batch):
    import torch
    mols, off = batch
    xyz0 = np.concatenate([m.xyz for m in mols])
    rad = np.concatenate([m.radii for m in mols])
    X = torch.from_numpy(xyz0.copy()).cuda()
    R = torch.from_numpy(rad).cuda()
    print(f"[case] plan over {len(mols)} molecules, {len(rad)} balls", flush=True)
    plan = acx.Plan(X, R, off, 0.0)
    plan.launch()
    got = plan.result()
    assert plan.stopped() == 0
    ref = acx.ac_alpha_complex_batch(X, R, off, 0.0)
    _same(got, ref, "first replay")
    # molecule 3 against the oracle
    k = 3
    a, b = int(off[k]), int(off[k + 1])
    want = oracle.alpha_complex(mols[k].xyz, mols[k].radii, 0.0)

    class _Mol:
        def __init__(self, c):
            self.rows = [c.molecule_rows(d) for d in range(4)]
            self.c = c

        def simplices(self, d):
            return self.c.simplices(d)[self.rows[d][k]:self.rows[d][k + 1]] - a

        def sizes(self, d):
            return self.c.sizes(d)[self.rows[d][k]:self.rows[d][k + 1]]

    assert_same_complex(_Mol(got), want, "plan molecule 3")
    got.close()
    ref.close()
    # jittered frames written in place; eager work between the replays
    for f in range(3):
        fr = np.concatenate([synth.jittered(m, 0.1, 7000 + 31 * f + i).xyz for i, m in enumerate(mols)])
        X.copy_(torch.from_numpy(fr))
        junk = (X * 2.0).sum().item()  # eager kernels and a synchronisation between replays
        assert np.isfinite(junk)
        print(f"[case] plan replay, frame {f}", flush=True)
        plan.launch()
        got = plan.result()
        assert plan.stopped() == 0, plan.stopped()
        again_ref = acx.ac_alpha_complex_batch(X, R, off, 0.0)
        _same(got, again_ref, f"frame {f}")
        plan.launch()
        got2 = plan.result()
        _same(got, got2, f"frame {f} replayed twice")
        for c in (got, again_ref, got2):
            c.close()
    assert plan.ordinary_builds() == 0
    plan.close()


def test_inputs_beyond_the_recording_fall_back(acx, batch):
    import torch
    mols, off = batch
    xyz0 = np.concatenate([m.xyz for m in mols])
    rad = np.concatenate([m.radii for m in mols])
    X = torch.from_numpy(xyz0.copy()).cuda()
    R = torch.from_numpy(rad.copy()).cuda()
    plan = acx.Plan(X, R, off, 0.0, headroom=1.0)
    # a radius above the largest recorded one
    R[int(off[5]) + 3] = 1.95
    print("[case] plan replay with a larger radius", flush=True)
    plan.launch()
    got = plan.result()
    assert plan.stopped() & 1, plan.stopped()
    ref = acx.ac_alpha_complex_batch(X, R, off, 0.0)
    _same(got, ref, "larger radius")
    got.close()
    ref.close()
    # back to the recorded radii: the replay itself serves again
    R.copy_(torch.from_numpy(rad))
    plan.launch()
    got = plan.result()
    assert plan.stopped() == 0
    got.close()
    # one molecule spread out by 1.5: more grid cells than recorded
    a, b = int(off[7]), int(off[8])
    X[a:b] = X[a:b] * 1.5
    print("[case] plan replay with a spread molecule", flush=True)
    plan.launch()
    got = plan.result()
    assert plan.stopped() & 2, plan.stopped()
    ref = acx.ac_alpha_complex_batch(X, R, off, 0.0)
    _same(got, ref, "spread molecule")
    got.close()
    ref.close()
    # duplicate centres: the fallback reports them
    X.copy_(torch.from_numpy(xyz0))
    X[a + 1] = X[a]
    plan.launch()
    with pytest.raises(acx.AlphaCxError) as ei:
        plan.result()
    assert ei.value.status == 2
    assert plan.stopped() & 4
    assert plan.ordinary_builds() == 3
    plan.close()


def test_single_molecule_plan_alpha_and_morton(acx):
    import torch
    m = synth.molecule(12000, 4200)
    X = torch.from_numpy(m.xyz.copy()).cuda()
    R = torch.from_numpy(m.radii).cuda()
    for alpha, opts in ((1.0, {"cell_order": 1}), (0.0, {"cell_mA": 2500})):
        print(f"[case] single-molecule plan alpha={alpha} opts={opts}", flush=True)
        plan = acx.Plan(X, R, np.array([0, m.n]), alpha, options=opts)
        plan.launch()
        got = plan.result()
        assert plan.stopped() == 0
        ref = acx.ac_alpha_complex_batch(X, R, np.array([0, m.n]), alpha, options=opts)
        _same(got, ref, f"alpha {alpha}")
        dev = acx.ac_alpha_complex_device(X, R, alpha, options=opts)
        for d in range(4):
            assert np.array_equal(got.simplices(d), dev.simplices(d))
        for c in (got, ref, dev):
            c.close()
        plan.close()


def test_counted_fill_inputs_have_no_plan(acx):
    import torch
    m = synth.molecule(3000, 4300, sas=True)  # solvent-accessible rows outgrow the single-pass slots
    X = torch.from_numpy(m.xyz).cuda()
    R = torch.from_numpy(m.radii).cuda()
    with pytest.raises(acx.AlphaCxError) as ei:
        acx.Plan(X, R, np.array([0, m.n]), 0.0)
    assert ei.value.status == 6


def test_large_plan_with_two_streams(acx):
    """A recorded batch of more than 2^20 balls: its capture forks the emit
    of tetrahedra, triangles and vertices onto a second stream and joins it
    again; every replay must equal the ordinary batch build bit for bit."""
    import torch
    mols = [synth.molecule(20000, 4400 + i) for i in range(56)]
    off = np.concatenate([[0], np.cumsum([m.n for m in mols])]).astype(np.int64)
    assert off[-1] >= (1 << 20)
    X = torch.from_numpy(np.concatenate([m.xyz for m in mols])).cuda()
    R = torch.from_numpy(np.concatenate([m.radii for m in mols])).cuda()
    print(f"[case] plan over {len(mols)} molecules, {int(off[-1])} balls", flush=True)
    plan = acx.Plan(X, R, off, 0.0)
    ref = acx.ac_alpha_complex_batch(X, R, off, 0.0)
    for rep in range(2):
        plan.launch()
        got = plan.result()
        assert plan.stopped() == 0
        _same(got, ref, f"replay {rep}")
        got.close()
    ref.close()
    plan.close()
