"""The build without allocation (ac_alpha_complex_noalloc) through the C ABI
against ac_alpha_complex_device, the entry point whose kernels it shares:
two calls in a row on one device (the second with a smaller input) give
exactly the rows and Sizes of the allocating call; the smaller one is also
checked against the oracle. Output buffers that are too small are reported
with the counts needed and left untouched.
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


def _buffers(caps, fill=-7):
    import torch
    simp = [torch.full((c, d + 1), fill, dtype=torch.int32, device="cuda:0") for d, c in enumerate(caps)]
    size = [torch.full((c,), float(fill), dtype=torch.float64, device="cuda:0") for c in caps]
    return simp, size


def _reference(acx, X, R, alpha, opts):
    c = acx.ac_alpha_complex_device(X, R, alpha, options=opts)
    out = [(c.simplices(d), c.sizes(d)) for d in range(4)]
    c.close()
    return out


def _check_same(counts, simp, size, ref, what):
    import torch
    torch.cuda.synchronize()
    for d in range(4):
        rows, sz = ref[d]
        assert counts[d] == len(rows), (what, d, counts[d], len(rows))
        got = simp[d][: counts[d]].cpu().numpy()
        assert np.array_equal(got, rows), (what, d)
        # the same kernels compute the Sizes: bit-identical
        assert np.array_equal(size[d][: counts[d]].cpu().numpy().view(np.int64), sz.view(np.int64)), (what, d)


@pytest.mark.parametrize("sas", [False, True])
def test_two_calls_against_allocating_entry(acx, sas):
    # solvent-accessible radii give about ten times the candidates per ball:
    # a smaller molecule keeps the build within the fixed scratch
    big = synth.molecule(6000 if sas else 20000, 71, sas=sas)
    small = synth.molecule(3000, 72, sas=sas)
    for alpha, opts in ((0.0, None), (1.0, {"cell_order": 1})):
        refs = []
        for m in (big, small):
            X, R = _dev(m.xyz), _dev(m.radii)
            refs.append((X, R, _reference(acx, X, R, alpha, opts)))
        # one set of output buffers, sized for the larger result plus slack
        caps = [max(len(refs[0][2][d][0]), len(refs[1][2][d][0])) + 5 for d in range(4)]
        simp, size = _buffers(caps)
        for k, (X, R, ref) in enumerate(refs):
            print(f"[case] noalloc call {k}: n={X.shape[0]} sas={sas} alpha={alpha} opts={opts}", flush=True)
            counts = acx.ac_alpha_complex_noalloc(X, R, alpha, simp, size, options=opts)
            _check_same(counts, simp, size, ref, f"call {k}")
        # the smaller input against the oracle as well
        got_rows = [simp[d][: counts[d]].cpu().numpy() for d in range(4)]
        got_size = [size[d][: counts[d]].cpu().numpy() for d in range(4)]
        want = oracle.alpha_complex(small.xyz, small.radii, alpha)

        class _Got:
            def simplices(self, d):
                return got_rows[d]

            def sizes(self, d):
                return got_size[d]

            def counts(self):
                return [len(r) for r in got_rows]

        assert_same_complex(_Got(), want, f"noalloc small sas={sas} alpha={alpha}")


def test_too_small_output_is_reported_and_untouched(acx):
    import torch
    m = synth.molecule(2000, 73)
    X, R = _dev(m.xyz), _dev(m.radii)
    ref = _reference(acx, X, R, 0.0, None)
    need = [len(ref[d][0]) for d in range(4)]
    caps = list(need)
    caps[2] -= 1  # one triangle short
    simp, size = _buffers(caps)
    print("[case] noalloc with a short triangle buffer", flush=True)
    with pytest.raises(acx.CapacityError) as ei:
        acx.ac_alpha_complex_noalloc(X, R, 0.0, simp, size)
    assert ei.value.counts == need
    torch.cuda.synchronize()
    for d in range(4):
        assert bool((simp[d] == -7).all()) and bool((size[d] == -7.0).all()), d
    # then a call with room for the result succeeds on the same scratch
    simp, size = _buffers(need)
    counts = acx.ac_alpha_complex_noalloc(X, R, 0.0, simp, size)
    _check_same(counts, simp, size, ref, "after a capacity error")


def test_argument_errors(acx):
    m = synth.molecule(500, 74)
    X, R = _dev(m.xyz), _dev(m.radii)
    simp, size = _buffers([600, 2000, 2000, 1000])
    with pytest.raises(acx.AlphaCxError) as ei:
        acx.ac_alpha_complex_noalloc(X, R, 0.0, simp, size, options={"profile": 1})
    assert ei.value.status == 1
    with pytest.raises(acx.AlphaCxError) as ei:
        acx.ac_alpha_complex_noalloc(X, R, float("nan"), simp, size)
    assert ei.value.status == 1


def test_input_beyond_the_scratch_is_refused(acx):
    """A build that needs more than the fixed scratch stops with a capacity
    error (nothing written to the outputs), and the next call works."""
    import torch
    big = synth.molecule(60000, 75, sas=True)
    X, R = _dev(big.xyz), _dev(big.radii)
    simp, size = _buffers([64, 64, 64, 64])
    print("[case] noalloc beyond the scratch: 60000 solvent-accessible balls", flush=True)
    with pytest.raises(acx.AlphaCxError) as ei:
        acx.ac_alpha_complex_noalloc(X, R, 0.0, simp, size)
    assert ei.value.status == 6 and "scratch" in ei.value.detail
    torch.cuda.synchronize()
    for d in range(4):
        assert bool((simp[d] == -7).all()), d
    m = synth.molecule(1000, 76)
    X, R = _dev(m.xyz), _dev(m.radii)
    ref = _reference(acx, X, R, 0.0, None)
    simp, size = _buffers([len(ref[d][0]) for d in range(4)])
    counts = acx.ac_alpha_complex_noalloc(X, R, 0.0, simp, size)
    _check_same(counts, simp, size, ref, "after a scratch overflow")
