"""GPU union volume / area and gradients through the C ABI against the oracle.

V and A must agree to 1e-11 relative (float64 on both sides, summed in other
orders); every gradient entry to 1e-9 of the largest entry of its array.
The oracle's formulas are pinned by slicing quadrature and finite differences
in test_measure_pins.py; here finite differences are also taken directly
against the GPU gradient on sampled balls of a jittered 100k-atom frame.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import measure

pytestmark = pytest.mark.gpu

REL_VA = 1e-11
REL_GRAD = 1e-9


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


def _gpu_all(acx, xyz, rad, gV=1.0, gA=0.0):
    import torch
    X, R = _dev(xyz), _dev(rad)
    c = acx.ac_alpha_complex_device(X, R, 0.0)
    V, A = acx.ac_union_measure(c, X, R)
    g = torch.tensor([gV, gA], dtype=torch.float64, device="cuda:0")
    dx, dr = acx.ac_union_measure_backward(c, X, R, g)
    return c, V, A, dx.cpu().numpy(), dr.cpu().numpy()


def _compare(acx, xyz, rad, label):
    print(f"[case] {label} n={len(rad)}", flush=True)
    want = oracle.alpha_complex(xyz, rad, 0.0)
    V0, A0, gVx, gVr, gAx, gAr = measure.union_measure(want.simplices, xyz, rad, with_grad=True)
    for gV, gA in ((1.0, 0.0), (0.0, 1.0), (0.7, -1.3)):
        c, V, A, dx, dr = _gpu_all(acx, xyz, rad, gV, gA)
        assert c.counts() == want.counts()
        assert abs(V - V0) <= REL_VA * abs(V0), (label, V, V0)
        assert abs(A - A0) <= REL_VA * abs(A0), (label, A, A0)
        wx = gV * gVx + gA * gAx
        wr = gV * gVr + gA * gAr
        sx = max(np.abs(wx).max(), 1e-300)
        sr = max(np.abs(wr).max(), 1e-300)
        assert np.abs(dx - wx).max() <= REL_GRAD * sx, (label, gV, gA, np.abs(dx - wx).max(), sx)
        assert np.abs(dr - wr).max() <= REL_GRAD * sr, (label, gV, gA, np.abs(dr - wr).max(), sr)


def test_few_balls(acx):
    cases = [
        ([[0, 0, 0]], [1.5]),
        ([[0, 0, 0], [2.0, 0.3, 0.1]], [1.5, 1.2]),
        ([[0, 0, 0], [2.0, 0.3, 0.1], [0.8, 1.6, 0.4]], [1.5, 1.2, 1.4]),
        ([[0, 0, 0], [2.0, 0.3, 0.1], [0.8, 1.6, 0.4], [0.9, 0.7, 1.5]], [1.5, 1.2, 1.4, 1.3]),
        ([[0, 0, 0], [2.6, 0, 0], [1.3, 2.0, 0], [1.3, 0.5, 0.35]], [1.6, 1.6, 1.6, 0.9]),
        ([[0, 0, 0], [5.0, 0, 0], [0, 6.0, 0]], [1.2, 1.9, 1.5]),
    ]
    for k, (xyz, rad) in enumerate(cases):
        _compare(acx, np.array(xyz, float), np.array(rad, float), f"few{k}")


def test_random_sets(acx):
    rng = np.random.RandomState(11)
    for t in range(10):
        n = int(rng.choice([6, 12, 30]))
        xyz = np.round(rng.uniform(-3.0, 3.0, (n, 3)), 3)
        rad = np.round(rng.uniform(1.0, 1.8, n), 3)
        _compare(acx, xyz, rad, f"rand{t}")


@pytest.mark.parametrize("sas", [False, True])
def test_molecule_4k(acx, sas):
    m = synth.molecule(4000, 31)
    if sas:
        m = m.with_sas(1400)
    _compare(acx, m.xyz, m.radii, f"mol4k sas={sas}")


def test_hidden_ball_gets_zero(acx):
    # a small ball inside a large one is hidden: in no simplex, zero gradient
    xyz = np.array([[0.0, 0, 0], [0.3, 0.1, 0.0], [2.5, 0.0, 0.0]])
    rad = np.array([2.0, 0.5, 1.4])
    _compare(acx, xyz, rad, "hidden")
    _, _, _, dx, dr = _gpu_all(acx, xyz, rad, 1.0, 1.0)
    assert np.all(dx[1] == 0) and dr[1] == 0


def test_repeat_calls_are_bitwise_equal(acx):
    import torch
    m = synth.molecule(3000, 5).with_sas(1400)
    X, R = _dev(m.xyz), _dev(m.radii)
    c = acx.ac_alpha_complex_device(X, R, 0.0)
    g = torch.tensor([1.0, 0.25], dtype=torch.float64, device="cuda:0")
    first = acx.ac_union_measure(c, X, R)
    dx1, dr1 = acx.ac_union_measure_backward(c, X, R, g)
    for _ in range(3):
        assert acx.ac_union_measure(c, X, R) == first
        dx, dr = acx.ac_union_measure_backward(c, X, R, g)
        assert torch.equal(dx, dx1) and torch.equal(dr, dr1)
    assert torch.equal(acx.ac_union_measure_device(c, X, R).cpu(), torch.tensor(first, dtype=torch.float64))


def test_fused_forward_backward(acx):
    """One pass gives the forward's V, A (to rounding) and the backward's
    gradient bit for bit."""
    import torch
    m = synth.molecule(3000, 8).with_sas(1400)
    X, R = _dev(m.xyz), _dev(m.radii)
    c = acx.ac_alpha_complex_device(X, R, 0.0)
    for gv, ga in ((1.0, 0.0), (0.3, -2.0)):
        g = torch.tensor([gv, ga], dtype=torch.float64, device="cuda:0")
        va, dx, dr = acx.ac_union_measure_fused(c, X, R, g)
        V, A = acx.ac_union_measure(c, X, R)
        dx1, dr1 = acx.ac_union_measure_backward(c, X, R, g)
        assert abs(va[0].item() - V) <= 1e-13 * abs(V) and abs(va[1].item() - A) <= 1e-13 * abs(A)
        assert torch.equal(dx, dx1) and torch.equal(dr, dr1)


def test_autograd_function(acx):
    import torch
    m = synth.molecule(2000, 6)
    X = _dev(m.xyz).requires_grad_(True)
    R = _dev(m.radii).requires_grad_(True)
    c = acx.ac_alpha_complex_device(X.detach(), R.detach(), 0.0)
    va = acx.UnionMeasure.apply(X, R, c)
    loss = 2.0 * va[0] - 0.5 * va[1]
    loss.backward()
    want = oracle.alpha_complex(m.xyz, m.radii, 0.0)
    V0, A0, gVx, gVr, gAx, gAr = measure.union_measure(want.simplices, m.xyz, m.radii, with_grad=True)
    wx, wr = 2.0 * gVx - 0.5 * gAx, 2.0 * gVr - 0.5 * gAr
    assert abs(va[0].item() - V0) <= REL_VA * V0
    assert np.abs(X.grad.cpu().numpy() - wx).max() <= REL_GRAD * np.abs(wx).max()
    assert np.abs(R.grad.cpu().numpy() - wr).max() <= REL_GRAD * np.abs(wr).max()


def test_errors(acx):
    m = synth.molecule(200, 2)
    X, R = _dev(m.xyz), _dev(m.radii)
    c = acx.ac_alpha_complex_device(X, R, 0.0)
    with pytest.raises(acx.AlphaCxError) as e:
        acx.ac_union_measure(c, X[:100], R[:100])
    assert e.value.status == 1


def _star_fd(star, xyz, rad, i, k, h):
    """Central difference of (V, A) over the given simplices (those that
    contain ball i: the only terms that move with it)."""
    out = []
    for sgn in (1.0, -1.0):
        x, r = xyz.copy(), rad.copy()
        if k < 3:
            x[i, k] += sgn * h
        else:
            r[i] += sgn * h
        out.append(measure.union_measure(star, x, r))
    return np.array([(p - q) / (2 * h) for p, q in zip(out[0], out[1])])


def test_100k_frame_finite_differences(acx):
    """One jittered frame of the 100k-atom molecule: GPU gradients of V and A
    against central differences at h = 1e-4 A on 1,000 sampled balls, to 1e-6
    relative. Plain central differences carry a truncation error of order
    (h / rho)^2, which near-degenerate triangles (rho ~ 0.1 A) lift to 1e-6;
    the differences at h and h/2 are therefore Richardson-extrapolated, and
    the rounding of the star's sums (24 eps sum|term| / h) is admitted."""
    base = synth.config_100k()
    f = synth.jittered(base, 0.1, 2000)
    xyz, rad = f.xyz, f.radii
    c, V, A, dxV, drV = _gpu_all(acx, xyz, rad, 1.0, 0.0)
    _, _, _, dxA, drA = _gpu_all(acx, xyz, rad, 0.0, 1.0)
    simp = [c.simplices(d).astype(np.int64) for d in range(4)]
    # simplices of each ball (its star), through one sort per dimension
    inc = []
    for s in simp:
        flat = s.ravel()
        order = np.argsort(flat, kind="stable")
        start = np.searchsorted(flat[order], np.arange(f.n + 1))
        inc.append((order // s.shape[1], start))
    medV = np.median(np.abs(np.concatenate([dxV.ravel(), drV])))
    medA = np.median(np.abs(np.concatenate([dxA.ravel(), drA])))
    atoms = np.random.RandomState(3000).choice(f.n, 1000, replace=False)
    eps = np.finfo(np.float64).eps
    h = 1e-4
    for i in atoms:
        star = [s[rows[start[i]:start[i + 1]]] for s, (rows, start) in zip(simp, inc)]
        sv = sa = 0.0
        for s in star:
            if len(s):
                vol, area = measure.intersection_terms(xyz[s], rad[s])[:2]
                sv += np.abs(vol).sum()
                sa += np.abs(area).sum()
        for k in range(4):
            fv, fa = (4 * _star_fd(star, xyz, rad, i, k, h / 2) - _star_fd(star, xyz, rad, i, k, h)) / 3
            gv = dxV[i, k] if k < 3 else drV[i]
            ga = dxA[i, k] if k < 3 else drA[i]
            assert abs(fv - gv) <= 1e-6 * max(abs(gv), 1e-3 * medV) + 24 * eps * sv / h, (i, k, fv, gv)
            assert abs(fa - ga) <= 1e-6 * max(abs(ga), 1e-3 * medA) + 24 * eps * sa / h, (i, k, fa, ga)


def test_graph_replay_of_forward_backward(acx):
    """With the complex held fixed (as in an optimisation loop), V, A and the
    backward allocate nothing and never synchronise after the first call, so
    they can be captured once in a HIP graph and replayed with new
    coordinates written into the same buffers; every replay must equal the
    eager calls bit for bit."""
    import torch
    m = synth.molecule(3000, 17)
    X = _dev(m.xyz)
    R = _dev(m.radii)
    c = acx.ac_alpha_complex_device(X, R, 0.0)
    g = torch.tensor([1.0, 0.5], dtype=torch.float64, device="cuda:0")
    out = torch.empty(2, dtype=torch.float64, device="cuda:0")
    dx = torch.empty_like(X)
    dr = torch.empty_like(R)
    lib = acx.library()
    s = torch.cuda.Stream()

    def step():
        st = torch.cuda.current_stream()
        h = acx.ctypes.c_void_p(st.cuda_stream)
        assert lib.ac_union_measure_device(c._h, X.data_ptr(), R.data_ptr(), m.n, out.data_ptr(), h) == 0
        assert lib.ac_union_measure_backward(c._h, X.data_ptr(), R.data_ptr(), m.n, g.data_ptr(), dx.data_ptr(),
                                             dr.data_ptr(), h) == 0

    with torch.cuda.stream(s):
        step()  # first call: sorts the incidences, allocates the work buffers
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            step()
    torch.cuda.synchronize()
    rng = np.random.RandomState(5)
    for rep in range(4):
        shift = rng.normal(0.0, 0.01, size=m.xyz.shape)
        X.copy_(_dev(m.xyz + shift))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = (out.clone(), dx.clone(), dr.clone())
        with torch.cuda.stream(s):
            step()
        torch.cuda.synchronize()
        assert torch.equal(got[0], out) and torch.equal(got[1], dx) and torch.equal(got[2], dr), rep
        V, A = acx.ac_union_measure(c, X, R)
        assert (V, A) == tuple(out.cpu().tolist())


def test_100k_frame_against_oracle(acx):
    """The differentiation workload's first frame in full (the 100k-atom
    molecule with Gaussian jitter 0.1 A, seed 2000): the GPU complex equals the
    oracle's simplex for simplex, and V, A and both gradients over all 100,000
    balls agree with the oracle's formulas evaluated on the oracle's complex."""
    import torch
    from parity import assert_same_complex
    f = synth.jittered(synth.config_100k(), 0.1, 2000)
    print("[case] 100k frame 0: oracle complex and measure", flush=True)
    want = oracle.alpha_complex(f.xyz, f.radii, 0.0)
    V0, A0, gVx, gVr, gAx, gAr = measure.union_measure(want.simplices, f.xyz, f.radii, with_grad=True)
    X, R = _dev(f.xyz), _dev(f.radii)
    c = acx.ac_alpha_complex_device(X, R, 0.0)
    assert_same_complex(c, want, "100k frame 0")
    V, A = acx.ac_union_measure(c, X, R)
    assert abs(V - V0) <= REL_VA * abs(V0), (V, V0)
    assert abs(A - A0) <= REL_VA * abs(A0), (A, A0)
    for (gV, gA), (wx, wr) in (((1.0, 0.0), (gVx, gVr)), ((0.0, 1.0), (gAx, gAr))):
        g = torch.tensor([gV, gA], dtype=torch.float64, device="cuda:0")
        dx, dr = acx.ac_union_measure_backward(c, X, R, g)
        dx, dr = dx.cpu().numpy(), dr.cpu().numpy()
        assert np.abs(dx - wx).max() <= REL_GRAD * np.abs(wx).max(), (gV, gA)
        assert np.abs(dr - wr).max() <= REL_GRAD * np.abs(wr).max(), (gV, gA)


def test_measure_needs_a_complex_built_at_alpha_zero(acx):
    """V and A come from K_0; a complex built at another alpha is refused
    (the union of grown balls is measured from the complex of the grown radii
    at alpha = 0)."""
    m = synth.molecule(300, 4)
    X, R = _dev(m.xyz), _dev(m.radii)
    for alpha in (1.0, -0.5):
        c = acx.ac_alpha_complex_device(X, R, alpha)
        with pytest.raises(acx.AlphaCxError) as e:
            acx.ac_union_measure(c, X, R)
        assert e.value.status == 1
    # the grown balls' own complex at alpha = 0 is accepted (it equals K_1 up
    # to the rounding of the grown radii to the milli-angstrom lattice)
    grown = np.sqrt(m.radii ** 2 + 1.0)
    c0 = acx.ac_alpha_complex_device(X, _dev(grown), 0.0)
    V, A = acx.ac_union_measure(c0, X, _dev(grown))
    assert V > 0 and A > 0
