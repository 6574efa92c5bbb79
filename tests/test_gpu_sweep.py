"""GPU alpha sweep: one candidate search at the largest alpha, then every
alpha's complex. Each result must equal the single-alpha call at that alpha
bit for bit (simplices and Sizes), and the oracle at small sizes."""
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


def _check_sweep(acx, xyz, rad, alphas, label, options=None, oracle_check=False):
    print(f"[case] sweep {label}: n={len(rad)} alphas={list(alphas)}", flush=True)
    X, R = _dev(xyz), _dev(rad)
    outs = acx.ac_alpha_sweep_device(X, R, alphas, options=options)
    assert len(outs) == len(alphas)
    for a, c in zip(alphas, outs):
        single = acx.ac_alpha_complex_device(X, R, a, options=options)
        assert c.counts() == single.counts(), (label, a)
        for d in range(4):
            assert np.array_equal(c.simplices(d), single.simplices(d)), (label, a, d)
            assert np.array_equal(c.sizes(d), single.sizes(d)), (label, a, d)
            assert c.candidate_count(d) >= single.candidate_count(d)
        if oracle_check:
            assert_same_complex(c, oracle.alpha_complex(xyz, rad, a), f"{label} alpha={a}")
        single.close()
    for c in outs:
        c.close()


def test_small_against_oracle(acx):
    m = synth.molecule(1000, 1)
    _check_sweep(acx, m.xyz, m.radii, [1.5, -0.5, 0.0, 0.7, 0.7, 3.0], "1k", oracle_check=True)
    s = m.with_sas(1400)
    _check_sweep(acx, s.xyz, s.radii, [0.0, 2.0, 0.25], "1k sas", oracle_check=True)


def test_100k(acx):
    m = synth.config_100k()
    _check_sweep(acx, m.xyz, m.radii, [0.0, 0.25, 0.5, 1.0, 2.0], "100k")
    s = synth.config_100k(sas=True)
    _check_sweep(acx, s.xyz, s.radii, [2.0, 0.0, 1.0], "100k sas")


def test_options_and_edge_cases(acx):
    m = synth.molecule(400, 7)
    _check_sweep(acx, m.xyz, m.radii, [0.0, 1.0], "force_exact", options={"force_exact": 1})
    _check_sweep(acx, m.xyz, m.radii, [0.0, 1.0], "shortcut", options={"vertex_shortcut": 1})
    _check_sweep(acx, m.xyz, m.radii, [0.4], "one value")
    # below -r_max^2 no ball is a vertex: every result empty
    _check_sweep(acx, m.xyz, m.radii, [-5.0, -4.0, 0.0], "negative", oracle_check=True)
    _check_sweep(acx, m.xyz[:1], m.radii[:1], [0.0, 1.0], "one ball", oracle_check=True)
    _check_sweep(acx, m.xyz[:2], m.radii[:2], [-1.0, 0.0, 5.0], "two balls", oracle_check=True)
    # regular lattice: simulation of simplicity decides exact ties
    g = np.stack(np.meshgrid(*[np.arange(4) * 2.5] * 3, indexing="ij"), -1).reshape(-1, 3)
    _check_sweep(acx, g, np.full(len(g), 1.6), [0.0, 1.0, 3.0], "lattice", oracle_check=True)


def test_many_values_and_errors(acx):
    m = synth.molecule(300, 9)
    alphas = list(np.linspace(-1.0, 3.0, 40))
    _check_sweep(acx, m.xyz, m.radii, alphas, "40 values")
    X, R = _dev(m.xyz), _dev(m.radii)
    for bad in ([], [0.0, float("nan")], [0.0] * 1025):
        with pytest.raises(acx.AlphaCxError) as e:
            acx.ac_alpha_sweep_device(X, R, bad)
        assert e.value.status == 1
