"""GPU partitioned builds: slabs along x with a halo, owned rows merged. The
result must equal the single build bit for bit (simplices and Sizes), and the
oracle at small sizes; the halo bound rests on the locality pinned on the
oracle (test_locality_of_regions)."""
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


def _check(acx, xyz, rad, alpha, parts, label, oracle_check=False):
    """Both partitioned builds, device-resident and streamed from host memory,
    against the single build bit for bit (and the oracle)."""
    print(f"[case] partitioned {label}: n={len(rad)} alpha={alpha} parts={parts}", flush=True)
    X, R = _dev(xyz), _dev(rad)
    single = acx.ac_alpha_complex_device(X, R, alpha)
    want = oracle.alpha_complex(xyz, rad, alpha) if oracle_check else None
    for p in parts:
        for how, c in (("device", acx.ac_alpha_complex_partitioned(X, R, alpha, p)),
                       ("host", acx.ac_alpha_complex_partitioned_host(xyz, rad, alpha, p))):
            assert c.counts() == single.counts(), (label, how, p)
            for d in range(4):
                assert np.array_equal(c.simplices(d), single.simplices(d)), (label, how, p, d)
                assert np.array_equal(c.sizes(d), single.sizes(d)), (label, how, p, d)
            if want is not None:
                assert_same_complex(c, want, f"{label} {how} parts={p}")
            c.close()
    single.close()


def test_small(acx):
    m = synth.molecule(1000, 1)
    for alpha in (0.0, 1.0):
        _check(acx, m.xyz, m.radii, alpha, [1, 2, 3, 7], f"1k a={alpha}", oracle_check=True)
    s = m.with_sas(1400)
    _check(acx, s.xyz, s.radii, 0.0, [2, 5], "1k sas", oracle_check=True)


def test_100k(acx):
    m = synth.config_100k()
    _check(acx, m.xyz, m.radii, 0.0, [4, 16], "100k")
    s = synth.config_100k(sas=True)
    _check(acx, s.xyz, s.radii, 0.0, [3], "100k sas")


def test_edge_cases(acx):
    m = synth.molecule(300, 4)
    _check(acx, m.xyz[:5], m.radii[:5], 0.0, [8, 64], "more slabs than balls", oracle_check=True)
    _check(acx, m.xyz[:1], m.radii[:1], 0.0, [3], "one ball", oracle_check=True)
    _check(acx, m.xyz, m.radii, -5.0, [4], "empty", oracle_check=True)
    # every centre on one x plane: a single occupied slab (the oracle takes
    # coplanar inputs of up to 4096 balls)
    flat = m.xyz.copy()
    flat[:, 0] = 1.234
    _check(acx, flat, m.radii, 0.0, [4], "one plane", oracle_check=True)
    _check(acx, flat[:40], m.radii[:40], 0.0, [4], "one plane, 40 balls", oracle_check=True)
    # lattice with ties decided by simulation of simplicity
    g = np.stack(np.meshgrid(*[np.arange(4) * 2.5] * 3, indexing="ij"), -1).reshape(-1, 3)
    _check(acx, g, np.full(len(g), 1.6), 1.0, [2, 3], "lattice", oracle_check=True)


def test_errors(acx):
    m = synth.molecule(100, 3)
    X, R = _dev(m.xyz), _dev(m.radii)
    for parts in (0, 65):
        with pytest.raises(acx.AlphaCxError) as e:
            acx.ac_alpha_complex_partitioned(X, R, 0.0, parts)
        assert e.value.status == 1
    for parts in (0, 1025):
        with pytest.raises(acx.AlphaCxError) as e:
            acx.ac_alpha_complex_partitioned_host(m.xyz, m.radii, 0.0, parts)
        assert e.value.status == 1
    dup = np.concatenate([m.xyz, m.xyz[:1]])
    with pytest.raises(acx.AlphaCxError) as e:
        acx.ac_alpha_complex_partitioned(_dev(dup), _dev(np.concatenate([m.radii, m.radii[:1]])), 0.0, 3)
    assert e.value.status == 2
    with pytest.raises(acx.AlphaCxError) as e:
        acx.ac_alpha_complex_partitioned_host(dup, np.concatenate([m.radii, m.radii[:1]]), 0.0, 3)
    assert e.value.status == 2
    bad = m.radii.copy()
    bad[7] = -1.0  # found by the slab's own build on the device
    with pytest.raises(acx.AlphaCxError) as e:
        acx.ac_alpha_complex_partitioned_host(m.xyz, bad, 0.0, 2)
    assert e.value.status == 1


def test_host_streamed_many_slabs(acx):
    """The 100k-atom molecule from host memory in 64 and 200 slabs (most balls
    are halo in the thin ones), equal to the single build."""
    m = synth.config_100k()
    X, R = _dev(m.xyz), _dev(m.radii)
    single = acx.ac_alpha_complex_device(X, R, 0.0)
    for p in (64, 200):
        print(f"[case] host-streamed 100k, {p} slabs", flush=True)
        c = acx.ac_alpha_complex_partitioned_host(m.xyz, m.radii, 0.0, p)
        for d in range(4):
            assert np.array_equal(c.simplices(d), single.simplices(d)), (p, d)
            assert np.array_equal(c.sizes(d), single.sizes(d)), (p, d)
        assert acx.library().ac_simplices_device(c._h, 1) is None
