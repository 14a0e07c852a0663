"""Host FP64 calls of the C ABI against the oracle (no GPU needed).

islf_energy (Sec. II.A Eq. 1) and islf_integrate (Eq. 9 / Eq. 22, and the
beta path of Eq. 19) take host arrays and touch no device, so they are
checked here, through ctypes, bit for bit against the oracle's functions on
the same inputs.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O


@pytest.fixture(scope="module")
def islf():
    from paper_1411_5588_amd import islf as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1411_5588_amd import build
        build.build()
    return m


def test_energy_of_host_records_matches_oracle(islf):
    rng = np.random.default_rng(11)
    for _ in range(20):
        J, H, h1, hn = rng.normal(size=4)
        rep = islf.Replica(4, 6, 8, J=J, H=H, h1=h1, hn=hn)
        rec = rng.integers(-10**9, 10**9, size=(257, 4), dtype=np.int64)
        got = islf.energy(rep, rec)
        ref = np.array([O.energy(J, H, h1, hn, r) for r in rec])
        assert np.array_equal(got, ref)


def test_energy_of_an_oracle_chain(islf):
    p = dict(Lx=4, Ly=6, Lz=8, ybc=O.GAPBC, J=1.0, beta=0.4, H=0.05, h1=0.5, hn=-0.3, seed=5, replica=2)
    L = O.Lattice(**p)
    rec = L.run(30)
    rep = islf.Replica(**p)
    assert np.array_equal(islf.energy(rep, rec), [L.energy(r) for r in rec])


def test_energy_edge_cases(islf):
    rep = islf.Replica(2, 2, 2)
    assert islf.energy(rep, np.zeros((0, 4), dtype=np.int64)).shape == (0,)
    with pytest.raises(islf.IslfError) as e:
        islf.energy(islf.Replica(2, 2, 2, J=float("inf")), np.zeros((1, 4), dtype=np.int64))
    assert e.value.status == islf.EINVAL


def test_integrate_host_arrays_matches_oracle(islf):
    rng = np.random.default_rng(2)
    for n in (1, 2, 3, 64, 513):
        h = np.sort(rng.uniform(-1, 1, n))
        m1, mn = rng.normal(size=n), rng.normal(size=n)
        for c1, cn, norm in ((-1.0, 1.0, 1.0 / 14400), (-1.0, -1.0, 0.5), (0.3, -1.7, 0.01)):
            got = islf.integrate(h, m1, mn, c1, cn, norm)
            assert np.array_equal(got, O.integrate(h, m1, mn, c1, cn, norm))
            assert got[0] == 0.0
    with pytest.raises(islf.IslfError) as e:
        islf.integrate([], [], [])
    assert e.value.status == islf.EINVAL
    with pytest.raises(ValueError):
        islf.integrate([0.0, 1.0], [1.0], [1.0])
