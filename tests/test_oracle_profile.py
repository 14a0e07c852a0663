"""Pins of the oracle's layer profile (Sec. II.B, Eq. 17).

The profile is pinned by quantities the oracle computes elsewhere, from its
bond list: summed over all rows it is M, over the rows of layer x = 0 it is M1
and over those of x = Lx-1 it is Mn (Eq. 7).  Uniform states give Lz in every
row, and a brute-force sum over an explicit coordinate loop matches on small
random lattices.
"""
import numpy as np
import pytest

from oracle import oracle as O

from _helpers import SEED, random_shape


@pytest.mark.parametrize("ybc", [O.PBC, O.APBC, O.GAPBC])
def test_profile_sums_are_the_magnetisations(ybc):
    rng = np.random.default_rng(SEED + ybc)
    for k in range(12):
        Lx, Ly, Lz = random_shape(rng)
        L = O.Lattice(Lx, Ly, Lz, ybc, beta=0.4, h1=0.3, hn=-0.3, seed=SEED + k, replica=k)
        L.run(int(rng.integers(0, 4)))
        P = L.layer_profile()
        B, M, M1, Mn = L.observables()
        assert P.shape == (Lx, Ly)
        assert P.sum() == M
        assert P[0].sum() == M1
        assert P[-1].sum() == Mn
        assert np.all(np.abs(P) <= Lz) and np.all((P - Lz) % 2 == 0)


def test_uniform_states():
    for init, v in ((O.INIT_UP, 1), (O.INIT_DOWN, -1)):
        L = O.Lattice(3, 5, 8, O.GAPBC, init=init)
        assert np.array_equal(L.layer_profile(), np.full((3, 5), 8 * v))


def test_brute_force_rows():
    rng = np.random.default_rng(SEED)
    for k in range(6):
        Lx, Ly, Lz = random_shape(rng)
        s = rng.choice(np.array([-1, 1], dtype=np.int8), size=Lx * Ly * Lz)
        L = O.Lattice(Lx, Ly, Lz, O.GAPBC, spins=s)
        want = np.zeros((Lx, Ly), dtype=np.int64)
        for x in range(Lx):
            for y in range(Ly):
                for z in range(Lz):
                    want[x, y] += int(s[(x * Ly + y) * Lz + z])
        assert np.array_equal(L.layer_profile(), want)
