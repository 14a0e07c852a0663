"""Pins the oracle's Metropolis thresholds and its local energy change.

thr = 2^32 if dE <= 0 else floor(2^32 exp(-beta dE)) is checked against the
same quantity evaluated in 60-digit arithmetic (mpmath); the local energy
change used by the oracle is checked against differences of the full
Hamiltonian (Sec. II.A Eq. 1) evaluated by the independent enumerator.
"""
import itertools
import math

import mpmath
import numpy as np
import pytest

from oracle import enumerate_exact as X
from oracle import oracle as O

TWO32 = 1 << 32


def exact_thr(beta, dE):
    if dE <= 0:
        return TWO32, 0.0
    with mpmath.workdps(60):
        v = mpmath.exp(-mpmath.mpf(beta) * mpmath.mpf(dE)) * TWO32
        fl = int(mpmath.floor(v))
        frac = float(v - fl)
    return fl, frac


@pytest.mark.parametrize("beta", [0.05, 0.2217, 0.25, 1.0 / 3.0, 0.4, 0.5, 1.0, 2.0, 10.0])
def test_thresholds_vs_mpmath(beta):
    J = 1.0
    fields = [0.0, 0.5, -0.5, 0.55, -0.55, 0.25, 0.75, 1.0 / 63.0, 0.1]
    checked = 0
    for h in fields:
        for n in range(-6, 7):
            for s in (-1, 1):
                dE = 2.0 * s * (J * float(n) + h)
                got = O.threshold_of_de(beta, dE)
                ref, frac = exact_thr(beta, dE)
                assert abs(got - ref) <= 1
                if 1e-6 < frac < 1 - 1e-6:
                    assert got == ref, (beta, dE)
                checked += 1
    assert checked == 9 * 13 * 2


def test_threshold_limits():
    for dE in (-12.0, -0.5, 0.0):
        assert O.threshold_of_de(0.3, dE) == TWO32
        assert O.threshold_of_de(math.inf, dE) == TWO32
    for dE in (0.5, 4.0, 12.0):
        assert O.threshold_of_de(0.0, dE) == TWO32      # T -> infinity: always accept
        assert O.threshold_of_de(math.inf, dE) == 0     # T -> 0: never go uphill
    assert O.threshold_of_de(1e9, 1e-9) < TWO32


@pytest.mark.parametrize("shape,ybc", [((2, 3, 2), X.GAPBC), ((1, 4, 2), X.APBC),
                                       ((3, 2, 2), X.PBC), ((2, 2, 4), X.GAPBC)])
def test_local_delta_e_matches_full_hamiltonian(shape, ybc):
    """oracle dE(i) == E(s with i flipped) - E(s), E from the enumerator's Eq. 1."""
    J, H, h1, hn = 1.3, 0.2, 0.5, -0.7
    Lx, Ly, Lz = shape
    ex = X.Exact(Lx, Ly, Lz, ybc, J=J, beta=0.3, H=H, h1=h1, hn=hn)
    flat = ex.flat_states()
    N = flat.shape[1]
    L = O.Lattice(Lx, Ly, Lz, ybc, J=J, beta=0.3, H=H, h1=h1, hn=hn)
    # state number k has +1 at site i iff bit i is 0, so flipping i toggles bit i
    rng = np.random.default_rng(1)
    for k in rng.choice(flat.shape[0], size=min(200, flat.shape[0]), replace=False):
        s = np.ascontiguousarray(flat[k])
        for i in range(N):
            dE = L.delta_e(i, s)
            ref = ex.E[k ^ (1 << i)] - ex.E[k]
            assert abs(dE - ref) < 1e-9


def test_site_threshold_is_threshold_of_local_de():
    L = O.Lattice(3, 4, 6, O.GAPBC, beta=0.37, h1=0.55, hn=-0.55, seed=3)
    for i in range(L.N):
        assert L.site_threshold(i) == O.threshold_of_de(0.37, L.delta_e(i))


def test_delta_e_sign_symmetry_is_bit_exact():
    """dE(s, h) == dE(-s, -h) bit for bit: round-to-nearest is sign-symmetric."""
    for (J, H, h1, hn) in itertools.product([1.0, 0.7], [0.0, 0.13], [0.55, 1.0 / 63.0], [-0.55, 0.3]):
        a = O.Lattice(1, 3, 4, O.GAPBC, J=J, H=H, h1=h1, hn=hn, seed=11)
        b = O.Lattice(1, 3, 4, O.GAPBC, J=J, H=-H, h1=-h1, hn=-hn, spins=-a.s)
        for i in range(a.N):
            assert a.delta_e(i) == b.delta_e(i)
