"""Pins the oracle's energy of a record (Sec. II.A Eq. 1).

The oracle evaluates E from the integer record (B, M, M1, Mn).  These tests
tie that value to things it does not compute itself:

- the energy written directly from the spins of every state of small
  lattices, with the field of each site taken per site (H on every site, h1
  added on x = 0, hn on x = Lx-1) and the bonds walked as neighbour pairs of
  the coordinate array, not through B, M, M1, Mn;
- the enumerator's Hamiltonian on every state;
- the oracle's local energy change, which drives its Metropolis dynamics:
  E(after a flip of site i) - E(before) must equal dE_i for every site of
  every state, so a dropped field term or a wrong sign shows up here;
- the closed forms of the uniform states (the broken-bond count of the
  antiperiodic seams) and the spin-plus-field reversal of Eqs. 3-4.
Parameters are distinct and nonzero so that a swapped pair (h1 <-> hn,
J <-> H) cannot cancel.
"""
import itertools

import numpy as np
import pytest

from oracle import enumerate_exact as X
from oracle import oracle as O

LATTICES = [(2, 3, 2), (3, 2, 2), (1, 3, 4), (2, 2, 4)]
PARAMS = dict(J=0.8125, H=0.3671875, h1=-0.703125, hn=0.2265625)


def direct_energy(s3, ybc, J, H, h1, hn):
    """Eq. 1 from the spins: bonds as (site, partner, sign) pairs and a
    per-site field."""
    Lx, Ly, Lz = s3.shape
    e = 0.0
    for x, y, z in itertools.product(range(Lx), range(Ly), range(Lz)):
        s = int(s3[x, y, z])
        partners = []
        if x + 1 < Lx:
            partners.append((s3[x + 1, y, z], 1))
        partners.append((s3[x, y, (z + 1) % Lz], 1))
        if y + 1 < Ly:
            partners.append((s3[x, y + 1, z], 1))
        elif ybc == O.PBC:
            partners.append((s3[x, 0, z], 1))
        elif ybc == O.APBC:
            partners.append((s3[x, 0, z], -1))
        else:  # Eq. 11: reflect x and change the sign across the seam
            partners.append((s3[Lx - 1 - x, 0, z], -1))
        for t, eps in partners:
            e -= J * eps * s * int(t)
        field = H + (h1 if x == 0 else 0.0) + (hn if x == Lx - 1 else 0.0)
        e -= field * s
    return e


def lattice(shape, ybc, **p):
    return O.Lattice(*shape, ybc, beta=0.3, **p)


@pytest.mark.parametrize("shape", LATTICES)
@pytest.mark.parametrize("ybc", [O.PBC, O.APBC, O.GAPBC])
def test_energy_of_every_state(shape, ybc):
    L = lattice(shape, ybc, **PARAMS)
    S = X.all_states(*shape)
    enum_E = X.energies(X.observables(S, ybc), **PARAMS)
    flat = S.reshape(S.shape[0], -1)
    # every state against the enumerator; every 7th also from the spins
    for k in range(S.shape[0]):
        e = L.energy(L.observables(flat[k]))
        assert e == pytest.approx(enum_E[k], rel=1e-13, abs=1e-12)
        if k % 7 == 0:
            assert e == pytest.approx(direct_energy(S[k], ybc, **PARAMS), rel=1e-13, abs=1e-12)


@pytest.mark.parametrize("shape", LATTICES[:3])
@pytest.mark.parametrize("ybc", [O.PBC, O.APBC, O.GAPBC])
def test_energy_differences_are_the_local_move_energies(shape, ybc):
    L = lattice(shape, ybc, **PARAMS)
    rng = np.random.default_rng(7)
    for _ in range(12):
        s = np.ascontiguousarray(rng.choice(np.array([-1, 1], dtype=np.int8), size=L.N))
        e0 = L.energy(L.observables(s))
        for i in range(L.N):
            t = s.copy()
            t[i] = -t[i]
            de = L.energy(L.observables(t)) - e0
            assert de == pytest.approx(L.delta_e(i, s), rel=1e-12, abs=1e-12), (i, s)


@pytest.mark.parametrize("shape", [(3, 4, 6), (1, 5, 4), (4, 3, 2)])
@pytest.mark.parametrize("ybc", [O.PBC, O.APBC, O.GAPBC])
def test_uniform_state_closed_forms(shape, ybc):
    Lx, Ly, Lz = shape
    N, A = Lx * Ly * Lz, Ly * Lz
    L = lattice(shape, ybc, **PARAMS)
    J, H, h1, hn = PARAMS["J"], PARAMS["H"], PARAMS["h1"], PARAMS["hn"]
    # bonds: x (Lx-1) Ly Lz + y Lx Ly Lz + z Lx Ly Lz; an antiperiodic seam
    # breaks its Lx Lz bonds in a uniform state
    B = (3 * Lx - 1) * Ly * Lz - (0 if ybc == O.PBC else 2 * Lx * Lz)
    for sign in (1, -1):
        s = np.full(N, sign, dtype=np.int8)
        obs = L.observables(s)
        assert obs.tolist() == [B, sign * N, sign * A, sign * A]
        expect = -J * B - sign * (H * N + h1 * A + hn * A)
        assert L.energy(obs) == pytest.approx(expect, rel=1e-14)


@pytest.mark.parametrize("ybc", [O.PBC, O.APBC, O.GAPBC])
def test_spin_and_field_reversal(ybc):
    """Eqs. 3-4: E(-s; -H, -h1, -hn) = E(s; H, h1, hn), exactly."""
    shape = (2, 3, 4)
    L = lattice(shape, ybc, **PARAMS)
    R = lattice(shape, ybc, J=PARAMS["J"], H=-PARAMS["H"], h1=-PARAMS["h1"], hn=-PARAMS["hn"])
    rng = np.random.default_rng(3)
    for _ in range(50):
        s = np.ascontiguousarray(rng.choice(np.array([-1, 1], dtype=np.int8), size=L.N))
        assert L.energy(L.observables(s)) == R.energy(R.observables(-s))


def test_energy_at_means_is_the_mean_energy():
    """The energy is linear in (B, M, M1, Mn): Eq. 1 at the mean record equals
    the mean of the records' energies (up to rounding)."""
    rng = np.random.default_rng(19)
    for _ in range(20):
        J, H, h1, hn = rng.normal(size=4)
        rec = rng.integers(-50000, 50000, size=(400, 4), dtype=np.int64)
        es = np.array([O.energy(J, H, h1, hn, r) for r in rec])
        m = rec.astype(np.float64).mean(axis=0)
        e_at = O.energy(J, H, h1, hn, m)
        assert e_at == pytest.approx(es.mean(), rel=1e-12, abs=1e-9)
        # an integer record given as floats gives the same value
        assert O.energy(J, H, h1, hn, rec[0].astype(np.float64)) == es[0]
