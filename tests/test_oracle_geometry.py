"""Pins the oracle's bond list, seam and checkerboard phase map.

Checks: neighbour lists are symmetric with matching signs; coordination
numbers (6 inside, 5 on a free surface, 4 for a one-layer film); the seam of
the generalized antiperiodic condition (Sec. II.A Eq. 11) is an involution
that reflects x; the four-phase map never puts two bonded sites in one phase,
while a two-colour checkerboard does whenever the seam joins equal colours.
Bond sums agree with the enumerator's direct evaluation of Eq. 1 on every
state of small lattices, and with the closed forms of the uniform states.
"""
import itertools

import numpy as np
import pytest

from oracle import enumerate_exact as X
from oracle import oracle as O

SHAPES = [(Lx, Ly, Lz) for Lx in (1, 2, 3, 4, 5) for Ly in (2, 3, 4, 5, 6) for Lz in (2, 4, 6)]


def coords(i, Ly, Lz):
    return i // (Ly * Lz), (i // Lz) % Ly, i % Lz


@pytest.mark.parametrize("ybc", [O.PBC, O.APBC, O.GAPBC])
def test_neighbour_lists_symmetric_and_phases_valid(ybc):
    for (Lx, Ly, Lz) in SHAPES:
        L = O.Lattice(Lx, Ly, Lz, ybc)
        for i in range(L.N):
            nb, sg = L.neighbours(i)
            x, y, z = coords(i, Ly, Lz)
            expect = 6 - (x == 0) - (x == Lx - 1)
            assert len(nb) == expect
            for j, e in zip(nb, sg):
                nbj, sgj = L.neighbours(j)
                # j sees i with the same sign, as many times as i sees j
                assert sorted(sgj[nbj == i].tolist()) == sorted(sg[nb == j].tolist())
                assert L.phase(j) != L.phase(i)
                assert e in (-1, 1)
                if e == -1:
                    assert ybc != O.PBC


def test_seam_reflects_x_and_flips_sign():
    Lx, Ly, Lz = 4, 3, 4
    L = O.Lattice(Lx, Ly, Lz, O.GAPBC)
    for x in range(Lx):
        for z in range(Lz):
            i = (x * Ly + (Ly - 1)) * Lz + z
            nb, sg = L.neighbours(i)
            seam = [(j, e) for j, e in zip(nb, sg) if e == -1]
            assert len(seam) == 1
            j = seam[0][0]
            assert coords(j, Ly, Lz) == (Lx - 1 - x, 0, z)
            # involution: from row 0 the seam leads back to the start
            nbj, sgj = L.neighbours(j)
            back = [int(k) for k, e in zip(nbj, sgj) if e == -1]
            assert back == [i]


def test_two_colour_checkerboard_fails_under_gapbc_iff_lx_plus_ly_even():
    for (Lx, Ly, Lz) in SHAPES:
        if Ly < 3:
            continue
        L = O.Lattice(Lx, Ly, Lz, O.GAPBC)
        clash = False
        for i in range(L.N):
            x, y, z = coords(i, Ly, Lz)
            for j in L.neighbours(i)[0]:
                xj, yj, zj = coords(j, Ly, Lz)
                if (x + y + z) % 2 == (xj + yj + zj) % 2:
                    clash = True
        assert clash == ((Lx + Ly) % 2 == 0)


def test_phase_sizes():
    Lx, Ly, Lz = 4, 6, 8
    L = O.Lattice(Lx, Ly, Lz, O.GAPBC)
    counts = np.bincount([L.phase(i) for i in range(L.N)], minlength=4)
    assert counts.tolist() == [Lx * (Ly - 1) * Lz // 2] * 2 + [Lx * Lz // 2] * 2


@pytest.mark.parametrize("ybc", [O.PBC, O.APBC, O.GAPBC])
def test_observables_match_enumerator_on_every_state(ybc):
    for (Lx, Ly, Lz) in [(2, 3, 2), (1, 4, 4), (3, 2, 2), (2, 2, 4)]:
        S = X.all_states(Lx, Ly, Lz)
        ref = X.observables(S, ybc)
        L = O.Lattice(Lx, Ly, Lz, ybc)
        flat = S.reshape(S.shape[0], -1)
        for k in range(flat.shape[0]):
            assert np.array_equal(L.observables(np.ascontiguousarray(flat[k])), ref[k])


@pytest.mark.parametrize("Lx,Ly,Lz", [(1, 2, 2), (3, 4, 6), (12, 24, 24), (5, 7, 10)])
def test_uniform_state_bond_counts(Lx, Ly, Lz):
    """All-up: every slot satisfied except the seam slots under (G)APBC, which
    cost one broken bond per seam slot (Lx*Lz of them)."""
    for ybc in (O.PBC, O.APBC, O.GAPBC):
        for init, sign in ((O.INIT_UP, 1), (O.INIT_DOWN, -1)):
            L = O.Lattice(Lx, Ly, Lz, ybc, init=init)
            B, M, M1, Mn = L.observables().tolist()
            full = (3 * Lx - 1) * Ly * Lz
            assert B == (full if ybc == O.PBC else full - 2 * Lx * Lz)
            assert M == sign * Lx * Ly * Lz
            assert M1 == sign * Ly * Lz and Mn == sign * Ly * Lz


def test_counter_range_check():
    assert O.Lattice(4, 4, 4).counter_fits()


def test_invalid_shapes_rejected():
    for bad in [(0, 4, 4), (2, 1, 4), (2, 4, 3), (2, 4, 0)]:
        with pytest.raises(ValueError):
            O.Lattice(*bad)
