"""Exact (pathwise) invariants of the oracle's Markov chain.

- T -> infinity (beta = 0): every proposal is accepted, so one sweep maps s to
  -s, two sweeps are the identity and the bond sum never changes.
- T -> 0: a ground state with no zero-cost move is a fixed point.
- Spin + field reversal (Sec. II.A Eqs. 3-4): starting from -s0 with all fields
  negated and the same random stream, the chain is exactly -s(t).
- Within a phase the visiting order is irrelevant (no bond inside a phase).
- Resume: run(2k) == run(k) then a fresh lattice holding the state runs k more.
"""
import numpy as np
import pytest

from oracle import oracle as O


@pytest.mark.parametrize("ybc", [O.PBC, O.APBC, O.GAPBC])
def test_beta_zero_sweep_is_global_flip(ybc):
    L = O.Lattice(3, 4, 6, ybc, beta=0.0, h1=0.5, hn=-0.5, seed=7)
    s0 = L.s.copy()
    obs0 = L.observables()
    rec = L.run(1)
    assert np.array_equal(L.s, -s0)
    assert rec[0, 0] == obs0[0]
    assert np.array_equal(rec[0, 1:], -obs0[1:])
    L.run(1)
    assert np.array_equal(L.s, s0)


def test_ground_state_is_fixed_point_at_low_temperature():
    for ybc in (O.PBC,):
        L = O.Lattice(4, 6, 8, ybc, beta=50.0, h1=0.5, hn=-0.5, init=O.INIT_UP, seed=3)
        s0 = L.s.copy()
        rec = L.run(20)
        assert np.array_equal(L.s, s0)
        assert (rec == rec[0]).all()


@pytest.mark.parametrize("ybc", [O.PBC, O.APBC, O.GAPBC])
def test_spin_and_field_reversal_is_pathwise(ybc):
    kw = dict(J=1.0, beta=0.3, seed=14115588, replica=2)
    a = O.Lattice(4, 6, 10, ybc, H=0.05, h1=0.55, hn=-0.3, **kw)
    b = O.Lattice(4, 6, 10, ybc, H=-0.05, h1=-0.55, hn=0.3, spins=-a.s, **kw)
    ra = a.run(25)
    rb = b.run(25)
    assert np.array_equal(b.s, -a.s)
    assert np.array_equal(rb[:, 0], ra[:, 0])
    assert np.array_equal(rb[:, 1:], -ra[:, 1:])
    # the trajectory is not trivial
    assert len(np.unique(ra[:, 1])) > 5


@pytest.mark.parametrize("ybc", [O.PBC, O.GAPBC])
def test_visiting_order_within_phase_is_irrelevant(ybc):
    a = O.Lattice(3, 5, 8, ybc, beta=0.25, h1=0.4, hn=-0.4, seed=17)
    b = O.Lattice(3, 5, 8, ybc, beta=0.25, h1=0.4, hn=-0.4, seed=17)
    rng = np.random.default_rng(0)
    for _ in range(10):
        a.sweep()
        b.sweep(order=rng.permutation(b.N))
        assert np.array_equal(a.s, b.s)


def test_resume_is_bit_exact():
    kw = dict(beta=1.0 / 3.0, h1=0.5, hn=-0.5, seed=14115588, replica=0)
    a = O.Lattice(12, 24, 24, O.GAPBC, **kw)
    ra = a.run(10)
    b = O.Lattice(12, 24, 24, O.GAPBC, **kw)
    rb1 = b.run(5)
    c = O.Lattice(12, 24, 24, O.GAPBC, spins=b.s, **kw)
    c.t = b.t
    rb2 = c.run(5)
    assert np.array_equal(np.concatenate([rb1, rb2]), ra)
    assert np.array_equal(c.s, a.s)


def test_replicas_and_seeds_give_distinct_streams():
    a = O.Lattice(3, 4, 8, O.GAPBC, seed=1, replica=0)
    b = O.Lattice(3, 4, 8, O.GAPBC, seed=1, replica=1)
    c = O.Lattice(3, 4, 8, O.GAPBC, seed=2, replica=0)
    assert not np.array_equal(a.s, b.s) and not np.array_equal(a.s, c.s)
