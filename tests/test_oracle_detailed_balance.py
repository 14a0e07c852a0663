"""Detailed balance and stationarity of the oracle's per-phase updates.

For lattices of at most 10 spins the transition matrix of every phase is built
from the oracle's own acceptance thresholds (sites of one phase share no bond,
so a phase flips each of its sites independently with probability thr/2^32).
With Boltzmann weights from the enumerator's direct evaluation of Eq. 1:
  pi(s) P(s -> s') = pi(s') P(s' -> s)   up to the 2^-32 quantisation,
and pi is stationary under a whole sweep (phases 0, 1, 2, 3).  A long oracle
run on an 8-spin lattice also passes a chi-square test against pi.
"""
import numpy as np
import pytest

from oracle import enumerate_exact as X
from oracle import oracle as O

TWO32 = float(1 << 32)


def phase_matrix(L, flat, p):
    n_states, N = flat.shape
    sites = [i for i in range(N) if L.phase(i) == p]
    P = np.zeros((n_states, n_states))
    for k in range(n_states):
        s = np.ascontiguousarray(flat[k])
        acc = np.array([L.site_threshold(i, s) / TWO32 for i in sites])
        # every subset F of the phase's sites flips with prod(acc_F) prod(1-acc_rest)
        for mask in range(1 << len(sites)):
            prob = 1.0
            kk = k
            for b, i in enumerate(sites):
                if (mask >> b) & 1:
                    prob *= acc[b]
                    kk ^= (1 << i)
                else:
                    prob *= 1.0 - acc[b]
            P[k, kk] += prob
    return P, len(sites)


CASES = [((2, 3, 1 * 2), X.GAPBC, 0.4, 0.0, 0.5, -0.5),
         ((1, 2, 4), X.APBC, 1.0, 0.1, 0.3, -0.6),
         ((2, 2, 2), X.PBC, 0.25, 0.0, 0.55, -0.55),
         ((1, 5, 2), X.GAPBC, 0.7, 0.0, 1.0, 0.2)]


@pytest.mark.parametrize("case", CASES, ids=[str(c[0]) + f"-ybc{c[1]}" for c in CASES])
def test_detailed_balance_per_phase_and_stationarity(case):
    shape, ybc, beta, H, h1, hn = case
    ex = X.Exact(*shape, ybc, beta=beta, H=H, h1=h1, hn=hn)
    flat = ex.flat_states()
    pi = ex.p
    L = O.Lattice(*shape, ybc, beta=beta, H=H, h1=h1, hn=hn)
    sweep = np.eye(len(pi))
    for p in range(4):
        P, n_p = phase_matrix(L, flat, p)
        assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
        flux = pi[:, None] * P
        tol = n_p * 2.0 ** -31 * np.maximum(pi[:, None], pi[None, :]) + 1e-15
        assert (np.abs(flux - flux.T) <= tol).all()
        sweep = sweep @ P
        # and the phase matrix agrees with the oracle's actual phase step
        rng = np.random.default_rng(p)
        for k in rng.choice(len(pi), size=8, replace=False):
            s = np.ascontiguousarray(flat[k]).copy()
            L.phase_step(p, t=5, s=s)
            kk = int(sum(1 << i for i in range(len(s)) if s[i] == -1))
            assert P[k, kk] > 0
    assert np.allclose(pi @ sweep, pi, atol=1e-8)


def test_state_histogram_chi_square():
    shape, ybc, beta = (2, 2, 2), X.GAPBC, 0.3
    ex = X.Exact(*shape, ybc, beta=beta, h1=0.5, hn=-0.5)
    L = O.Lattice(*shape, ybc, beta=beta, h1=0.5, hn=-0.5, seed=2024)
    counts = np.zeros(len(ex.p))
    weights = 1 << np.arange(L.N)
    L.run(100)
    for _ in range(40000):
        L.run(3)           # thin the chain to weaken correlations
        counts[int(((L.s == -1) * weights).sum())] += 1
    expected = ex.p * counts.sum()
    keep = expected > 5
    chi2 = (((counts - expected) ** 2 / expected)[keep]).sum()
    dof = keep.sum() - 1
    assert chi2 < dof + 6 * np.sqrt(2 * dof), (chi2, dof)
