"""Pins the oracle's thermodynamic integration (Sec. II.A Eq. 9, Sec. II.C Eq. 22).

- The trapezoid rule is exact for a linear integrand.
- On a tiny lattice, integrating the exact field-conjugate integrand
  -<M1 - Mn> along hn = -h reproduces F(h) - F(0) = -(ln Z(h) - ln Z(0))/beta
  from exact enumeration (Eq. 7: m1 = -df1/dH1).
- Odd integrand -> even integral; first cumulative entry is zero.
"""
import numpy as np

from oracle import enumerate_exact as X
from oracle import oracle as O


def test_trapezoid_exact_for_linear_integrand():
    h = np.array([0.0, 0.1, 0.25, 0.3, 0.7, 1.0])
    a1, b1, an, bn = 0.3, -1.2, -0.1, 0.8
    m1 = a1 + b1 * h
    mn = an + bn * h
    c1, cn, norm = -1.0, 1.0, 0.5
    cum = O.integrate(h, m1, mn, c1, cn, norm)
    g0 = norm * (c1 * a1 + cn * an)
    g1 = norm * (c1 * b1 + cn * bn)
    assert cum[0] == 0.0
    assert np.allclose(cum, g0 * h + 0.5 * g1 * h ** 2, rtol=1e-13, atol=1e-15)


def test_integral_of_conjugate_magnetisation_is_free_energy_difference():
    shape, ybc, beta = (2, 3, 2), X.GAPBC, 1.0 / 3.0
    hs = np.linspace(0.0, 1.0, 201)
    m1, mn, lnZ = [], [], []
    for h in hs:
        ex = X.Exact(*shape, ybc, beta=beta, h1=h, hn=-h)
        m = ex.means
        m1.append(m["M1"])
        mn.append(m["Mn"])
        lnZ.append(ex.lnZ)
    cum = O.integrate(hs, m1, mn, -1.0, 1.0, 1.0)
    dF = -(np.array(lnZ) - lnZ[0]) / beta
    assert np.allclose(cum[1:], dF[1:], rtol=2e-5)
    # the literal sum m1 + mn vanishes identically here (Eq. 12 symmetry)
    lit = O.integrate(hs, m1, mn, -1.0, -1.0, 1.0)
    assert np.abs(lit).max() < 1e-9


def test_odd_integrand_gives_even_integral():
    h = np.linspace(-1.0, 1.0, 41)
    m1 = np.tanh(2 * h)
    mn = -np.tanh(2 * h)
    cum = O.integrate(h, m1, mn, -1.0, 1.0, 1.0)
    rel = cum - cum[20]
    assert np.allclose(rel, rel[::-1], atol=1e-12)


def test_means_and_energy_order():
    rec = np.array([[10, 2, 1, -1], [12, 4, 3, -3], [8, 0, 1, -1]], dtype=np.int64)
    assert O.mean(rec, 1) == 2.0
    assert O.mean(rec, 0, first=1) == 10.0
    e = O.energy(1.0, 0.1, 0.5, -0.5, rec[0])
    assert e == ((-1.0 * 10 - 0.1 * 2) - 0.5 * 1) - (-0.5) * (-1)
