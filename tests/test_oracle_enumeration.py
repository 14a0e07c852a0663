"""Oracle chain averages vs exact enumeration of all 2^N states (N <= 18).

Long oracle runs on tiny lattices under PBC, APBC and the generalized
antiperiodic condition are compared with exact Boltzmann averages of E, M, M1
and Mn computed by the independent enumerator; errors come from a blocking
analysis and the test asks |z| < 4.5 for every quantity.  Also the exact
symmetry <M1> = -<Mn> of Sec. II.A Eq. 12 (H = 0, hn = -h1) on the enumerator.
"""
import numpy as np
import pytest

from oracle import enumerate_exact as X
from oracle import oracle as O

CASES = [
    # (shape, ybc, beta, H, h1, hn)
    ((2, 3, 2), X.GAPBC, 1.0 / 3.0, 0.0, 0.5, -0.5),
    ((2, 3, 2), X.PBC, 0.05, 0.0, 0.5, -0.5),
    ((2, 3, 2), X.APBC, 0.4, 0.1, 0.3, -0.6),
    ((3, 3, 2), X.GAPBC, 0.25, 0.0, 0.55, -0.55),
    ((2, 2, 4), X.APBC, 1.0 / 3.0, 0.0, 0.2, -0.2),
    ((1, 4, 4), X.GAPBC, 0.3, 0.05, 0.4, -0.4),
    ((4, 2, 2), X.PBC, 0.5, 0.0, 0.5, -0.5),
    # deep in the ordered phase the chain does not tunnel between the two
    # ordered states within the run, so only E and |M| are compared there
    ((2, 4, 2), X.GAPBC, 2.0, 0.0, 0.5, -0.5),
    ((2, 2, 2), X.PBC, 0.8, 0.0, 0.0, 0.0),
    ((2, 2, 2), X.APBC, 2.0, 0.0, 0.0, 0.0),
    ((3, 2, 2), X.GAPBC, 0.2, 0.0, 1.0, 0.25),
]


def blocked_z(series, exact, nblocks=50):
    n = len(series) // nblocks * nblocks
    blocks = series[:n].reshape(nblocks, -1).mean(axis=1)
    m = blocks.mean()
    se = blocks.std(ddof=1) / np.sqrt(nblocks)
    if se == 0:
        # a chain frozen in a ground state: T -> 0 agreement up to the
        # exponentially small excitation weight
        return 0.0 if abs(m - exact) < 1e-4 * max(1.0, abs(exact)) else np.inf
    return (m - exact) / se


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-ybc{c[1]}-b{c[2]:.3g}" for c in CASES])
def test_chain_matches_exact_enumeration(case):
    shape, ybc, beta, H, h1, hn = case
    ex = X.Exact(*shape, ybc, J=1.0, beta=beta, H=H, h1=h1, hn=hn)
    L = O.Lattice(*shape, ybc, J=1.0, beta=beta, H=H, h1=h1, hn=hn, seed=14115588, replica=1)
    L.run(2000)
    rec = L.run(150000).astype(np.float64)
    E = -1.0 * rec[:, 0] - H * rec[:, 1] - h1 * rec[:, 2] - hn * rec[:, 3]
    exact = ex.means
    exact["absM"] = ex.mean(np.abs(ex.obs[:, 1]).astype(np.float64))
    quantities = [("E", E), ("absM", np.abs(rec[:, 1]))]
    if beta < 1.0:
        quantities += [("M", rec[:, 1]), ("M1", rec[:, 2]), ("Mn", rec[:, 3])]
    for name, series in quantities:
        z = blocked_z(series, exact[name])
        assert abs(z) < 4.5, (name, series.mean(), exact[name], z)


def test_surface_profile_symmetry_is_exact():
    """H = 0 and hn = -h1: <M1> = -<Mn> exactly under every y boundary (Eq. 12)."""
    for ybc in (X.PBC, X.APBC, X.GAPBC):
        for beta in (0.1, 1.0 / 3.0, 1.0):
            ex = X.Exact(2, 3, 2, ybc, beta=beta, h1=0.55, hn=-0.55)
            m = ex.means
            assert abs(m["M1"] + m["Mn"]) < 1e-12 * max(1.0, abs(m["M1"]))
            assert abs(m["M1"]) > 1e-3
    # and it is not an identity: it fails without the antisymmetric fields
    ex = X.Exact(2, 3, 2, X.GAPBC, beta=1.0 / 3.0, h1=0.55, hn=-0.2)
    assert abs(ex.means["M1"] + ex.means["Mn"]) > 1e-3


def test_golden_enumeration_values():
    """Stored exact values (written by tests/golden/make_golden.py) still hold."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "enumeration_exact.json")
    with open(path) as f:
        data = json.load(f)
    for rec in data["cases"]:
        ex = X.Exact(*rec["shape"], rec["ybc"], J=rec["J"], beta=rec["beta"], H=rec["H"],
                     h1=rec["h1"], hn=rec["hn"])
        for k, v in rec["means"].items():
            assert abs(ex.means[k] - v) <= 1e-10 * max(1.0, abs(v))
        assert abs(ex.lnZ - rec["lnZ"]) <= 1e-10 * abs(rec["lnZ"])
