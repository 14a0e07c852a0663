"""Writes enumeration_exact.json: exact Boltzmann averages of small thin-film
lattices from the oracle's enumerator (Sec. II.A Eq. 1 with the y boundaries of
Eq. 11).  Calls nothing outside oracle/.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import enumerate_exact as X  # noqa: E402

CASES = [
    ((2, 3, 2), X.GAPBC, 1.0, 1.0 / 3.0, 0.0, 0.5, -0.5),
    ((2, 3, 2), X.PBC, 1.0, 1.0 / 3.0, 0.0, 0.5, -0.5),
    ((2, 3, 2), X.APBC, 1.0, 1.0 / 3.0, 0.0, 0.5, -0.5),
    ((3, 3, 2), X.GAPBC, 1.0, 0.25, 0.0, 0.55, -0.55),
    ((1, 4, 4), X.GAPBC, 1.0, 0.3, 0.05, 0.4, -0.4),
    ((2, 4, 2), X.GAPBC, 1.0, 2.0, 0.0, 0.5, -0.5),
]


def main():
    out = {"source": "oracle/enumerate_exact.py (exact sum over all 2^N states)",
           "paper": "Hamiltonian Sec. II.A Eq. 1; y boundaries Sec. II.A Eq. 11",
           "cases": []}
    for shape, ybc, J, beta, H, h1, hn in CASES:
        ex = X.Exact(*shape, ybc, J=J, beta=beta, H=H, h1=h1, hn=hn)
        out["cases"].append({"shape": list(shape), "ybc": ybc, "J": J, "beta": beta, "H": H,
                             "h1": h1, "hn": hn, "means": ex.means, "lnZ": ex.lnZ})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "enumeration_exact.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
