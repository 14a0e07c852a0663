"""Beta-path thermodynamic integration (Sec. II.C, Eqs. 19-20) on the GPU.

A ladder of replicas with periodic and antiperiodic y boundaries over beta
runs as one batch; its per-replica mean energies must equal the oracle's
exactly (they are ratios of the same integer sums), the device-side
trapezoid over beta must equal the oracle's to 1e-12, and so must the
free-energy difference the host analysis forms from them.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1411_5588_amd import analysis as A  # noqa: E402
from paper_1411_5588_amd import islf  # noqa: E402

from _helpers import SEED, oracle_lattice, parallel_map  # noqa: E402


@pytest.mark.parametrize("fmt", [islf.INT8, islf.BITPACK])
def test_beta_ladder_matches_oracle(fmt):
    betas = np.linspace(0.2, 0.5, 7)
    shape = dict(Lx=6, Ly=10, Lz=12)
    params = []
    for ybc in (O.APBC, O.PBC):
        for r, b in enumerate(betas):
            params.append(dict(shape, ybc=ybc, J=1.0, beta=float(b), H=0.0, h1=0.0, hn=0.0,
                               seed=SEED + 10 * ybc + r, replica=len(params), init=O.INIT_UP))
    n, t0 = 40, 10
    with islf.Context([islf.Replica(**p) for p in params], spin_format=fmt, obs_capacity=n + 4) as ctx:
        ctx.sweep(n)
        gm = np.array([ctx.replica_means(i, t0, n - t0) for i in range(len(params))])

    def run(p):
        L = oracle_lattice(p)
        rec = L.run(n)
        means = np.array([O.mean(rec, c, t0, n - t0) for c in range(4)])
        # mean energy: the oracle's Eq. 1 applied to the mean records
        return O.energy(p["J"], p["H"], p["h1"], p["hn"], means)

    om = np.array(parallel_map(run, params))
    assert np.array_equal(gm[:, 0], om)
    k = len(betas)
    ua, up = gm[:k, 0], gm[k:, 0]
    # device trapezoid of (U_APBC - U_PBC) over beta vs the oracle's
    dev = islf.integrate_device(betas, ua, up, c1=1.0, cn=-1.0, norm=1.0).cpu().numpy()
    assert np.array_equal(dev, islf.integrate(betas, ua, up, c1=1.0, cn=-1.0, norm=1.0))
    ref = O.integrate(betas, om[:k], om[k:], c1=1.0, cn=-1.0, norm=1.0)
    assert np.allclose(dev, ref, rtol=1e-12, atol=1e-12)
    dF = A.delta_free_energy(betas, ua, up)
    assert np.allclose(dF * betas, ref, rtol=1e-12, atol=1e-12)
