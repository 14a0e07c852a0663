"""Energies, means and thermodynamic integration on the GPU vs the oracle.

The FP64 results are required to match the oracle's formulas bit for bit
(same operation order, no fused multiply-add) and at least to 1e-12 relative.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1411_5588_amd import islf  # noqa: E402

from _helpers import config1, oracle_trajectory, parallel_map  # noqa: E402


def close(a, b, rtol=1e-12):
    a, b = np.asarray(a), np.asarray(b)
    return np.all(np.abs(a - b) <= rtol * np.maximum(np.abs(b), 1e-300))


def test_energy_records_match_oracle():
    p = config1(H=0.07, J=0.9)
    n = 200
    with islf.Context([islf.Replica(**p)], obs_capacity=n) as ctx:
        ctx.sweep(n)
        e = ctx.energy(0, 0, n)
        rec = ctx.measure(0, 0, n)
    _, o_rec, _ = oracle_trajectory(p, n)
    assert np.array_equal(rec, o_rec)
    ref = np.array([O.energy(p["J"], p["H"], p["h1"], p["hn"], r) for r in o_rec])
    assert np.array_equal(e, ref)
    # the host-array boundary call (islf_energy) on the device records
    assert np.array_equal(islf.energy(islf.Replica(**p), rec), ref)


def test_means_and_ti_pipeline_match_oracle():
    """A small thermodynamic-integration ladder over h1 (hn = -h1), Eq. 9."""
    R = 9
    hs = np.linspace(0.0, 1.0, R)
    ps = [config1(Lx=6, Ly=12, Lz=12, h1=float(h), hn=float(-h), seed=100 + r, replica=r)
          for r, h in enumerate(hs)]
    n, t0 = 300, 50
    with islf.Context([islf.Replica(**p) for p in ps], obs_capacity=n) as ctx:
        ctx.sweep(n)
        means = ctx.means(t0, n - t0)
        m1 = torch.tensor(means[:, 3], dtype=torch.float64, device="cuda")
        mn = torch.tensor(means[:, 4], dtype=torch.float64, device="cuda")
        norm = 1.0 / (12 * 12)
        cum = islf.integrate_device(hs, m1, mn, -1.0, 1.0, norm).cpu().numpy()
        lit = islf.integrate_device(hs, m1, mn, -1.0, -1.0, norm).cpu().numpy()
    # the host-array boundary call on the same means
    host = islf.integrate(hs, means[:, 3], means[:, 4], -1.0, 1.0, norm)
    assert np.array_equal(host, cum)
    outs = parallel_map(lambda p: oracle_trajectory(p, n)[1], ps)
    for r, o_rec in enumerate(outs):
        om = [O.mean(o_rec, k, first=t0) for k in range(4)]
        assert np.array_equal(means[r, 1:], om), r
        # mean energy: the oracle's Eq. 1 evaluated at the mean observables
        assert means[r, 0] == O.energy(ps[r]["J"], ps[r]["H"], ps[r]["h1"], ps[r]["hn"], np.array(om))
    o_m1 = np.array([O.mean(o, 2, first=t0) for o in outs])
    o_mn = np.array([O.mean(o, 3, first=t0) for o in outs])
    ref = O.integrate(hs, o_m1, o_mn, -1.0, 1.0, norm)
    assert np.array_equal(cum, ref) and close(cum, ref)
    assert np.array_equal(lit, O.integrate(hs, o_m1, o_mn, -1.0, -1.0, norm))


def test_integrate_edge_cases():
    one = islf.integrate_device([0.5], [1.0], [2.0]).cpu().numpy()
    assert one.tolist() == [0.0]
    rng = np.random.default_rng(1)
    h = np.sort(rng.uniform(-1, 1, 513))
    m1, mn = rng.normal(size=513), rng.normal(size=513)
    got = islf.integrate_device(h, m1, mn, 0.3, -1.7, 0.01).cpu().numpy()
    assert np.array_equal(got, O.integrate(h, m1, mn, 0.3, -1.7, 0.01))
    assert np.array_equal(got, islf.integrate(h, m1, mn, 0.3, -1.7, 0.01))
    with pytest.raises(islf.IslfError):
        islf.integrate_device([], [], [])
