"""The batched configurations at their full sizes, in the launch forms the
benchmark and the serving loop use.

* 64 replicas of 40 x 120 x 120 along the surface-field path (T = 3,
  h1 = r/63, hn = -h1), one persistent launch captured in a graph;
* 96 uneven replicas (Lx in {20, 40, 80}, Ly = Lz in {64, 128, 256},
  T in {2, 2.5, 3, 3.5, 4}, |h1| in {0.25, 0.5, 0.75}), int8, autotuned.

The oracle is too slow to follow every replica, so a sample of replicas is
compared bit for bit (spins and every record); for all replicas the last
record must equal a full recompute of the final spins, and the trapezoid over
the field path must equal the oracle's on the same means.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1411_5588_amd import islf  # noqa: E402

from _helpers import SEED, oracle_trajectory, parallel_map  # noqa: E402


def ti_batch():
    return [dict(Lx=40, Ly=120, Lz=120, ybc=O.GAPBC, J=1.0, beta=1.0 / 3.0, H=0.0, h1=r / 63.0, hn=-r / 63.0,
                 seed=SEED + r, replica=r, init=O.INIT_RANDOM) for r in range(64)]


def uneven_batch():
    out = []
    for r in range(96):
        c = r % 9
        Lx = (20, 40, 80)[c // 3]
        L = (64, 128, 256)[c % 3]
        T = (2.0, 2.5, 3.0, 3.5, 4.0)[(r // 9) % 5]
        h = (0.25, 0.5, 0.75)[(r // 45) % 3]
        out.append(dict(Lx=Lx, Ly=L, Lz=L, ybc=O.GAPBC, J=1.0, beta=1.0 / T, H=0.0, h1=h, hn=-h,
                        seed=SEED + 1000 + r, replica=r, init=O.INIT_RANDOM))
    return out


def check_sample(params, spins, recs, sample, n):
    outs = parallel_map(lambda i: oracle_trajectory(params[i], n), sample)
    for i, (s0, rec, s1) in zip(sample, outs):
        assert np.array_equal(recs[i], rec), i
        assert np.array_equal(spins[i], s1), i


@pytest.mark.parametrize("fmt", [islf.BITPACK, islf.INT8])
def test_ti_batch_persistent_graph(fmt):
    ps = ti_batch()
    n = 2
    with islf.Context([islf.Replica(**p) for p in ps], spin_format=fmt, obs_capacity=8,
                      exec_mode=islf.EXEC_PERSISTENT) as ctx:
        ctx.capture(n)
        ctx.replay(1)
        recs = [ctx.measure(i, 0, n) for i in range(64)]
        rc = [ctx.recompute(i) for i in range(64)]
        spins = {i: ctx.get_spins(i) for i in (0, 31, 63)}
        means = ctx.means(0, n)
        h = np.array([p["h1"] for p in ps])
        cum = islf.integrate_device(h, means[:, 3], means[:, 4], -1.0, 1.0, 1.0 / (120 * 120)).cpu().numpy()
    for i in range(64):
        assert np.array_equal(recs[i][-1], rc[i]), i
    check_sample(ps, spins, recs, [0, 31, 63], n)
    assert np.array_equal(cum, O.integrate(h, means[:, 3], means[:, 4], -1.0, 1.0, 1.0 / (120 * 120)))


def test_uneven_batch_autotuned():
    ps = uneven_batch()
    n = 2
    with islf.Context([islf.Replica(**p) for p in ps], spin_format=islf.INT8, obs_capacity=8) as ctx:
        ctx.autotune(2)
        tiles = [ctx.get_tile(i) for i in range(96)]
        ctx.sweep(n)
        recs = [ctx.measure(i, 0, n) for i in range(96)]
        rc = [ctx.recompute(i) for i in range(96)]
        sample = list(range(9))   # one replica of every size class
        spins = {i: ctx.get_spins(i) for i in sample}
    assert all(0 <= t < islf.num_tiles(islf.INT8) for t in tiles)
    for i in range(96):
        assert np.array_equal(recs[i][-1], rc[i]), i
    check_sample(ps, spins, recs, sample, n)
