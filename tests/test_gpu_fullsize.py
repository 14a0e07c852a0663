"""Paper-scale lattice (160 x 480 x 600, 46.08 M sites) on the GPU vs the oracle.

The oracle runs the full lattice for a few sweeps (seconds on the host); the
GPU runs the same sweeps in the execution forms the benchmark times, and every
spin and every per-sweep record must agree.  Longer runs are checked through
properties that hold at any size: the fused per-sweep reductions equal a full
recompute, int8 equals bit-packed, and the records stay within bounds.
"""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1411_5588_amd import islf  # noqa: E402

SHAPE = (160, 480, 600)


def params(T, replica):
    Lx, Ly, Lz = SHAPE
    return dict(Lx=Lx, Ly=Ly, Lz=Lz, ybc=islf.GAPBC, J=1.0, beta=1.0 / T, H=0.0, h1=0.55, hn=-0.55,
                seed=14115588 + replica, replica=replica, init=islf.INIT_RANDOM)


TEMPS = (2.0, 3.0, 4.0)


@pytest.fixture(scope="module")
def oracle_all():
    """Oracle: 2 sweeps of each replica of the benchmark batch (T = 2, 3, 4:
    below and above the roughening temperature), one thread per replica,
    running beside the GPU work."""
    out = {i: {} for i in range(len(TEMPS))}

    def work(i):
        p = params(TEMPS[i], i)
        L = O.Lattice(p["Lx"], p["Ly"], p["Lz"], O.GAPBC, J=1.0, beta=p["beta"], h1=0.55, hn=-0.55,
                      seed=p["seed"], replica=p["replica"])
        out[i]["s0"] = L.s.copy()
        out[i]["rec"] = L.run(2)
        out[i]["s2"] = L.s.copy()

    ths = [threading.Thread(target=work, args=(i,)) for i in range(len(TEMPS))]
    for th in ths:
        th.start()
    yield ths, out


@pytest.mark.parametrize("fmt,exec_mode,graph,barriers", [(islf.INT8, islf.EXEC_BATCHED, False, None),
                                                          (islf.INT8, islf.EXEC_BATCHED, True, None),
                                                          (islf.BITPACK, islf.EXEC_BATCHED, False, None),
                                                          (islf.BITPACK, islf.EXEC_BATCHED, True, None),
                                                          (islf.INT8, islf.EXEC_PERSISTENT, True, islf.BARRIER_TEAM),
                                                          (islf.BITPACK, islf.EXEC_PERSISTENT, True, islf.BARRIER_TEAM),
                                                          (islf.BITPACK, islf.EXEC_PERSISTENT, True, islf.BARRIER_GRID),
                                                          (islf.INT8, islf.EXEC_PLAIN, False, None),
                                                          (islf.BITPACK, islf.EXEC_PLAIN, True, None)])
def test_paper_scale_two_sweeps_bit_exact(oracle_all, fmt, exec_mode, graph, barriers):
    ths, out = oracle_all
    # the batch the benchmark runs: T = 2, 3, 4 side by side, in its default
    # launch configuration (concurrent replica groups); graph: captured and
    # replayed as the benchmark does.  Every replica is compared.
    reps = [islf.Replica(**params(T, i)) for i, T in enumerate(TEMPS)]
    with islf.Context(reps, spin_format=fmt, obs_capacity=16, exec_mode=exec_mode) as ctx:
        if barriers is not None:
            ctx.set_barriers(barriers)
        s0 = [ctx.get_spins(i) for i in range(3)]
        if graph:
            ctx.capture(2)
            ctx.replay(1)
        else:
            ctx.sweep(2)
        rec = [ctx.measure(i, 0, 2) for i in range(3)]
        s2 = [ctx.get_spins(i) for i in range(3)]
        rc = [ctx.recompute(i) for i in range(3)]
    for th in ths:
        th.join()
    for i in range(3):
        assert np.array_equal(s0[i], out[i]["s0"]), i
        assert np.array_equal(rec[i], out[i]["rec"]), i
        assert np.array_equal(s2[i], out[i]["s2"]), i
        assert np.array_equal(rc[i], out[i]["rec"][-1]), i


def test_paper_scale_long_run_properties():
    """200 sweeps: reductions == recompute, int8 == bit-packed == the persistent
    form (whose blocks exchange every plane through device-coherent accesses
    across its grid barriers), |M| <= N, B in range."""
    N = SHAPE[0] * SHAPE[1] * SHAPE[2]
    res = {}
    runs = ((islf.INT8, islf.EXEC_BATCHED), (islf.BITPACK, islf.EXEC_BATCHED), (islf.BITPACK, islf.EXEC_PERSISTENT),
            (islf.INT8, islf.EXEC_PERSISTENT))
    for fmt, exec_mode in runs:
        reps = [islf.Replica(**params(T, i)) for i, T in enumerate((2.0, 3.0, 4.0))]
        with islf.Context(reps, spin_format=fmt, obs_capacity=256, exec_mode=exec_mode) as ctx:
            ctx.capture(50)
            ctx.replay(4)
            recs = [ctx.measure(i, 0, 200) for i in range(3)]
            rcs = [ctx.recompute(i) for i in range(3)]
            spins = [ctx.get_spins(i) for i in range(3)]
        res[fmt, exec_mode] = (recs, rcs, spins)
        for r, rc in zip(recs, rcs):
            assert np.array_equal(r[-1], rc)
            assert (np.abs(r[:, 1]) <= N).all()
            assert (np.abs(r[:, 0]) <= 3 * N).all()
    ref = res[runs[0]]
    for run in runs[1:]:
        for i in range(3):
            assert np.array_equal(ref[0][i], res[run][0][i]), (run, i)
            assert np.array_equal(ref[2][i], res[run][2][i]), (run, i)
