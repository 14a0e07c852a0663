"""The persistent form's failure path and its grid bound.

A persistent launch whose grid barrier gives up leaves its sweeps half done.
The error word is raised here from the host (a test-only entry point of the
library, not in the public header) before the launch, so every block stops
at its first barrier and exits normally: no launch really fails.  The next
read must report EDEVICE, later calls on the cut-short replicas ESTATE, and
islf_set_spins must restart a replica so that its chain is exact again.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1411_5588_amd import islf  # noqa: E402

from _helpers import config1, oracle_trajectory  # noqa: E402


def raise_barrier_error(ctx):
    f = islf.lib().islf_testing_raise_barrier_error
    assert f(ctx._h) == islf.OK


@pytest.mark.parametrize("fmt", [islf.INT8, islf.BITPACK])
def test_failed_persistent_launch_marks_replicas_and_restarts(fmt):
    ps = [config1(replica=0), config1(Lx=6, Ly=10, Lz=16, beta=0.4, seed=77, replica=1)]
    with islf.Context([islf.Replica(**p) for p in ps], spin_format=fmt, obs_capacity=64,
                      exec_mode=islf.EXEC_PERSISTENT) as ctx:
        ctx.sweep(3)
        assert ctx.sweep_count(0) == 3
        raise_barrier_error(ctx)
        ctx.sweep(4)                      # every block stops at its first barrier
        with pytest.raises(islf.IslfError) as e:
            ctx.measure(0, 0, 3)
        assert e.value.status == islf.EDEVICE
        for call in (lambda: ctx.measure(0, 0, 3), lambda: ctx.get_spins(1), lambda: ctx.sweep(1),
                     lambda: ctx.recompute(0), lambda: ctx.sweep_count(1), lambda: ctx.means(0, 3),
                     lambda: ctx.capture(2)):
            with pytest.raises(islf.IslfError) as e:
                call()
            assert e.value.status == islf.ESTATE
        # restart both chains from chosen spins; they are exact from there on
        rng = np.random.default_rng(5)
        starts = [rng.choice(np.array([-1, 1], dtype=np.int8), size=islf.Replica(**p).N) for p in ps]
        for i, s in enumerate(starts):
            ctx.set_spins(i, s)
        ctx.sweep(6)
        recs = [ctx.measure(i, 0, 6) for i in range(2)]
        spins = [ctx.get_spins(i) for i in range(2)]
    for i, p in enumerate(ps):
        _, o_rec, o_s = oracle_trajectory(p, 6, spins=starts[i])
        assert np.array_equal(recs[i], o_rec), i
        assert np.array_equal(spins[i], o_s), i


def test_persistent_grid_bound():
    p = config1()
    with islf.Context([islf.Replica(**p)], spin_format=islf.BITPACK, obs_capacity=16,
                      exec_mode=islf.EXEC_PERSISTENT) as ctx:
        default = ctx.get_grid()
        assert default >= 256
        with pytest.raises(islf.IslfError) as e:
            ctx.set_grid(100000)
        assert e.value.status == islf.ERANGE
        assert ctx.get_grid() == default
        ctx.set_grid(300)
        assert ctx.get_grid() == 300
        ctx.sweep(5)
        rec = ctx.measure(0, 0, 5)
        s = ctx.get_spins(0)
        # a larger grid chosen for the batched form is refused once the
        # context turns persistent
        ctx.set_exec(islf.EXEC_BATCHED)
        ctx.set_grid(100000)
        ctx.set_exec(islf.EXEC_PERSISTENT)
        with pytest.raises(islf.IslfError) as e:
            ctx.sweep(1)
        assert e.value.status == islf.ERANGE
    _, o_rec, o_s = oracle_trajectory(p, 5)
    assert np.array_equal(rec, o_rec)
    assert np.array_equal(s, o_s)


def test_retire_returns_replica_memory():
    ps = [config1(replica=0), config1(Lx=20, Ly=64, Lz=64, replica=1), config1(Lx=4, Ly=8, Lz=8, replica=2)]
    with islf.Context([islf.Replica(**p) for p in ps], spin_format=islf.INT8, obs_capacity=32) as ctx:
        total0, reps0 = ctx.device_bytes()
        assert reps0 > 0 and total0 >= reps0
        ctx.sweep(2)
        ctx.retire(1)
        total1, reps1 = ctx.device_bytes()
        assert reps1 < reps0 and total1 < total0
        per = [islf.footprint_bytes(islf.Replica(**p), islf.INT8, 32) for p in ps]
        assert reps1 <= per[0] + per[2]
        slot = ctx.add(islf.Replica(**config1(Lx=3, Ly=6, Lz=6, replica=3)))
        assert slot == 1
        _, reps2 = ctx.device_bytes()
        assert reps2 < reps0
        ctx.sweep(3)
        assert ctx.sweep_count(1) == 3
