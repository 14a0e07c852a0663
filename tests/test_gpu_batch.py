"""Batching, graphs and serving-style admission keep the arithmetic unchanged.

A replica gives the same chain alone, in a batch of uneven shapes, admitted
into a running batch at a later time, and under graph replay; retiring a
neighbour does not disturb it.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1411_5588_amd import islf  # noqa: E402

from _helpers import config1, oracle_trajectory  # noqa: E402


def batch_params():
    return [config1(replica=0),
            config1(Lx=20, Ly=64, Lz=64, beta=0.5, h1=0.25, hn=-0.25, replica=1),
            config1(Lx=3, Ly=5, Lz=14, ybc=O.PBC, replica=2),
            config1(Lx=40, Ly=32, Lz=40, beta=0.25, h1=0.75, hn=-0.75, replica=3)]


@pytest.mark.parametrize("fmt", [islf.INT8, islf.BITPACK])
@pytest.mark.parametrize("exec_mode", [islf.EXEC_BATCHED, islf.EXEC_PERSISTENT])
def test_graph_replay_equals_stream_launches(fmt, exec_mode):
    ps = batch_params()
    with islf.Context([islf.Replica(**p) for p in ps], spin_format=fmt, obs_capacity=64,
                      exec_mode=exec_mode) as ctx:
        ctx.capture(4)
        ctx.replay(5)
        ctx.sweep(3)
        ctx.replay(2)
        recs = [ctx.measure(i, 0, 31) for i in range(len(ps))]
        spins = [ctx.get_spins(i) for i in range(len(ps))]
    for i, p in enumerate(ps):
        _, o_rec, o_s = oracle_trajectory(p, 31)
        assert np.array_equal(recs[i], o_rec), i
        assert np.array_equal(spins[i], o_s), i


@pytest.mark.parametrize("groups,grid", [(1, 0), (2, 0), (3, 96), (4, 0)])
def test_concurrent_groups_graph_and_eager(groups, grid):
    # the batched form with the replicas dealt into concurrent groups, each
    # on its own stream (one graph per group); eager sweeps between replays
    # and a change of the grouping in mid-run keep every chain exact
    ps = batch_params()
    with islf.Context([islf.Replica(**p) for p in ps], spin_format=islf.BITPACK, obs_capacity=64) as ctx:
        ctx.set_groups(groups)
        ctx.set_grid(grid)
        assert ctx.get_groups() == groups
        ctx.capture(3)
        ctx.replay(2)
        ctx.sweep(4)
        ctx.replay(1)
        ctx.set_groups(5 - groups)
        with pytest.raises(islf.IslfError) as e:
            ctx.replay(1)
        assert e.value.status == islf.ESTATE
        ctx.sweep(2)
        ctx.capture(5)
        ctx.replay(2)
        recs = [ctx.measure(i, 0, 25) for i in range(len(ps))]
        spins = [ctx.get_spins(i) for i in range(len(ps))]
    for i, p in enumerate(ps):
        _, o_rec, o_s = oracle_trajectory(p, 25)
        assert np.array_equal(recs[i], o_rec), i
        assert np.array_equal(spins[i], o_s), i


def test_persistent_grid_is_co_resident():
    # the cooperative launch takes one workgroup per CU below the persistent
    # kernel's co-residency bound by default; a chosen grid replaces it
    import torch
    num_cu = torch.cuda.get_device_properties(0).multi_processor_count
    ps = batch_params()
    reps = [islf.Replica(**p) for p in ps]
    with islf.Context(reps, spin_format=islf.BITPACK, obs_capacity=16) as ctx:
        ctx.set_groups(1)
        resident = ctx.get_grid() // 2
    with islf.Context(reps, spin_format=islf.BITPACK, obs_capacity=16, exec_mode=islf.EXEC_PERSISTENT) as ctx:
        grid = ctx.get_grid()
        assert grid % num_cu == 0 and 0 < grid < resident + num_cu
        ctx.set_grid(100)
        assert ctx.get_grid() == 100
        ctx.set_grid(0)
        assert ctx.get_grid() == grid


def test_group_and_grid_settings():
    # automatic grouping takes min(3, live replicas); the default grid of a
    # grouped launch is 3/2 per resident slot split over the groups (the
    # single chain's default is two per slot); bad values are refused
    ps = batch_params()
    with islf.Context([islf.Replica(**p) for p in ps], spin_format=islf.BITPACK, obs_capacity=16) as ctx:
        assert ctx.get_groups() == 3
        ctx.set_groups(16)
        assert ctx.get_groups() == 4
        ctx.set_groups(1)
        chain = ctx.get_grid()
        resident = chain // 2
        for g in (2, 3, 4):
            ctx.set_groups(g)
            assert ctx.get_groups() == g
            assert ctx.get_grid() == max(64, (3 * resident + g) // (2 * g))
        ctx.set_grid(100)
        assert ctx.get_grid() == 100
        for bad_groups in (-1, 17):
            with pytest.raises(islf.IslfError) as e:
                ctx.set_groups(bad_groups)
            assert e.value.status == islf.EINVAL
        for bad_grid in (-1, (1 << 20) + 1):
            with pytest.raises(islf.IslfError) as e:
                ctx.set_grid(bad_grid)
            assert e.value.status == islf.EINVAL
        ctx.set_grid(0)
        ctx.set_groups(0)
        ctx.sweep(3)
        recs = [ctx.measure(i, 0, 3) for i in range(len(ps))]
    for i, p in enumerate(ps):
        _, o_rec, _ = oracle_trajectory(p, 3)
        assert np.array_equal(recs[i], o_rec), i


def test_alone_equals_in_mix_with_admission_and_retirement():
    ps = batch_params()
    target = ps[1]
    with islf.Context([islf.Replica(**ps[0]), islf.Replica(**ps[2])], obs_capacity=128) as ctx:
        ctx.sweep(10)
        slot = ctx.add(islf.Replica(**target))     # admitted while others are at sweep 10
        ctx.sweep(5)
        extra = ctx.add(islf.Replica(**ps[3]))
        ctx.sweep(7)
        ctx.retire(0)                              # a neighbour leaves
        ctx.sweep(8)
        got = ctx.measure(slot, 0, 20)
        got_s = ctx.get_spins(slot)
        t_extra = ctx.sweep_count(extra)
        other = ctx.measure(1, 0, 30)
    _, o_rec, o_s = oracle_trajectory(target, 20)
    assert np.array_equal(got, o_rec)
    assert np.array_equal(got_s, o_s)
    assert t_extra == 15
    _, o_rec2, _ = oracle_trajectory(ps[2], 30)
    assert np.array_equal(other, o_rec2)


def test_slot_reuse_after_retire():
    ps = batch_params()
    with islf.Context([islf.Replica(**ps[0]), islf.Replica(**ps[2])], obs_capacity=64) as ctx:
        ctx.sweep(4)
        ctx.retire(0)
        s = ctx.add(islf.Replica(**ps[1]))
        assert s == 0
        ctx.sweep(6)
        got = ctx.measure(0, 0, 6)
        with pytest.raises(islf.IslfError):
            ctx.measure(0, 0, 7)
    _, o_rec, _ = oracle_trajectory(ps[1], 6)
    assert np.array_equal(got, o_rec)


def test_graph_invalidated_by_membership_change():
    ps = batch_params()
    with islf.Context([islf.Replica(**ps[0])], obs_capacity=16) as ctx:
        ctx.capture(2)
        ctx.add(islf.Replica(**ps[2]))
        with pytest.raises(islf.IslfError) as e:
            ctx.replay(1)
        assert e.value.status == islf.ESTATE


def test_phase_timings_are_real_sweeps():
    ps = batch_params()
    with islf.Context([islf.Replica(**p) for p in ps], obs_capacity=32) as ctx:
        ms, cnt = ctx.phase_timings(3)
        ctx.sweep(2)
        recs = [ctx.measure(i, 0, 5) for i in range(len(ps))]
    assert list(cnt) == [3, 3, 1]
    assert (ms > 0).all()
    for i, p in enumerate(ps):
        _, o_rec, _ = oracle_trajectory(p, 5)
        assert np.array_equal(recs[i], o_rec)


@pytest.mark.parametrize("fmt", [islf.INT8, islf.BITPACK])
@pytest.mark.parametrize("barriers", [islf.BARRIER_TEAM, islf.BARRIER_GRID, islf.BARRIER_AUTO])
def test_persistent_barrier_forms(fmt, barriers):
    # team barriers (each replica's workgroups meet on their own) and grid
    # barriers give the same chains, eager and under graph replay; a grid
    # smaller than the replica count falls back to grid barriers; the
    # automatic choice takes teams for int8 spins or 8 and more replicas
    ps = batch_params()
    with islf.Context([islf.Replica(**p) for p in ps], spin_format=fmt, obs_capacity=64,
                      exec_mode=islf.EXEC_PERSISTENT) as ctx:
        auto = islf.BARRIER_TEAM if fmt == islf.INT8 or len(ps) >= 8 else islf.BARRIER_GRID
        assert ctx.get_barriers() == auto
        ctx.set_barriers(barriers)
        assert ctx.get_barriers() == (auto if barriers == islf.BARRIER_AUTO else barriers)
        ctx.sweep(3)
        ctx.capture(4)
        ctx.replay(2)
        ctx.set_grid(3)                     # fewer workgroups than replicas
        assert ctx.get_barriers() == islf.BARRIER_GRID
        ctx.sweep(2)
        ctx.set_grid(0)
        ctx.sweep(1)
        recs = [ctx.measure(i, 0, 14) for i in range(len(ps))]
        spins = [ctx.get_spins(i) for i in range(len(ps))]
    for i, p in enumerate(ps):
        _, o_rec, o_s = oracle_trajectory(p, 14)
        assert np.array_equal(recs[i], o_rec), i
        assert np.array_equal(spins[i], o_s), i
