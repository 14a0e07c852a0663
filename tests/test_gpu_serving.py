"""Serving: continuous batching keeps every request's answer unchanged.

Requests of different sizes arrive over time, are admitted when slots and
memory free up, share batched launches with whatever else is resident, and
retire independently.  Each answer must equal the same chain run alone and
the oracle's.  Also: the autotuner changes only speed, never results.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1411_5588_amd import islf, serving  # noqa: E402

from _helpers import oracle_trajectory, parallel_map  # noqa: E402


def params_of(r: islf.Replica):
    return dict(Lx=r.Lx, Ly=r.Ly, Lz=r.Lz, ybc=r.ybc, J=r.J, beta=r.beta, H=r.H, h1=r.h1, hn=r.hn,
                seed=r.seed, replica=r.replica, init=r.init)


def small_workload(n=14, seed=7):
    return serving.poisson_workload(n, rate=400.0, seed=seed, min_sites=2e3, max_sites=6e4,
                                    sweep_range=(10, 60))


@pytest.mark.parametrize("fmt", [islf.INT8, islf.BITPACK])
def test_each_answer_is_the_same_alone_and_in_the_mix(fmt):
    reqs = small_workload()
    # room for the largest request plus about two mid-sized ones: admission binds
    fp = [islf.footprint_bytes(r.replica, fmt, 64) for r in reqs]
    budget = max(fp) + 2 * int(np.median(fp))
    srv = serving.Server(budget_bytes=budget, max_slots=4, spin_format=fmt, max_step=7, obs_capacity=64,
                         realtime=False)
    try:
        srv.run(reqs)
    finally:
        srv.close()
    assert all(r.finished >= r.admitted >= r.arrival for r in reqs)
    # alone: one context per request
    for r in reqs[:6]:
        with islf.Context([r.replica], spin_format=fmt, obs_capacity=64) as ctx:
            ctx.sweep(r.sweeps)
            alone = ctx.replica_means(0, 0, r.sweeps)
            last = ctx.measure(0, r.sweeps - 1, 1)[0]
        assert np.array_equal(alone, r.means)
        assert np.array_equal(last, r.last)
    outs = parallel_map(lambda r: oracle_trajectory(params_of(r.replica), r.sweeps)[1], reqs)
    for r, rec in zip(reqs, outs):
        assert np.array_equal(rec[-1], r.last), r.rid
        assert r.means[4] == O.mean(rec, 3)
    s = serving.summary(reqs, srv.wall_s, srv.busy_s)
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_served_workload_sizes_alone_and_in_the_mix():
    """Requests in the served size range (>= 1e5 sites, films of about
    1 : 3 : 3), admitted under a budget that binds; every answer equals the
    chain alone and the oracle's, and the replica memory the library holds
    never exceeds the budget."""
    reqs = serving.poisson_workload(6, rate=200.0, seed=21, min_sites=1e5, max_sites=4e5, sweep_range=(8, 24))
    assert min(r.replica.N for r in reqs) >= 1e5
    fmt = islf.BITPACK
    fp = [islf.footprint_bytes(r.replica, fmt, 32) for r in reqs]
    budget = max(fp) + int(np.median(fp))
    srv = serving.Server(budget_bytes=budget, max_slots=8, spin_format=fmt, max_step=5, obs_capacity=32,
                         realtime=False)
    held = []
    orig = srv._admit

    def spy(req, now):
        orig(req, now)
        held.append(srv.ctx.device_bytes()[1])
    srv._admit = spy
    try:
        srv.run(reqs)
    finally:
        srv.close()
    assert max(held) <= budget
    assert any(r.admitted > r.arrival for r in reqs)   # admission had to wait
    outs = parallel_map(lambda r: oracle_trajectory(params_of(r.replica), r.sweeps)[1], reqs)
    for r, rec in zip(reqs, outs):
        with islf.Context([r.replica], spin_format=fmt, obs_capacity=32) as ctx:
            ctx.sweep(r.sweeps)
            alone = ctx.replica_means(0, 0, r.sweeps)
        assert np.array_equal(alone, r.means), r.rid
        assert np.array_equal(rec[-1], r.last), r.rid
        assert r.means[3] == O.mean(rec, 2) and r.means[4] == O.mean(rec, 3)


def test_admission_respects_budget_and_slots():
    reqs = small_workload(10, seed=3)
    fp = [islf.footprint_bytes(r.replica, islf.BITPACK, 64) for r in reqs]
    srv = serving.Server(budget_bytes=max(fp) + 1, max_slots=2, spin_format=islf.BITPACK, max_step=5,
                         obs_capacity=64, realtime=False)
    peak = []
    orig = srv._admit

    def spy(req, now):
        orig(req, now)
        peak.append(srv.used)
        assert srv.used <= srv.budget
        # the replica blocks the library really holds stay within the budget
        assert srv.ctx.device_bytes()[1] <= srv.budget
    srv._admit = spy
    try:
        srv.run(reqs)
    finally:
        srv.close()
    assert max(peak) <= max(fp) + 1
    assert all(np.isfinite(r.finished) for r in reqs)


def test_autotune_changes_speed_not_results():
    ps = [dict(Lx=20, Ly=64, Lz=64, ybc=islf.GAPBC, beta=0.4, h1=0.25, hn=-0.25, seed=s, replica=s)
          for s in range(3)] + [dict(Lx=40, Ly=33, Lz=38, ybc=islf.APBC, beta=0.3, h1=0.5, hn=-0.5, seed=9,
                                     replica=9)]
    for fmt in (islf.INT8, islf.BITPACK):
        with islf.Context([islf.Replica(**p) for p in ps], spin_format=fmt, obs_capacity=64) as ctx:
            ctx.sweep(3)
            ctx.autotune(2)
            tiles = [ctx.get_tile(i) for i in range(len(ps))]
            taper, groups, grid = ctx.get_taper(), ctx.get_groups(), ctx.get_grid()
            ctx.sweep(5)
            recs = [ctx.measure(i, 0, 8) for i in range(len(ps))]
            t = [ctx.sweep_count(i) for i in range(len(ps))]
        assert t == [8] * len(ps)
        assert len(set(tiles[:3])) == 1
        assert taper in (0.0, 0.1, 0.2) and 1 <= groups <= 4 and grid >= 32
        outs = parallel_map(lambda p: oracle_trajectory(p, 8)[1], ps)
        for rec, o in zip(recs, outs):
            assert np.array_equal(rec, o)


def test_autotune_persistent_launch_keeps_results():
    ps = [dict(Lx=20, Ly=64, Lz=64, ybc=islf.GAPBC, beta=0.4, h1=0.25, hn=-0.25, seed=s, replica=s)
          for s in range(4)]
    with islf.Context([islf.Replica(**p) for p in ps], spin_format=islf.BITPACK, obs_capacity=64,
                      exec_mode=islf.EXEC_PERSISTENT) as ctx:
        default = ctx.get_grid()
        ctx.sweep(2)
        ctx.autotune(2)
        assert 0 < ctx.get_grid() <= default and ctx.get_taper() in (0.0, 0.2, 0.4, 0.6)
        ctx.capture(3)
        ctx.replay(2)
        recs = [ctx.measure(i, 0, 8) for i in range(len(ps))]
    outs = parallel_map(lambda p: oracle_trajectory(p, 8)[1], ps)
    for rec, o in zip(recs, outs):
        assert np.array_equal(rec, o)
