"""GPU (HIP) path vs the CPU oracle, bit for bit.

Spins and the per-sweep integer observables (B, M, M1, Mn) of the library
must equal the oracle's exactly (the Markov chain is a deterministic function
of its inputs), for both spin formats, all execution forms, every tile
variant, ragged shapes, the degenerate one-layer film and Ly = 2 / Lz = 2.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1411_5588_amd import islf  # noqa: E402

from _helpers import SEED, config1, oracle_trajectory, parallel_map, random_shape  # noqa: E402

FORMATS = [islf.INT8, islf.BITPACK]
EXECS = [islf.EXEC_PLAIN, islf.EXEC_BATCHED, islf.EXEC_PERSISTENT]


def rep(p):
    return islf.Replica(**p)


def gpu_trajectory(params, n, fmt=islf.INT8, exec_mode=islf.EXEC_BATCHED, spins=None, tiles=None, chunk=None):
    reps = [rep(p) for p in params]
    with islf.Context(reps, spin_format=fmt, obs_capacity=max(n, 1) + 8, exec_mode=exec_mode) as ctx:
        if spins is not None:
            for i, s in enumerate(spins):
                if s is not None:
                    ctx.set_spins(i, s)
        if tiles is not None:
            for i, t in enumerate(tiles):
                ctx.set_tile(i, t)
        s0 = [ctx.get_spins(i) for i in range(len(reps))]
        done = 0
        chunk = chunk or n
        while done < n:
            k = min(chunk, n - done)
            ctx.sweep(k)
            done += k
        recs = [ctx.measure(i, 0, n) if n else np.zeros((0, 4), np.int64) for i in range(len(reps))]
        s1 = [ctx.get_spins(i) for i in range(len(reps))]
        rc = [ctx.recompute(i) for i in range(len(reps))]
        t = [ctx.sweep_count(i) for i in range(len(reps))]
    return s0, recs, s1, rc, t


def assert_same(p, n, g_s0, g_rec, g_s1, g_rc, g_t, spins=None):
    o_s0, o_rec, o_s1 = oracle_trajectory(p, n, spins)
    assert np.array_equal(g_s0, o_s0), "initial spins differ"
    assert np.array_equal(g_rec, o_rec), "per-sweep records differ"
    assert np.array_equal(g_s1, o_s1), "final spins differ"
    if n:
        assert np.array_equal(g_rc, o_rec[-1]), "fused reductions != full recompute"
    assert g_t == n


@pytest.mark.parametrize("fmt", FORMATS)
def test_config1_full_run(fmt):
    """The 12x24x24 film at T = 3 for 1000 sweeps, every record."""
    p = config1()
    n = 1000
    s0, rec, s1, rc, t = gpu_trajectory([p], n, fmt=fmt, chunk=250)
    assert_same(p, n, s0[0], rec[0], s1[0], rc[0], t[0])


@pytest.mark.parametrize("exec_mode", EXECS)
@pytest.mark.parametrize("fmt", FORMATS)
def test_execution_forms(fmt, exec_mode):
    ps = [config1(replica=0),
          config1(Lx=5, Ly=7, Lz=18, ybc=O.PBC, beta=0.25, h1=0.3, hn=-0.7, replica=1),
          config1(Lx=1, Ly=2, Lz=2, ybc=O.GAPBC, beta=0.4, replica=2),
          config1(Lx=3, Ly=9, Lz=66, ybc=O.APBC, beta=0.5, H=0.05, seed=7, replica=3)]
    n = 30
    s0, rec, s1, rc, t = gpu_trajectory(ps, n, fmt=fmt, exec_mode=exec_mode, chunk=7)
    outs = parallel_map(lambda p: oracle_trajectory(p, n), ps)
    for i, (o_s0, o_rec, o_s1) in enumerate(outs):
        assert np.array_equal(s0[i], o_s0)
        assert np.array_equal(rec[i], o_rec), f"replica {i}"
        assert np.array_equal(s1[i], o_s1), f"replica {i}"
        assert np.array_equal(rc[i], o_rec[-1])
        assert t[i] == n


@pytest.mark.parametrize("fmt", FORMATS)
def test_random_shapes_all_boundaries(fmt):
    rng = np.random.default_rng(SEED)
    ps = []
    for k in range(24):
        Lx, Ly, Lz = random_shape(rng)
        ps.append(dict(Lx=Lx, Ly=Ly, Lz=Lz, ybc=k % 3, J=float(rng.choice([1.0, 0.7])),
                       beta=float(rng.choice([0.0, 0.1, 0.25, 1 / 3, 0.6, 2.0])),
                       H=float(rng.choice([0.0, 0.1])), h1=float(rng.uniform(-1, 1)),
                       hn=float(rng.uniform(-1, 1)), seed=int(rng.integers(0, 2**63)),
                       replica=k, init=int(k % 3)))
    n = 12
    s0, rec, s1, rc, t = gpu_trajectory(ps, n, fmt=fmt)
    outs = parallel_map(lambda p: oracle_trajectory(p, n), ps)
    for i, (o_s0, o_rec, o_s1) in enumerate(outs):
        assert np.array_equal(s0[i], o_s0), ps[i]
        assert np.array_equal(rec[i], o_rec), ps[i]
        assert np.array_equal(s1[i], o_s1), ps[i]


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("shape", [(7, 13, 90), (4, 90, 202)])
def test_every_tile_variant_gives_the_same_chain(fmt, shape):
    # (4, 90, 202): several linear tiles per plane with a ragged last one, a
    # ragged int8 row (202 = 8 x 25 + 2) and a partial last bit-packed word
    Lx, Ly, Lz = shape
    p = config1(Lx=Lx, Ly=Ly, Lz=Lz, replica=5)
    n = 6
    o_s0, o_rec, o_s1 = oracle_trajectory(p, n)
    for tile in range(islf.num_tiles(fmt)):
        s0, rec, s1, rc, t = gpu_trajectory([p], n, fmt=fmt, tiles=[tile])
        assert np.array_equal(rec[0], o_rec), f"tile {tile}"
        assert np.array_equal(s1[0], o_s1), f"tile {tile}"


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("Lx", [1, 2, 3])
def test_films_of_surface_planes(fmt, Lx):
    # Lx = 1: both surface fields on one plane (4 neighbours); Lx = 2: every
    # plane a surface; Lx = 3: one bulk plane between them.  Main rows
    # (Ly = 10), a ragged int8 row and a partial bit-packed word (Lz = 70),
    # and a bulk field H, so the surface terms of the observable changes are
    # all exercised.
    p = config1(Lx=Lx, Ly=10, Lz=70, ybc=O.GAPBC, beta=0.45, H=0.05, h1=0.6, hn=-0.4, replica=10 + Lx)
    n = 15
    s0, rec, s1, rc, t = gpu_trajectory([p], n, fmt=fmt)
    assert_same(p, n, s0[0], rec[0], s1[0], rc[0], t[0])


@pytest.mark.parametrize("fmt", FORMATS)
def test_infinite_beta_goes_only_downhill(fmt):
    # beta = inf (T = 0): every uphill move has threshold 0 and is never
    # taken, every level or downhill move is always taken; both formats take
    # their never-accepted path on every plane.  The chain equals the
    # oracle's, and since the sites of one phase are not neighbours, the
    # energy never rises from one record to the next.
    ps = [config1(Lx=Lx, Ly=10, Lz=70, ybc=ybc, beta=float("inf"), H=0.05, h1=0.6, hn=-0.4, replica=20 + Lx)
          for Lx, ybc in ((1, O.GAPBC), (2, O.APBC), (6, O.PBC), (5, O.GAPBC))]
    n = 10
    s0, rec, s1, rc, t = gpu_trajectory(ps, n, fmt=fmt)
    for i, p in enumerate(ps):
        assert_same(p, n, s0[i], rec[i], s1[i], rc[i], t[i])
        E = [O.energy(p["J"], p["H"], p["h1"], p["hn"], r) for r in rec[i]]
        assert all(E[k + 1] <= E[k] for k in range(n - 1)), (p, E)


@pytest.mark.parametrize("fmt", FORMATS)
def test_host_spins(fmt):
    p = config1(Lx=4, Ly=6, Lz=10, init=islf.INIT_HOST)
    rng = np.random.default_rng(3)
    s = rng.choice(np.array([-1, 1], dtype=np.int8), size=4 * 6 * 10)
    g_s0, g_rec, g_s1, g_rc, g_t = gpu_trajectory([p], 20, fmt=fmt, spins=[s])
    assert np.array_equal(g_s0[0], s)
    assert_same(p, 20, g_s0[0], g_rec[0], g_s1[0], g_rc[0], g_t[0], spins=s)


@pytest.mark.parametrize("fmt", FORMATS)
def test_beta_zero_is_global_flip_and_reversal_symmetry(fmt):
    p = config1(beta=0.0)
    s0, rec, s1, rc, t = gpu_trajectory([p], 2, fmt=fmt)
    ref = s0[0]
    assert rec[0][0, 0] == rec[0][1, 0]
    assert np.array_equal(s1[0], ref)
    q = config1(h1=-0.5, hn=0.5, init=islf.INIT_HOST)
    a = gpu_trajectory([config1()], 15, fmt=fmt)
    b = gpu_trajectory([q], 15, fmt=fmt, spins=[-a[0][0]])
    assert np.array_equal(b[2][0], -a[2][0])
    assert np.array_equal(b[1][0][:, 0], a[1][0][:, 0])
    assert np.array_equal(b[1][0][:, 1:], -a[1][0][:, 1:])


def test_int8_equals_bitpack_long_run():
    ps = [config1(Lx=20, Ly=64, Lz=64, beta=0.5, h1=0.25, hn=-0.25, replica=9)]
    a = gpu_trajectory(ps, 200, fmt=islf.INT8)
    b = gpu_trajectory(ps, 200, fmt=islf.BITPACK)
    assert np.array_equal(a[1][0], b[1][0])
    assert np.array_equal(a[2][0], b[2][0])


def test_ring_keeps_latest_records():
    p = config1(Lx=4, Ly=4, Lz=8)
    with islf.Context([rep(p)], obs_capacity=5) as ctx:
        ctx.sweep(12)
        got = ctx.measure(0, 7, 5)
        with pytest.raises(islf.IslfError) as e:
            ctx.measure(0, 6, 2)
        assert e.value.status == islf.ERANGE
        with pytest.raises(islf.IslfError):
            ctx.measure(0, 10, 3)
    _, o_rec, _ = oracle_trajectory(p, 12)
    assert np.array_equal(got, o_rec[7:12])


def test_error_paths():
    p = config1(Lx=4, Ly=4, Lz=8)
    with islf.Context([rep(p)]) as ctx:
        ctx.sweep(1)
        with pytest.raises(islf.IslfError) as e:
            ctx.set_spins(0, np.ones(4 * 4 * 8, np.int8))
        assert e.value.status == islf.ESTATE
        with pytest.raises(islf.IslfError) as e:
            ctx.get_spins(3)
        assert e.value.status == islf.ERANGE
        with pytest.raises(islf.IslfError) as e:
            ctx.set_exec(9)
        assert e.value.status == islf.EINVAL
    with pytest.raises(islf.IslfError) as e:
        islf.Context([islf.Replica(3, 3, 3)])
    assert e.value.status == islf.EINVAL
    with islf.Context([islf.Replica(2, 3, 4, init=islf.INIT_HOST)]) as ctx:
        bad = np.ones(24, np.int8)
        bad[5] = 0
        with pytest.raises(islf.IslfError) as e:
            ctx.set_spins(0, bad)
        assert e.value.status == islf.EINVAL


@pytest.mark.parametrize("fmt", FORMATS)
def test_empty_and_zero_counts(fmt):
    # zero sweeps and zero replays change nothing; zero-length reads are
    # refused; a context whose replicas are all retired sweeps nothing and
    # takes new replicas, which start at sweep 0
    ps = [config1(Lx=3, Ly=5, Lz=10, replica=0), config1(Lx=2, Ly=4, Lz=6, replica=1)]
    with islf.Context([rep(p) for p in ps], spin_format=fmt, obs_capacity=16) as ctx:
        ctx.sweep(0)
        ctx.sweep(2)
        ctx.capture(2)
        ctx.replay(0)
        ctx.sweep(0)
        assert [ctx.sweep_count(i) for i in range(2)] == [2, 2]
        recs = [ctx.measure(i, 0, 2) for i in range(2)]
        for i, p in enumerate(ps):
            _, o_rec, o_s = oracle_trajectory(p, 2)
            assert np.array_equal(recs[i], o_rec)
            assert np.array_equal(ctx.get_spins(i), o_s)
        for call in (lambda: ctx.measure(0, 0, 0), lambda: ctx.means(0, 0), lambda: ctx.capture(0)):
            with pytest.raises(islf.IslfError) as e:
                call()
            assert e.value.status == islf.EINVAL
        ctx.retire(0)
        ctx.retire(1)
        ctx.sweep(3)                           # nothing live: nothing to do
        slot = ctx.add(rep(ps[1]))
        ctx.sweep(2)
        assert ctx.sweep_count(slot) == 2
        _, o_rec, _ = oracle_trajectory(ps[1], 2)
        assert np.array_equal(ctx.measure(slot, 0, 2), o_rec)
