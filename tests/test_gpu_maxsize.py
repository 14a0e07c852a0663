"""The largest lattice the library accepts, on the GPU.

1023 x 1024 x 4096 (4.29e9 sites) holds 4,290,772,992 bytes of int8 spins,
just below the 4 GiB that the kernels' 32-bit byte offsets address (one more
plane, 1024 x 1024 x 4096, is refused; a host test checks that).  The lattice
is far beyond what the oracle can run, so the test uses what the oracle can
compute site by site and properties that hold at any size:
- the random initial state at sampled sites (the last plane, row and column
  among them) against the oracle's Philox word under the counter map of the
  draws (the random-number reading: counter (g, 0, replica, 1), word
  (z >> 1) & 3, spin +1 when its top bit is 0);
- two sweeps in both spin formats, whose per-sweep records equal a full
  recompute and each other, and whose spins are equal site for site, before
  and after (the two formats share no layout, so an offset that wrapped in
  one of them would show as a difference); the persistent form's two sweeps
  (device-coherent accesses, one cooperative launch) equal the batched ones.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1411_5588_amd import islf  # noqa: E402

SHAPE = (1023, 1024, 4096)
SEED = 14115588 + 7


def params():
    Lx, Ly, Lz = SHAPE
    return dict(Lx=Lx, Ly=Ly, Lz=Lz, ybc=islf.GAPBC, J=1.0, beta=1.0 / 3.0, H=0.0, h1=0.55, hn=-0.55,
                seed=SEED, replica=5, init=islf.INIT_RANDOM)


def init_spin(x, y, z):
    """The oracle's initial spin of site (x, y, z): its Philox word in domain 1."""
    Lx, Ly, Lz = SHAPE
    C = (Lz + 7) // 8
    g = ((((x * Ly + y) * C + (z >> 3)) << 1) | (z & 1)) & 0xFFFFFFFF
    w = O.philox([g, 0, params()["replica"], 1], [SEED & 0xFFFFFFFF, SEED >> 32])[(z >> 1) & 3]
    return 1 if (int(w) >> 31) == 0 else -1


def same(a, b, chunk=1 << 28):
    """Site-for-site equality of two large int8 arrays, a chunk at a time."""
    assert a.shape == b.shape
    for i in range(0, a.size, chunk):
        if not np.array_equal(a[i:i + chunk], b[i:i + chunk]):
            bad = i + int(np.flatnonzero(a[i:i + chunk] != b[i:i + chunk])[0])
            return bad
    return -1


def run(fmt, exec_mode=islf.EXEC_BATCHED):
    with islf.Context([islf.Replica(**params())], spin_format=fmt, obs_capacity=4, exec_mode=exec_mode) as ctx:
        s0 = ctx.get_spins(0)
        ctx.sweep(2)
        rec = ctx.measure(0, 0, 2)
        recomputed = ctx.recompute(0)
        s2 = ctx.get_spins(0)
    torch.cuda.empty_cache()
    return s0, rec, recomputed, s2


def test_largest_lattice_both_formats():
    Lx, Ly, Lz = SHAPE
    N = Lx * Ly * Lz
    assert 16 * Lx * Ly * ((Lz + 15) // 16) < 1 << 32
    print(f"largest lattice {Lx}x{Ly}x{Lz}: int8", flush=True)
    s0_i8, rec_i8, rc_i8, s2_i8 = run(islf.INT8)
    assert s0_i8.size == N and s2_i8.size == N

    # sampled initial spins: corners, the last plane / row / column, and
    # random sites
    rng = np.random.default_rng(SEED)
    pts = [(0, 0, 0), (Lx - 1, Ly - 1, Lz - 1), (Lx - 1, 0, 0), (0, Ly - 1, Lz - 1), (Lx - 1, Ly - 1, 0),
           (Lx - 1, Ly - 2, Lz - 2), (Lx - 2, Ly - 1, 1)]
    pts += [tuple(int(v) for v in p) for p in zip(rng.integers(0, Lx, 600), rng.integers(0, Ly, 600),
                                                 rng.integers(0, Lz, 600))]
    pts += [(Lx - 1, int(y), int(z)) for y, z in zip(rng.integers(0, Ly, 200), rng.integers(0, Lz, 200))]
    for (x, y, z) in pts:
        assert s0_i8[(x * Ly + y) * Lz + z] == init_spin(x, y, z), (x, y, z)

    # fused per-sweep reductions equal the recompute of the final spins
    assert np.array_equal(rec_i8[1], rc_i8)
    # and the two sweeps' records differ (the chain moves)
    assert not np.array_equal(rec_i8[0], rec_i8[1])

    print(f"largest lattice {Lx}x{Ly}x{Lz}: bit-packed", flush=True)
    s0_bp, rec_bp, rc_bp, s2_bp = run(islf.BITPACK)
    assert same(s0_i8, s0_bp) == -1
    del s0_i8, s0_bp
    assert np.array_equal(rec_bp, rec_i8)
    assert np.array_equal(rec_bp[1], rc_bp)
    bad = same(s2_i8, s2_bp)
    assert bad == -1, f"site {bad} differs between int8 and bit-packed after two sweeps"
    del s2_i8

    print(f"largest lattice {Lx}x{Ly}x{Lz}: bit-packed, persistent", flush=True)
    _, rec_p, rc_p, s2_p = run(islf.BITPACK, islf.EXEC_PERSISTENT)
    assert np.array_equal(rec_p, rec_bp)
    assert np.array_equal(rc_p, rc_bp)
    bad = same(s2_p, s2_bp)
    assert bad == -1, f"site {bad} differs between the persistent and batched forms after two sweeps"
