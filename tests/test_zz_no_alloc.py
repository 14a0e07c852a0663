"""The allocation-free means entry point (islf_means_noalloc) against
islf_means, through the C ABI.

Two calls in a row, the second on a smaller input: a context of twelve
replicas of uneven shapes with two retired slots, then a context of three.
Each result must equal islf_means bit for bit (NaN rows of retired slots
included) and the oracle's means on a sampled replica, and the call must not
request any device memory from the context's allocator.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import oracle as O  # noqa: E402
from paper_1411_5588_amd import islf  # noqa: E402

from _helpers import config1, oracle_trajectory  # noqa: E402


def means_noalloc_cabi(ctx, first, count):
    n = C.c_int32()
    assert islf.lib().islf_num_replicas(ctx._h, C.byref(n)) == islf.OK
    out = np.full((n.value, 5), 7.0, dtype=np.float64)
    st = islf.lib().islf_means_noalloc(ctx._h, first, count, out.ctypes.data_as(C.c_void_p))
    if st != islf.OK:
        raise islf.IslfError(st, islf.lib().islf_last_error().decode())
    return out


def check_call(ctx, first, count):
    ref = ctx.means(first, count)
    calls, bytes0 = ctx._alloc.calls, ctx.device_bytes()
    got = means_noalloc_cabi(ctx, first, count)
    assert ctx._alloc.calls == calls and ctx.device_bytes() == bytes0
    assert np.array_equal(got, ref, equal_nan=True)
    return got


def test_noalloc_means_two_calls_second_smaller():
    ps = [config1(Lx=2 + (r % 5), Ly=6 + 2 * (r % 4), Lz=4 + 6 * (r % 3), beta=0.2 + 0.05 * r,
                  h1=0.1 * r, hn=-0.1 * r, seed=300 + r, replica=r) for r in range(12)]
    with islf.Context([islf.Replica(**p) for p in ps], spin_format=islf.INT8, obs_capacity=64) as ctx:
        ctx.sweep(40)
        ctx.retire(2)
        ctx.retire(7)
        got = check_call(ctx, 5, 30)
    assert np.isnan(got[[2, 7]]).all() and np.isfinite(np.delete(got, [2, 7], axis=0)).all()
    _, rec, _ = oracle_trajectory(ps[9], 40)
    om = np.array([O.mean(rec, k, first=5, count=30) for k in range(4)])
    assert np.array_equal(got[9, 1:], om)
    assert got[9, 0] == O.energy(ps[9]["J"], ps[9]["H"], ps[9]["h1"], ps[9]["hn"], om)

    small = ps[:3]
    with islf.Context([islf.Replica(**p) for p in small], spin_format=islf.BITPACK, obs_capacity=16) as ctx:
        ctx.sweep(10)
        got = check_call(ctx, 0, 10)
        with pytest.raises(islf.IslfError) as e:
            means_noalloc_cabi(ctx, 5, 10)
        assert e.value.status == islf.ERANGE
        # tables out of date after a tile change: refused, not rebuilt
        ctx.set_tile(0, 0)
        with pytest.raises(islf.IslfError) as e:
            means_noalloc_cabi(ctx, 0, 10)
        assert e.value.status == islf.ESTATE
    for i, p in enumerate(small):
        _, rec, _ = oracle_trajectory(p, 10)
        assert np.array_equal(got[i, 1:], [O.mean(rec, k) for k in range(4)]), i
