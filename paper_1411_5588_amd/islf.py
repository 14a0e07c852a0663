"""Python binding of libislf (include/islf.h): argument marshalling only.

Every step of the Monte Carlo path runs in the library's HIP kernels on the
GPU; this module converts Python values to the C ABI and back.  PyTorch
supplies device memory (its caching allocator backs the library's
allocations) and the HIP stream the work is issued on.

Model and update rule: thin-film Ising model of arXiv:1411.5588 (Sec. II.A
Eq. 1, y boundaries of Eq. 11), checkerboard Metropolis (Appendix), observables
of Eq. 7 / Eq. 19, thermodynamic integration of Eq. 9 / Eq. 22.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libislf.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ERANGE = range(6)
PBC, APBC, GAPBC = 0, 1, 2
INT8, BITPACK = 0, 1
INIT_RANDOM, INIT_UP, INIT_DOWN, INIT_HOST = 0, 1, 2, 3
EXEC_PLAIN, EXEC_BATCHED, EXEC_PERSISTENT = 0, 1, 2
BARRIER_GRID, BARRIER_TEAM, BARRIER_AUTO = 0, 1, 2

_STATUS = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ESTATE: "ESTATE", ERANGE: "ERANGE"}


class IslfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class ReplicaDesc(C.Structure):
    _fields_ = [("Lx", C.c_int32), ("Ly", C.c_int32), ("Lz", C.c_int32), ("ybc", C.c_int32),
                ("J", C.c_double), ("beta", C.c_double), ("H", C.c_double), ("h1", C.c_double),
                ("hn", C.c_double), ("seed", C.c_uint64), ("replica", C.c_uint32), ("init", C.c_int32)]


class Obs(C.Structure):
    _fields_ = [("B", C.c_int64), ("M", C.c_int64), ("M1", C.c_int64), ("Mn", C.c_int64)]


@dataclass
class Replica:
    """Parameters of one Markov chain (Sec. II.A Eq. 1; h1 on x = 0, hn on x = Lx-1)."""
    Lx: int
    Ly: int
    Lz: int
    ybc: int = GAPBC
    J: float = 1.0
    beta: float = 1.0 / 3.0
    H: float = 0.0
    h1: float = 0.0
    hn: float = 0.0
    seed: int = 0
    replica: int = 0
    init: int = INIT_RANDOM

    def to_c(self) -> ReplicaDesc:
        return ReplicaDesc(self.Lx, self.Ly, self.Lz, self.ybc, self.J, self.beta, self.H, self.h1,
                           self.hn, self.seed & (2**64 - 1), self.replica & (2**32 - 1), self.init)

    @property
    def N(self) -> int:
        return self.Lx * self.Ly * self.Lz


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None


def lib():
    """Loads libislf.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1411_5588_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, u32, u64, i64, dbl, sz = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_int64, C.c_double, C.c_size_t
        P = C.POINTER
        sig = {
            "islf_create": [P(ReplicaDesc), i32, i32, u32, vp, P(vp)],
            "islf_create_with_allocator": [P(ReplicaDesc), i32, i32, u32, vp, _ALLOC_FN, _FREE_FN, vp, P(vp)],
            "islf_destroy": [vp],
            "islf_num_replicas": [vp, P(i32)],
            "islf_get_desc": [vp, i32, P(ReplicaDesc)],
            "islf_set_spins": [vp, i32, vp, sz],
            "islf_get_spins": [vp, i32, vp, sz],
            "islf_set_exec": [vp, i32],
            "islf_sweep": [vp, u32],
            "islf_sweep_count": [vp, i32, P(u64)],
            "islf_measure": [vp, i32, u64, u32, vp],
            "islf_recompute": [vp, i32, P(Obs)],
            "islf_record_energy": [vp, i32, u64, u32, vp],
            "islf_energy": [P(ReplicaDesc), vp, sz, vp],
            "islf_means": [vp, u64, u32, vp],
            "islf_means_noalloc": [vp, u64, u32, vp],
            "islf_integrate": [vp, vp, vp, i32, dbl, dbl, dbl, vp],
            "islf_integrate_device": [vp, vp, vp, i32, dbl, dbl, dbl, vp, vp],
            "islf_footprint_bytes": [P(ReplicaDesc), i32, u32, P(u64)],
            "islf_plan_preview": [vp, i32, i32, i32, i32, vp, vp, i32, P(i32), vp, i32, P(i32)],
            "islf_batch_add": [vp, P(ReplicaDesc), P(i32)],
            "islf_batch_retire": [vp, i32],
            "islf_graph_capture": [vp, u32],
            "islf_run_graph": [vp, u32],
            "islf_num_tiles": [i32, P(i32)],
            "islf_get_tile": [vp, i32, P(i32)],
            "islf_set_tile": [vp, i32, i32],
            "islf_autotune": [vp, u32],
            "islf_set_grid": [vp, i32],
            "islf_layer_profile": [vp, i32, vp],
            "islf_layer_profile_add": [vp, i32, vp],
            "islf_get_grid": [vp, P(i32)],
            "islf_set_groups": [vp, i32],
            "islf_get_groups": [vp, P(i32)],
            "islf_phase_timings": [vp, u32, vp, vp],
            "islf_replica_means": [vp, i32, u64, u32, vp],
            "islf_device_bytes": [vp, P(u64), P(u64)],
            "islf_set_taper": [vp, dbl],
            "islf_set_barriers": [vp, i32],
            "islf_get_barriers": [vp, P(i32)],
            "islf_get_taper": [vp, P(dbl)],
            "islf_testing_raise_barrier_error": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.islf_last_error.restype = C.c_char_p
        L.islf_last_error.argtypes = []
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise IslfError(status, lib().islf_last_error().decode(errors="replace"))


def exported_symbols() -> list[str]:
    return [n for n in dir(lib()) if n.startswith("islf_")]


class _TorchAllocator:
    """Routes the library's device allocations through torch's caching allocator."""

    def __init__(self, torch, device, stream):
        self.torch = torch
        self.device = device
        self.stream = stream

        self.calls = 0   # allocation requests the library has made through this hook

        def _alloc(nbytes, user):
            self.calls += 1
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device,
                                                              stream=self.stream))
            except Exception:  # out of memory: the library reports ENOMEM
                return None

        def _free(ptr, user):
            if ptr:
                torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc = _ALLOC_FN(_alloc)
        self.free = _FREE_FN(_free)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the islf path runs only on an MI355X (gfx950) device")
    return torch


# Contexts still open when the interpreter exits are closed by an exit hook,
# registered after torch is imported so that it runs before torch's own exit
# hooks: their device memory goes back through torch's allocator while it
# still exists, and their graphs, streams and events are released before
# the HIP runtime shuts down.
_open_contexts: "weakref.WeakSet[Context]" = weakref.WeakSet()
_exit_hook = False


def _close_open_contexts():
    for ctx in list(_open_contexts):
        try:
            ctx.close()
        except Exception:
            pass


class Context:
    """A set of replicas on one GPU (islf_ctx)."""

    def __init__(self, replicas, spin_format=INT8, obs_capacity=1024, stream=None, exec_mode=EXEC_BATCHED,
                 torch_allocator=True):
        torch = _torch()
        self.torch = torch
        # a stream of its own (default priority), so that graph capture works
        self.stream = stream if stream is not None else torch.cuda.Stream()
        reps = list(replicas)
        arr = (ReplicaDesc * len(reps))(*[r.to_c() for r in reps])
        self.replicas = reps
        self.fmt = spin_format
        self.cap = obs_capacity
        h = C.c_void_p()
        if torch_allocator:
            self._alloc = _TorchAllocator(torch, torch.cuda.current_device(), self.stream)
            _check(lib().islf_create_with_allocator(arr, len(reps), spin_format, obs_capacity,
                                                    C.c_void_p(self.stream.cuda_stream), self._alloc.alloc,
                                                    self._alloc.free, None, C.byref(h)))
        else:
            self._alloc = None
            _check(lib().islf_create(arr, len(reps), spin_format, obs_capacity,
                                     C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        global _exit_hook
        if not _exit_hook:
            atexit.register(_close_open_contexts)
            _exit_hook = True
        _open_contexts.add(self)
        self.set_exec(exec_mode)

    # lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _check(lib().islf_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # spins ----------------------------------------------------------------
    def _N(self, rep):
        d = ReplicaDesc()
        _check(lib().islf_get_desc(self._h, rep, C.byref(d)))
        return d.Lx * d.Ly * d.Lz, (d.Lx, d.Ly, d.Lz)

    def get_spins(self, rep=0) -> np.ndarray:
        N, shape = self._N(rep)
        out = np.empty(N, dtype=np.int8)
        _check(lib().islf_get_spins(self._h, rep, out.ctypes.data_as(C.c_void_p), N))
        return out

    def set_spins(self, rep, spins):
        s = np.ascontiguousarray(np.asarray(spins, dtype=np.int8).reshape(-1))
        _check(lib().islf_set_spins(self._h, rep, s.ctypes.data_as(C.c_void_p), s.size))

    # sweeps ---------------------------------------------------------------
    def set_exec(self, mode: int):
        _check(lib().islf_set_exec(self._h, mode))

    def sweep(self, n: int = 1):
        _check(lib().islf_sweep(self._h, n))

    def sweep_count(self, rep=0) -> int:
        t = C.c_uint64()
        _check(lib().islf_sweep_count(self._h, rep, C.byref(t)))
        return t.value

    # measurement ----------------------------------------------------------
    def measure(self, rep=0, first=0, count=None) -> np.ndarray:
        if count is None:
            count = self.sweep_count(rep) - first
        out = np.zeros((count, 4), dtype=np.int64)
        _check(lib().islf_measure(self._h, rep, first, count, out.ctypes.data_as(C.c_void_p)))
        return out

    def recompute(self, rep=0) -> np.ndarray:
        o = Obs()
        _check(lib().islf_recompute(self._h, rep, C.byref(o)))
        return np.array([o.B, o.M, o.M1, o.Mn], dtype=np.int64)

    def energy(self, rep=0, first=0, count=None) -> np.ndarray:
        if count is None:
            count = self.sweep_count(rep) - first
        out = np.zeros(count, dtype=np.float64)
        _check(lib().islf_record_energy(self._h, rep, first, count, out.ctypes.data_as(C.c_void_p)))
        return out

    def means(self, first, count) -> np.ndarray:
        n = C.c_int32()
        _check(lib().islf_num_replicas(self._h, C.byref(n)))
        out = np.zeros((n.value, 5), dtype=np.float64)
        _check(lib().islf_means(self._h, first, count, out.ctypes.data_as(C.c_void_p)))
        return out

    def means_noalloc(self, first, count) -> np.ndarray:
        """means() through the allocation-free entry point (islf_means_noalloc)."""
        n = C.c_int32()
        _check(lib().islf_num_replicas(self._h, C.byref(n)))
        out = np.zeros((n.value, 5), dtype=np.float64)
        _check(lib().islf_means_noalloc(self._h, first, count, out.ctypes.data_as(C.c_void_p)))
        return out

    def replica_means(self, rep, first, count) -> np.ndarray:
        """mean (E, B, M, M1, Mn) of one replica's records first .. first+count-1."""
        out = np.zeros(5, dtype=np.float64)
        _check(lib().islf_replica_means(self._h, rep, first, count, out.ctypes.data_as(C.c_void_p)))
        return out

    # batching / graphs / tuning -------------------------------------------
    def add(self, replica: Replica) -> int:
        slot = C.c_int32()
        d = replica.to_c()
        _check(lib().islf_batch_add(self._h, C.byref(d), C.byref(slot)))
        return slot.value

    def retire(self, slot: int):
        _check(lib().islf_batch_retire(self._h, slot))

    def capture(self, k_sweeps: int):
        _check(lib().islf_graph_capture(self._h, k_sweeps))

    def replay(self, n: int = 1):
        _check(lib().islf_run_graph(self._h, n))

    def get_tile(self, rep=0) -> int:
        t = C.c_int32()
        _check(lib().islf_get_tile(self._h, rep, C.byref(t)))
        return t.value

    def set_tile(self, rep, tile):
        _check(lib().islf_set_tile(self._h, rep, tile))

    def autotune(self, sweeps=4):
        _check(lib().islf_autotune(self._h, sweeps))

    def _enqueue_on_ctx(self, fn):
        # caller tensors come from torch's current stream: the context's stream
        # waits for it before the kernel, and later work on the current stream
        # waits for the kernel
        cur = self.torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        fn()
        cur.wait_stream(self.stream)

    def layer_profile(self, rep: int, out=None):
        """Row sums over z of replica rep's current spins (Eq. 17 times Lz): a
        (Lx, Ly) int32 device tensor, ordered before later work on torch's
        current stream."""
        _, (Lx, Ly, _) = self._N(rep)
        if out is None:
            out = self.torch.empty((Lx, Ly), dtype=self.torch.int32, device="cuda")
        self._enqueue_on_ctx(lambda: _check(lib().islf_layer_profile(self._h, rep, C.c_void_p(out.data_ptr()))))
        return out

    def layer_profile_add(self, rep: int, acc):
        """Adds replica rep's row sums to the (Lx, Ly) int64 device tensor acc."""
        self._enqueue_on_ctx(lambda: _check(lib().islf_layer_profile_add(self._h, rep,
                                                                       C.c_void_p(acc.data_ptr()))))
        return acc

    def set_grid(self, workgroups: int):
        """Workgroups per A / B launch (0 = two per resident slot)."""
        _check(lib().islf_set_grid(self._h, workgroups))

    def set_groups(self, groups: int):
        """Concurrent replica groups of the batched form (0 = min(3, live replicas))."""
        _check(lib().islf_set_groups(self._h, groups))

    def get_groups(self) -> int:
        n = C.c_int32()
        _check(lib().islf_get_groups(self._h, C.byref(n)))
        return n.value

    def device_bytes(self):
        """(total, replica blocks): device bytes the context holds now."""
        t, r = C.c_uint64(), C.c_uint64()
        _check(lib().islf_device_bytes(self._h, C.byref(t), C.byref(r)))
        return t.value, r.value

    def set_barriers(self, mode: int):
        """Barriers of the persistent form: BARRIER_TEAM (per replica), BARRIER_GRID or BARRIER_AUTO."""
        _check(lib().islf_set_barriers(self._h, mode))

    def get_barriers(self) -> int:
        m = C.c_int32()
        _check(lib().islf_get_barriers(self._h, C.byref(m)))
        return m.value

    def set_taper(self, taper: float):
        """Share taper of the batched and persistent plans (< 0: built-in)."""
        _check(lib().islf_set_taper(self._h, taper))

    def get_taper(self) -> float:
        t = C.c_double()
        _check(lib().islf_get_taper(self._h, C.byref(t)))
        return t.value

    def get_grid(self) -> int:
        n = C.c_int32()
        _check(lib().islf_get_grid(self._h, C.byref(n)))
        return n.value

    def phase_timings(self, n_sweeps=4):
        """Mean ms per launch and launch counts of (A, B, closing F + fold):
        A = phase 3 of the previous sweep on row 0 + phase 0, B = phases 1 and 2."""
        ms = np.zeros(3, dtype=np.float64)
        cnt = np.zeros(3, dtype=np.uint32)
        _check(lib().islf_phase_timings(self._h, n_sweeps, ms.ctypes.data_as(C.c_void_p),
                                        cnt.ctypes.data_as(C.c_void_p)))
        return ms, cnt


def num_tiles(spin_format=INT8) -> int:
    n = C.c_int32()
    _check(lib().islf_num_tiles(spin_format, C.byref(n)))
    return n.value


def footprint_bytes(replica: Replica, spin_format=INT8, obs_capacity=1024) -> int:
    b = C.c_uint64()
    d = replica.to_c()
    _check(lib().islf_footprint_bytes(C.byref(d), spin_format, obs_capacity, C.byref(b)))
    return b.value


def plan_preview(replicas, spin_format=INT8, tile=-1, grid=2048):
    """The batched form's launch plan for these replicas as one launch chain
    of `grid` workgroups, computed on the host (no GPU): a dict with
    `shapes` (n, 4) = (tile variant, box columns or 0 for linear, box rows,
    x planes), `items` (k, 6) = (replica, x0, y0, j0, x steps, kind) and
    `first` (workgroup b runs items first[b] .. first[b+1]-1)."""
    n = len(replicas)
    descs = (ReplicaDesc * n)(*[r.to_c() for r in replicas])
    ni, nf = C.c_int32(), C.c_int32()
    _check(lib().islf_plan_preview(descs, n, spin_format, tile, grid, None, None, 0, C.byref(ni), None, 0,
                                   C.byref(nf)))
    shapes = np.zeros((n, 4), dtype=np.int32)
    items = np.zeros((max(ni.value, 1), 6), dtype=np.int32)
    first = np.zeros(max(nf.value, 1), dtype=np.int32)
    _check(lib().islf_plan_preview(descs, n, spin_format, tile, grid, shapes.ctypes.data_as(C.c_void_p),
                                   items.ctypes.data_as(C.c_void_p), items.shape[0], C.byref(ni),
                                   first.ctypes.data_as(C.c_void_p), first.shape[0], C.byref(nf)))
    return {"shapes": shapes, "items": items[:ni.value], "first": first[:nf.value]}


def energy(replica: Replica, records) -> np.ndarray:
    """Eq. 1 energies of (n, 4) int64 records (B, M, M1, Mn) with the
    replica's J, H, h1, hn: host FP64, no GPU (islf_energy)."""
    rec = np.ascontiguousarray(np.asarray(records, dtype=np.int64).reshape(-1, 4))
    out = np.zeros(rec.shape[0], dtype=np.float64)
    d = replica.to_c()
    _check(lib().islf_energy(C.byref(d), rec.ctypes.data_as(C.c_void_p), rec.shape[0],
                             out.ctypes.data_as(C.c_void_p)))
    return out


def integrate(h, mean_m1, mean_mn, c1=-1.0, cn=1.0, norm=1.0) -> np.ndarray:
    """Cumulative trapezoid of g = norm (c1 m1 + cn mn) over h (Eq. 9 / Eq. 22):
    host FP64 arrays in and out, no GPU (islf_integrate)."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    m1 = np.ascontiguousarray(mean_m1, dtype=np.float64)
    mn = np.ascontiguousarray(mean_mn, dtype=np.float64)
    if not (h.shape == m1.shape == mn.shape) or h.ndim != 1:
        raise ValueError("h, mean_m1, mean_mn must be 1-D arrays of one length")
    out = np.zeros(h.size, dtype=np.float64)
    _check(lib().islf_integrate(h.ctypes.data_as(C.c_void_p), m1.ctypes.data_as(C.c_void_p),
                                mn.ctypes.data_as(C.c_void_p), h.size, c1, cn, norm,
                                out.ctypes.data_as(C.c_void_p)))
    return out


def integrate_device(h, m1, mn, c1=-1.0, cn=1.0, norm=1.0, stream=None):
    """The same trapezoid by a kernel on the GPU (islf_integrate_device).

    Inputs are torch float64 CUDA tensors (or array-likes, copied to the GPU).
    Returns a float64 CUDA tensor.
    """
    torch = _torch()
    dev = torch.device("cuda")
    h = torch.as_tensor(h, dtype=torch.float64, device=dev).contiguous()
    m1 = torch.as_tensor(m1, dtype=torch.float64, device=dev).contiguous()
    mn = torch.as_tensor(mn, dtype=torch.float64, device=dev).contiguous()
    out = torch.empty_like(h)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().islf_integrate_device(C.c_void_p(h.data_ptr()), C.c_void_p(m1.data_ptr()),
                                       C.c_void_p(mn.data_ptr()), h.numel(), c1, cn, norm,
                                       C.c_void_p(out.data_ptr()), C.c_void_p(s.cuda_stream)))
    return out
