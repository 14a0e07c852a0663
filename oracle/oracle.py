"""ctypes front end of the plain C oracle (``islf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.

The C file implements, for the thin-film Ising model of arXiv:1411.5588:
the Hamiltonian of Sec. II.A Eq. 1 with free x-surfaces carrying fields h1
(x = 0, the paper's layer 1) and hn (x = Lx-1, layer n), periodic z, and a y
boundary that is periodic, antiperiodic or the generalized antiperiodic
condition of Eq. 11; checkerboard Metropolis sweeps (Appendix) with Philox
draws; full-recompute observables (Eq. 7, Eq. 19 integrands), the layer
profile of Eq. 17 and the trapezoid thermodynamic integration of Eq. 9 /
Eq. 22.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "islf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PBC, APBC, GAPBC = 0, 1, 2
INIT_RANDOM, INIT_UP, INIT_DOWN = 0, 1, 2


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no FMA contraction) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build_oracle()
        L = C.CDLL(_LIB)
        vp, i32, u32, u64, i64, dbl = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_int64, C.c_double
        L.oracle_new.restype = vp
        L.oracle_new.argtypes = [i32, i32, i32, i32, dbl, dbl, dbl, dbl, dbl, u64, u32]
        L.oracle_free.argtypes = [vp]
        L.oracle_nsites.restype = i64
        L.oracle_nsites.argtypes = [vp]
        L.oracle_neighbours.restype = i32
        L.oracle_neighbours.argtypes = [vp, i64, vp, vp]
        L.oracle_phase.restype = i32
        L.oracle_phase.argtypes = [vp, i64]
        L.oracle_delta_e.restype = dbl
        L.oracle_delta_e.argtypes = [vp, vp, i64]
        L.oracle_threshold_of_de.restype = u64
        L.oracle_threshold_of_de.argtypes = [dbl, dbl]
        L.oracle_site_threshold.restype = u64
        L.oracle_site_threshold.argtypes = [vp, vp, i64]
        L.oracle_site_draw.restype = u32
        L.oracle_site_draw.argtypes = [vp, i64, u32, u32]
        L.oracle_counter_fits.restype = i32
        L.oracle_counter_fits.argtypes = [vp]
        L.oracle_init.argtypes = [vp, vp, i32]
        L.oracle_sweep.argtypes = [vp, vp, u32, vp]
        L.oracle_phase_step.argtypes = [vp, vp, u32, i32]
        L.oracle_observables.argtypes = [vp, vp, vp]
        L.oracle_energy.restype = dbl
        L.oracle_energy.argtypes = [dbl, dbl, dbl, dbl, vp]
        L.oracle_energy_at.restype = dbl
        L.oracle_energy_at.argtypes = [dbl, dbl, dbl, dbl, vp]
        L.oracle_run.argtypes = [vp, vp, u32, u32, vp]
        L.oracle_mean.restype = dbl
        L.oracle_mean.argtypes = [vp, i64, i64]
        L.oracle_integrate.argtypes = [vp, vp, vp, i32, dbl, dbl, dbl, vp]
        L.oracle_philox.argtypes = [vp, vp, vp]
        L.oracle_layer_profile.argtypes = [vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox(counter, key) -> np.ndarray:
    """Philox4x32-10 of a 4-word counter under a 2-word key."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def threshold_of_de(beta: float, dE: float) -> int:
    return int(lib().oracle_threshold_of_de(beta, dE))


def energy(J, H, h1, hn, obs) -> float:
    """Eq. 1 at one record (B, M, M1, Mn): an integer record, or (floats)
    the means of records."""
    a = np.asarray(obs)
    if np.issubdtype(a.dtype, np.integer):
        o = np.ascontiguousarray(a, dtype=np.int64)
        return float(lib().oracle_energy(J, H, h1, hn, _ptr(o)))
    o = np.ascontiguousarray(a, dtype=np.float64)
    return float(lib().oracle_energy_at(J, H, h1, hn, _ptr(o)))


def integrate(h, m1, mn, c1=-1.0, cn=1.0, norm=1.0) -> np.ndarray:
    """Cumulative trapezoid of g_r = norm (c1 m1_r + cn mn_r) over h (Eq. 9)."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    m1 = np.ascontiguousarray(m1, dtype=np.float64)
    mn = np.ascontiguousarray(mn, dtype=np.float64)
    out = np.zeros(len(h), dtype=np.float64)
    lib().oracle_integrate(_ptr(h), _ptr(m1), _ptr(mn), len(h), c1, cn, norm, _ptr(out))
    return out


def mean(records: np.ndarray, column: int, first: int = 0, count: int | None = None) -> float:
    """(double) sum / (double) count of one column of int64 records."""
    rec = np.ascontiguousarray(records, dtype=np.int64)
    if count is None:
        count = rec.shape[0] - first
    sub = np.ascontiguousarray(rec[first:first + count, column])
    return float(lib().oracle_mean(_ptr(sub), 1, count))


class Lattice:
    """One replica: geometry + parameters, an explicit bond list, and spins."""

    def __init__(self, Lx, Ly, Lz, ybc=GAPBC, J=1.0, beta=1.0 / 3.0, H=0.0, h1=0.0, hn=0.0,
                 seed=0, replica=0, init=INIT_RANDOM, spins=None):
        self.Lx, self.Ly, self.Lz, self.ybc = int(Lx), int(Ly), int(Lz), int(ybc)
        self.J, self.beta, self.H, self.h1, self.hn = float(J), float(beta), float(H), float(h1), float(hn)
        self.seed, self.replica = int(seed), int(replica)
        h = lib().oracle_new(self.Lx, self.Ly, self.Lz, self.ybc, self.J, self.beta, self.H,
                             self.h1, self.hn, self.seed & (2**64 - 1), self.replica)
        if not h:
            raise ValueError("invalid lattice parameters")
        self._h = h
        self.N = int(lib().oracle_nsites(h))
        self.t = 0
        self.s = np.zeros(self.N, dtype=np.int8)
        if spins is not None:
            self.s[:] = np.asarray(spins, dtype=np.int8).reshape(-1)
        else:
            lib().oracle_init(h, _ptr(self.s), int(init))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_free(h)
            self._h = None

    # geometry -----------------------------------------------------------
    def neighbours(self, i):
        nb = np.zeros(6, dtype=np.int32)
        sg = np.zeros(6, dtype=np.int8)
        k = lib().oracle_neighbours(self._h, int(i), _ptr(nb), _ptr(sg))
        return nb[:k].copy(), sg[:k].copy()

    def phase(self, i) -> int:
        return int(lib().oracle_phase(self._h, int(i)))

    def counter_fits(self) -> bool:
        return bool(lib().oracle_counter_fits(self._h))

    # local update rule --------------------------------------------------
    def delta_e(self, i, s=None) -> float:
        s = self.s if s is None else np.ascontiguousarray(s, dtype=np.int8)
        return float(lib().oracle_delta_e(self._h, _ptr(s), int(i)))

    def site_threshold(self, i, s=None) -> int:
        s = self.s if s is None else np.ascontiguousarray(s, dtype=np.int8)
        return int(lib().oracle_site_threshold(self._h, _ptr(s), int(i)))

    def site_draw(self, i, t, domain=0) -> int:
        return int(lib().oracle_site_draw(self._h, int(i), int(t), int(domain)))

    # dynamics -----------------------------------------------------------
    def sweep(self, order=None):
        o = None
        if order is not None:
            order = np.ascontiguousarray(order, dtype=np.int64)
            o = _ptr(order)
        lib().oracle_sweep(self._h, _ptr(self.s), self.t, o)
        self.t += 1

    def phase_step(self, p, t=None, s=None):
        s = self.s if s is None else s
        lib().oracle_phase_step(self._h, _ptr(s), self.t if t is None else int(t), int(p))

    def run(self, n) -> np.ndarray:
        rec = np.zeros((n, 4), dtype=np.int64)
        if n:
            lib().oracle_run(self._h, _ptr(self.s), self.t, n, _ptr(rec))
        self.t += n
        return rec

    def observables(self, s=None) -> np.ndarray:
        s = self.s if s is None else np.ascontiguousarray(s, dtype=np.int8)
        out = np.zeros(4, dtype=np.int64)
        lib().oracle_observables(self._h, _ptr(s), _ptr(out))
        return out

    def energy(self, obs) -> float:
        return energy(self.J, self.H, self.h1, self.hn, obs)

    def layer_profile(self, s=None) -> np.ndarray:
        """(Lx, Ly) int64: sum over z of the spins of each row (Eq. 17 times Lz)."""
        s = self.s if s is None else np.ascontiguousarray(s, dtype=np.int8)
        out = np.zeros(self.Lx * self.Ly, dtype=np.int64)
        lib().oracle_layer_profile(self._h, _ptr(s), _ptr(out))
        return out.reshape(self.Lx, self.Ly)

    def spins3d(self) -> np.ndarray:
        return self.s.reshape(self.Lx, self.Ly, self.Lz)
