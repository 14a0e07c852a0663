"""Shared test utilities: seeded configurations and oracle drivers.

Input generation only; none of the method's arithmetic lives here (the oracle
does that on one side, the HIP library on the other).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import oracle as O

SEED = 14115588


def config1(**over):
    """12 x 24 x 24 film, generalized antiperiodic y, T = 3, h1 = +0.5, hn = -0.5."""
    kw = dict(Lx=12, Ly=24, Lz=24, ybc=O.GAPBC, J=1.0, beta=1.0 / 3.0, H=0.0, h1=0.5, hn=-0.5,
              seed=SEED, replica=0, init=O.INIT_RANDOM)
    kw.update(over)
    return kw


def oracle_lattice(p: dict, spins=None) -> O.Lattice:
    init = p.get("init", O.INIT_RANDOM)
    if init == 3:  # host spins
        init = O.INIT_UP
    return O.Lattice(p["Lx"], p["Ly"], p["Lz"], p.get("ybc", O.GAPBC), J=p.get("J", 1.0),
                     beta=p.get("beta", 1.0 / 3.0), H=p.get("H", 0.0), h1=p.get("h1", 0.0),
                     hn=p.get("hn", 0.0), seed=p.get("seed", 0), replica=p.get("replica", 0),
                     init=init, spins=spins)


def oracle_trajectory(p: dict, n: int, spins=None):
    """Initial spins, per-sweep records and final spins of the oracle chain."""
    L = oracle_lattice(p, spins)
    s0 = L.s.copy()
    rec = L.run(n)
    return s0, rec, L.s.copy()


def parallel_map(fn, items, workers=None):
    """ctypes releases the GIL, so oracle runs of independent replicas overlap."""
    workers = workers or min(16, os.cpu_count() or 4, max(1, len(items)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


def random_shape(rng):
    Lx = int(rng.integers(1, 7))
    Ly = int(rng.integers(2, 12))
    Lz = 2 * int(rng.integers(1, 22))
    return Lx, Ly, Lz
