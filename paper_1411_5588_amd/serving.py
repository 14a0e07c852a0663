"""Serving loop: continuous batching of Monte Carlo requests on one GPU.

Each request is one Markov chain of the thin-film model (Sec. II.A Eq. 1 with
the generalized antiperiodic y boundary of Eq. 11) to be swept a given number
of times; its answer is the run's mean energy and (surface) magnetisations
(the Eq. 7 / Eq. 19 integrands) and its last record.  Requests arrive over
time; the server admits an arrived request as soon as a slot and enough of
the device-memory budget are free (footprint from islf_footprint_bytes),
keeps every admitted chain resident on the device, and sweeps all of them
together in batched launches.  A step sweeps the live chains by the smallest
number of sweeps any of them still needs (capped), so no chain overshoots;
finished chains are read back and retired, which frees their slot and memory
for the queue.

Every chain draws its randomness from its own (seed, replica id, sweep index),
so its answer is the same whether it runs alone or in any mix (tested).
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import islf


@dataclass
class Request:
    rid: int
    replica: islf.Replica
    sweeps: int
    arrival: float                      # seconds after the start of the run
    admitted: float = math.nan
    finished: float = math.nan
    slot: int = -1
    done: int = 0
    means: np.ndarray | None = None     # mean (E, B, M, M1, Mn) over all sweeps
    last: np.ndarray | None = None      # last (B, M, M1, Mn) record

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def updates(self) -> int:
        return self.replica.N * self.sweeps


def shape_for_sites(n_sites: float) -> tuple[int, int, int]:
    """A film of about n_sites sites with Lx : Ly : Lz close to 1 : 3 : 3."""
    Lx = max(2, int(round((n_sites / 9.0) ** (1.0 / 3.0))))
    L = max(2, 2 * int(round(math.sqrt(n_sites / Lx) / 2.0)))
    return Lx, L, L


def poisson_workload(n_requests: int, rate: float, seed: int = 14115588, min_sites: float = 1e5,
                     max_sites: float = 4.6e7, t_range=(2.0, 4.2), h1_range=(0.1, 1.0),
                     sweep_range=(500, 5000)) -> list[Request]:
    """Seeded synthetic request stream: Poisson arrivals at `rate` per second,
    sizes log-uniform on [min_sites, max_sites], T and h1 uniform, hn = -h1."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n = math.exp(rng.uniform(math.log(min_sites), math.log(max_sites)))
        Lx, Ly, Lz = shape_for_sites(n)
        T = rng.uniform(*t_range)
        h1 = rng.uniform(*h1_range)
        sweeps = int(rng.integers(sweep_range[0], sweep_range[1] + 1))
        rep = islf.Replica(Lx, Ly, Lz, islf.GAPBC, J=1.0, beta=1.0 / T, H=0.0, h1=h1, hn=-h1,
                           seed=seed + 1 + k, replica=k, init=islf.INIT_RANDOM)
        out.append(Request(k, rep, sweeps, t))
    return out


class Server:
    """Admission by memory footprint and slots, continuous batched sweeping."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, spin_format: int = islf.BITPACK,
                 max_step: int = 50, obs_capacity: int = 5000, realtime: bool = True):
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        self.fmt = spin_format
        self.max_step = max_step
        self.cap = obs_capacity
        self.realtime = realtime
        self.ctx: islf.Context | None = None
        self.used = 0
        self.busy_s = 0.0

    def footprint(self, req: Request) -> int:
        return islf.footprint_bytes(req.replica, self.fmt, self.cap)

    def _admit(self, req: Request, now: float):
        if self.ctx is None:
            self.ctx = islf.Context([req.replica], spin_format=self.fmt, obs_capacity=self.cap,
                                    exec_mode=islf.EXEC_BATCHED)
            req.slot = 0
        else:
            req.slot = self.ctx.add(req.replica)
        req.admitted = now
        self.used += self.footprint(req)

    def _finish(self, req: Request, now: float):
        req.means = self.ctx.replica_means(req.slot, 0, req.sweeps)
        req.last = self.ctx.measure(req.slot, req.sweeps - 1, 1)[0]
        self.ctx.retire(req.slot)
        self.used -= self.footprint(req)
        req.finished = now

    def run(self, requests: list[Request]) -> list[Request]:
        for r in requests:
            if r.sweeps > self.cap:
                raise ValueError(f"request {r.rid} needs {r.sweeps} records, capacity is {self.cap}")
            if self.footprint(r) > self.budget:
                raise ValueError(f"request {r.rid} does not fit the memory budget on its own")
        queue = deque(sorted(requests, key=lambda r: r.arrival))
        live: dict[int, Request] = {}
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if self.realtime else None
        sim_now = 0.0

        def now():
            return clock() if self.realtime else sim_now

        while queue or live:
            t = now()
            # admit arrived requests in arrival order while a slot and memory are free
            while queue and queue[0].arrival <= t and len(live) < self.max_slots and \
                    self.used + self.footprint(queue[0]) <= self.budget:
                req = queue.popleft()
                self._admit(req, t)
                live[req.slot] = req
            if not live:
                nxt = queue[0].arrival
                if self.realtime:
                    time.sleep(max(0.0, nxt - now()))
                else:
                    sim_now = nxt
                continue
            k = min(self.max_step, min(r.sweeps - r.done for r in live.values()))
            tb = time.perf_counter()
            self.ctx.sweep(k)
            for r in live.values():
                r.done += k
            finished = [r for r in live.values() if r.done == r.sweeps]
            if finished:
                for r in finished:
                    self._finish(r, now() if self.realtime else sim_now)
                    del live[r.slot]
            else:
                self.ctx.torch.cuda.synchronize()
            self.busy_s += time.perf_counter() - tb
            if not self.realtime:
                sim_now += time.perf_counter() - tb
        self.wall_s = now()
        return requests

    def close(self):
        if self.ctx is not None:
            self.ctx.close()
            self.ctx = None


def summary(requests: list[Request], wall_s: float, busy_s: float) -> dict:
    lat = np.array([r.latency for r in requests])
    total_updates = sum(r.updates for r in requests)
    return {"requests": len(requests),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "aggregate_updates_per_ns": total_updates / (wall_s * 1e9),
            "busy_updates_per_ns": total_updates / (busy_s * 1e9),
            "gpu_busy_fraction": busy_s / wall_s,
            "wall_s": wall_s}
