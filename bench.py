"""Throughput benchmark: spin updates/ns of checkerboard Metropolis sweeps.

Workload (default): the paper-scale thin film 160 x 480 x 600 (46.08 M sites),
generalized antiperiodic y boundary, J = 1, h1 = +0.55 on x = 0 and
hn = -0.55 on x = Lx-1, random initial state from the seed, one replica per
temperature T in {2, 3, 4} (beta = 1/T), all three swept together in one
persistent, graph-captured launch.  A step is one sweep of every replica:
four checkerboard phases with the fused per-sweep observable reductions.
Inputs are synthetic (seeded), resident in HBM before timing starts.

Prints one JSON line (rank 0, one GPU).  Also reports the plain
one-lattice-per-launch form and the bit-packed spin format on the same
workload, the roofline of the dominant kernel, and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SHAPE = (160, 480, 600)
TEMPS = (2.0, 3.0, 4.0)
H1 = 0.55
SEED = 14115588

# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
NUM_CU = 256
CLOCK_GHZ = 2.4
LANES_PER_CU = 64          # VALU lanes per CU per clock (4 SIMDs x 16)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--chunk", type=int, default=50, help="sweeps per captured graph launch")
    ap.add_argument("--form", choices=["persistent", "batched", "plain"], default="batched")
    ap.add_argument("--fmt", choices=["int8", "bitpack"], default="int8")
    ap.add_argument("--no-extras", action="store_true", help="skip the plain / bit-packed side runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sweeps", type=int, default=3)
    return ap.parse_args()


def replicas(islf):
    Lx, Ly, Lz = SHAPE
    return [islf.Replica(Lx, Ly, Lz, islf.GAPBC, J=1.0, beta=1.0 / T, H=0.0, h1=H1, hn=-H1, seed=SEED + i,
                         replica=i, init=islf.INIT_RANDOM) for i, T in enumerate(TEMPS)]


def run_form(islf, torch, form, fmt, steps, warmup, chunk):
    """Returns (ms per sweep, kernel ms per launch, launches, sweeps per launch)."""
    mode = {"persistent": islf.EXEC_PERSISTENT, "batched": islf.EXEC_BATCHED, "plain": islf.EXEC_PLAIN}[form]
    f = {"int8": islf.INT8, "bitpack": islf.BITPACK}[fmt]
    reps = replicas(islf)
    ctx = islf.Context(reps, spin_format=f, obs_capacity=steps + warmup + 8, exec_mode=mode)
    try:
        chunk = max(1, min(chunk, steps))
        if warmup:
            ctx.sweep(warmup)
        ctx.capture(chunk)
        n_launch = steps // chunk
        rest = steps - n_launch * chunk
        torch.cuda.synchronize()
        s = ctx.stream
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(n_launch)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(n_launch)]
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        t0.record(s)
        for i in range(n_launch):
            starts[i].record(s)
            ctx.replay(1)
            ends[i].record(s)
        if rest:
            ctx.sweep(rest)
        t1.record(s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        total_ms = t0.elapsed_time(t1)
        per_launch = [a.elapsed_time(b) for a, b in zip(starts, ends)]
        # the run must be whole: every replica advanced by warmup + steps sweeps
        for i in range(len(reps)):
            assert ctx.sweep_count(i) == warmup + steps
        rec = ctx.measure(0, warmup + steps - 1, 1)
        assert rec.shape == (1, 4)
        return dict(ms_per_sweep=total_ms / steps, wall_s=wall, launch_ms=sum(per_launch) / max(1, len(per_launch)),
                    sweeps_per_launch=chunk, launches=n_launch)
    finally:
        ctx.close()


def cpu_baseline(n_sweeps):
    """The oracle as it stands, single-threaded, on one replica of the workload."""
    from oracle import oracle as O
    Lx, Ly, Lz = SHAPE
    L = O.Lattice(Lx, Ly, Lz, O.GAPBC, J=1.0, beta=1.0 / 3.0, H=0.0, h1=H1, hn=-H1, seed=SEED + 1, replica=1)
    t = time.perf_counter()
    L.run(n_sweeps)
    dt = time.perf_counter() - t
    N = Lx * Ly * Lz
    return dict(value=N * n_sweeps / (dt * 1e9), unit="spin updates/ns", cores=1, kind="oracle",
                sample=f"{n_sweeps} sweeps of one {Lx}x{Ly}x{Lz} replica (T=3), observables recomputed "
                       f"after each sweep, {dt:.1f} s on the host CPU")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the sweep path is "
              f"single-GPU and multi-GPU sharding is not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1411_5588_amd import islf
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    Lx, Ly, Lz = SHAPE
    N = Lx * Ly * Lz
    n_reps = len(TEMPS)
    updates_per_sweep = N * n_reps

    main_run = run_form(islf, torch, args.form, args.fmt, args.steps, args.warmup, args.chunk)
    print(f"# {args.form}/{args.fmt}: {main_run}", file=sys.stderr, flush=True)
    value = updates_per_sweep / (main_run["ms_per_sweep"] * 1e6)

    extras = {}
    if not args.no_extras:
        for form, fmt in (("plain", "int8"), ("batched", "bitpack")):
            if (form, fmt) == (args.form, args.fmt):
                continue
            r = run_form(islf, torch, form, fmt, min(args.steps, 100), 5, min(args.chunk, 50))
            extras[f"{form}_{fmt}"] = round(updates_per_sweep / (r["ms_per_sweep"] * 1e6), 2)
            print(f"# {form}/{fmt}: {r}", file=sys.stderr, flush=True)

    # roofline of the dominant kernel (the sweep kernel: one launch covers
    # sweeps_per_launch sweeps of all replicas)
    bytes_per_update = 2.0 if args.fmt == "int8" else 0.25
    sweeps_per_launch = main_run["sweeps_per_launch"]
    launch_s = main_run["launch_ms"] * 1e-3
    achieved_gbs = bytes_per_update * updates_per_sweep * sweeps_per_launch / launch_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": None}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.cpu_sweeps)
        cpu["value"] = round(cpu["value"], 5)

    line = {
        "metric": "spin updates/ns", "value": round(value, 2), "unit": "spin updates/ns", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(main_run["ms_per_sweep"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.fmt if args.fmt == "int8" else "u32",
        "data": "synthetic",
        "config": {"workload": f"thin film {Lx}x{Ly}x{Lz} GAPBC, h1=+{H1}/hn=-{H1}, T in {list(TEMPS)}, "
                               f"{n_reps} replicas in one {args.form} graph-captured launch, {args.fmt} spins",
                   "sites_per_replica": N, "replicas": n_reps, "form": args.form, "spin_format": args.fmt,
                   "sweeps_per_launch": sweeps_per_launch},
        "forms": extras,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
