"""Throughput benchmark: spin updates/ns of checkerboard Metropolis sweeps.

Workload: the paper-scale thin film 160 x 480 x 600 (46.08 M sites),
generalized antiperiodic y boundary, J = 1, h1 = +0.55 on x = 0 and
hn = -0.55 on x = Lx-1, random initial state from the seed, one replica per
temperature T in {2, 3, 4} (beta = 1/T), all three swept together by one
graph launch per chunk of sweeps.  A step is one sweep of every replica: four
checkerboard phases with the fused per-sweep observable reductions and the
per-sweep record.  Inputs are synthetic (seeded) and resident in HBM before
timing starts; nothing is copied to the host inside the timed region.

Prints one JSON line.  Besides the headline (bit-packed spins, batched form)
it reports the int8 format and the plain one-lattice-per-launch and
persistent forms on the same workload, the roofline of the dominant kernel
(the sweep kernel) and the CPU oracle timed on a bounded sample of the same
workload.

The batched form deals the replicas into concurrent groups, each sweeping on
its own stream, so the sweep kernel's launches of one kind (A or B) run as a
wave of concurrent dispatches that together update half a sweep of every
replica.  The roofline's unit is that launch wave: its algorithmic operations
over its average duration, i.e. the timed region (HIP events on the
context's stream, which forks to and joins from the group streams) divided by
the waves in it.  The same form run as one launch chain over all replicas,
timed the same way, gives the sweep kernel's own per-launch time beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SHAPE = (160, 480, 600)
TEMPS = (2.0, 3.0, 4.0)
H1 = 0.55
SEED = 14115588

# MI355X: 256 CUs x 4 SIMDs at 2.4 GHz.  A SIMD issues one wave64 VALU
# instruction per 4 cycles (16 lanes per clock: 39.3 T lane-ops/s), and a
# second one from another wave in the same 4 cycles when both are simple
# 32-bit operations (32 lanes per clock: 78.6 T lane-ops/s, the 157.3 TFLOP/s
# fp32 vector rate with an FMA counted twice); a 64-bit integer product
# (multiply-hi/lo) takes a whole issue slot.  HBM3E peak 8 TB/s.
VALU32_PEAK = 256 * 4 * 32 * 2.4e9
VALU64_PEAK = 256 * 4 * 16 * 2.4e9
SINGLE_ISSUE_PEAK = VALU64_PEAK   # every instruction in its own issue slot
HBM_PEAK_GBS = 8000.0
# algorithmic integer operations per spin update: Philox4x32-10 gives four
# words for 10 rounds x (2 multiply-hi/lo + 2 three-input xor), i.e. 5 products
# and 5 xors per update; the Metropolis test adds 7 (5 adds for the
# six-neighbour sum, 1 compare against the tabulated threshold, 1 select of the
# flip).  The ALU roofline is that mix at the two issue rates, an upper bound:
# the products and the three-input xors of Philox do not dual-issue in
# practice, so the single-issue rate is reported beside it.
OPS64, OPS32 = 5, 12
OPS_PER_UPDATE = OPS64 + OPS32
PEAK_UPDATES = 1.0 / (OPS64 / VALU64_PEAK + OPS32 / VALU32_PEAK)   # updates per second
ALU_PEAK_TOPS = OPS_PER_UPDATE * PEAK_UPDATES / 1e12
BYTES_PER_UPDATE = {"int8": 2.0, "bitpack": 0.25}   # each spin read and written once per sweep
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_sweep_kernel_160x480x600x3.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1411_5588_amd", "csrc", "islf_kernels.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--chunk", type=int, default=50, help="sweeps per captured graph launch")
    ap.add_argument("--groups", type=int, default=0,
                    help="concurrent replica groups of the batched form (0: automatic, 1: one launch chain)")
    ap.add_argument("--form", choices=["persistent", "batched", "plain"], default="batched")
    ap.add_argument("--fmt", choices=["int8", "bitpack"], default="bitpack")
    ap.add_argument("--no-extras", action="store_true", help="skip the other forms and formats")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sweeps", type=int, default=3)
    ap.add_argument("--serve", type=int, default=0, metavar="N",
                    help="instead: the serving workload, N Poisson requests (20/s, log-uniform sizes)")
    ap.add_argument("--serve-budget-mib", type=int, default=256)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (traffic counter calibration)")
    return ap.parse_args()


def replicas(islf, n=None):
    """One replica per temperature; n > 3 cycles through the temperatures
    (larger-than-cache batches)."""
    Lx, Ly, Lz = SHAPE
    n = len(TEMPS) if n is None else n
    return [islf.Replica(Lx, Ly, Lz, islf.GAPBC, J=1.0, beta=1.0 / TEMPS[i % len(TEMPS)], H=0.0, h1=H1, hn=-H1,
                         seed=SEED + i, replica=i, init=islf.INIT_RANDOM) for i in range(n)]


def run_form(islf, torch, form, fmt, steps, warmup, chunk, n_reps=None, groups=0):
    mode = {"persistent": islf.EXEC_PERSISTENT, "batched": islf.EXEC_BATCHED, "plain": islf.EXEC_PLAIN}[form]
    f = {"int8": islf.INT8, "bitpack": islf.BITPACK}[fmt]
    reps = replicas(islf, n_reps)
    ctx = islf.Context(reps, spin_format=f, obs_capacity=steps + warmup + 64, exec_mode=mode)
    try:
        chunk = max(1, min(chunk, steps))
        if groups:
            ctx.set_groups(groups)
        ctx.capture(chunk)
        # warm-up: replays of the same graph (its first launch is slower), then
        # eager sweeps for the remainder
        if warmup // chunk:
            ctx.replay(warmup // chunk)
        if warmup % chunk:
            ctx.sweep(warmup % chunk)
        n_launch = steps // chunk
        rest = steps - n_launch * chunk
        s = ctx.stream
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(s)
        for _ in range(n_launch):
            ctx.replay(1)
        if rest:
            ctx.sweep(rest)
        t1.record(s)
        torch.cuda.synchronize()
        total_ms = t0.elapsed_time(t1)
        for i in range(len(reps)):
            assert ctx.sweep_count(i) == warmup + steps
        return dict(ms_per_sweep=total_ms / steps, sweeps_per_launch=chunk, launches=n_launch,
                    groups=ctx.get_groups() if form == "batched" else 1, grid=ctx.get_grid())
    finally:
        ctx.close()


def layer_profile_rate(islf, torch, calls=20):
    """The layer-profile reduction (Eq. 17) on one bit-packed replica of the
    workload: microseconds per call (HIP events on the context's stream) and
    the spin bytes it reads per second."""
    Lx, Ly, Lz = SHAPE
    with islf.Context(replicas(islf)[:1], spin_format=islf.BITPACK, obs_capacity=8) as ctx:
        acc = torch.zeros((Lx, Ly), dtype=torch.int64, device="cuda")
        ctx.sweep(2)
        ctx.layer_profile_add(0, acc)
        s = ctx.stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        # back-to-back launches on the context's stream (no host round trips
        # between them), bracketed by events on that stream
        ptr = islf.C.c_void_p(acc.data_ptr())
        e0.record(s)
        for _ in range(calls):
            islf.lib().islf_layer_profile_add(ctx._h, 0, ptr)
        e1.record(s)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / calls
    spin_bytes = Lx * Ly * 2 * 4 * ((Lz + 63) // 64)
    return {"us_per_call": round(us, 2), "spin_GBs": round(spin_bytes / (us * 1e-6) / 1e9, 1),
            "replica": f"{Lx}x{Ly}x{Lz} bit-packed"}


def host_io_rate(islf, torch, fmt, chunk, ms_per_sweep):
    """The boundary's host hand-over for one replica of the workload: a full
    spin export (device kernel + copy into pageable host memory, int8 +-1 in
    the host layout) and a full import, wall-clock milliseconds; and the
    whole-job rate if every replica's spins went to the host after each graph
    launch of `chunk` sweeps."""
    Lx, Ly, Lz = SHAPE
    N = Lx * Ly * Lz
    f = {"int8": islf.INT8, "bitpack": islf.BITPACK}[fmt]
    r = replicas(islf)[:1]
    with islf.Context(r, spin_format=f, obs_capacity=8) as ctx:
        s = ctx.get_spins(0)
        t = time.perf_counter()
        for _ in range(3):
            s = ctx.get_spins(0)
        get_ms = (time.perf_counter() - t) * 1e3 / 3
    with islf.Context(r, spin_format=f, obs_capacity=8) as ctx:
        t = time.perf_counter()
        ctx.set_spins(0, s)
        set_ms = (time.perf_counter() - t) * 1e3
    n = len(TEMPS)
    launch_ms = chunk * ms_per_sweep
    return {"get_spins_ms": round(get_ms, 2), "set_spins_ms": round(set_ms, 2),
            "host_GBs": round(N / (get_ms * 1e-3) / 1e9, 1),
            "pcie_inclusive_value": round(n * N * chunk / ((launch_ms + n * get_ms) * 1e6), 2),
            "pcie_inclusive_case": f"all {n} replicas' spins copied to the host after every {chunk} sweeps"}


def kernel_code_hash():
    """Hash of the kernel source with // comments, trailing blanks and empty
    lines removed: edits to comments leave it, and the counters it guards,
    unchanged (the source has no block comments and no "//" in strings)."""
    lines = []
    with open(KERNEL_SOURCE, encoding="utf-8") as f:
        for ln in f:
            ln = ln.split("//", 1)[0].rstrip()
            if ln:
                lines.append(ln)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def committed_traffic(fmt):
    """HBM bytes per launch wave of the sweep kernel (the A or B dispatches of
    all groups, half a sweep of every replica) from the committed counter
    summary, or None when the kernel code has changed since it was taken."""
    try:
        text = open(PROFILE_TRAFFIC).read()
    except OSError:
        return None
    m = re.search(r"kernel_code_sha256_16:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_code_hash():
        return None
    m = re.search(rf"traffic_bytes_per_wave\[{fmt}\]:\s*([0-9.eE+]+)", text)
    return float(m.group(1)) if m else None


def cpu_baseline(n_sweeps, max_threads=16):
    """The oracle as it stands on the host: single-threaded on one replica of
    the workload, and replica-parallel (one replica per thread, each thread
    in the oracle's own C code, which holds no shared state) on up to
    `max_threads` of the cores this process may use.  Each thread's replica
    takes about 2.2 GB of oracle bond lists."""
    import threading

    from oracle import oracle as O
    Lx, Ly, Lz = SHAPE
    N = Lx * Ly * Lz

    def lattice(i):
        return O.Lattice(Lx, Ly, Lz, O.GAPBC, J=1.0, beta=1.0 / TEMPS[i % len(TEMPS)], H=0.0, h1=H1, hn=-H1,
                         seed=SEED + i, replica=i)

    L = lattice(1)
    t = time.perf_counter()
    L.run(n_sweeps)
    dt = time.perf_counter() - t
    del L
    out = dict(value=round(N * n_sweeps / (dt * 1e9), 5), unit="spin updates/ns", cores=1, kind="oracle",
               sample=f"{n_sweeps} sweeps of one {Lx}x{Ly}x{Lz} replica (T=3, GAPBC, h1=+-{H1}), observables "
                      f"recomputed after each sweep; {dt:.1f} s single-threaded on the host CPU")

    n = max(1, min(max_threads, len(os.sched_getaffinity(0))))
    lats = [None] * n
    span = [0.0, 0.0]
    ready = threading.Barrier(n + 1)
    done = threading.Barrier(n + 1)

    def work(i):
        lats[i] = lattice(i)
        ready.wait()
        lats[i].run(1)
        done.wait()

    threads = [threading.Thread(target=work, args=(i,)) for i in range(n)]
    for th in threads:
        th.start()
    ready.wait()
    span[0] = time.perf_counter()
    done.wait()
    span[1] = time.perf_counter()
    for th in threads:
        th.join()
    del lats
    dta = span[1] - span[0]
    out["all_core"] = dict(value=round(n * N / (dta * 1e9), 5), cores=n,
                           sample=f"{n} replicas of {Lx}x{Ly}x{Lz} (T cycling over {list(TEMPS)}), one sweep "
                                  f"each, one thread per replica; {dta:.1f} s wall")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the sweep path runs on a "
              f"single GPU and sharding across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1411_5588_amd import islf
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": n}), flush=True)
        return

    if args.serve:
        from paper_1411_5588_amd import serving
        reqs = serving.poisson_workload(args.serve, rate=20.0)
        srv = serving.Server(budget_bytes=args.serve_budget_mib << 20, max_slots=64, spin_format=islf.BITPACK,
                             max_step=50, obs_capacity=5000, realtime=True)
        try:
            srv.run(reqs)
        finally:
            srv.close()
        s = serving.summary(reqs, srv.wall_s, srv.busy_s)
        print(json.dumps({"metric": "serving", "workload": f"{args.serve} requests, Poisson 20/s, sites "
                          f"log-uniform on [1e5, 4.6e7], T~U[2,4.2], h1~U[0.1,1], hn=-h1, sweeps~U{{500..5000}}, "
                          f"bit-packed, memory budget {args.serve_budget_mib} MiB",
                          **{k: round(v, 4) for k, v in s.items()}}), flush=True)
        return

    Lx, Ly, Lz = SHAPE
    N = Lx * Ly * Lz
    n_reps = len(TEMPS)
    updates_per_sweep = N * n_reps

    main_run = run_form(islf, torch, args.form, args.fmt, args.steps, args.warmup, args.chunk, groups=args.groups)
    print(f"# {args.form}/{args.fmt}: {main_run}", file=sys.stderr, flush=True)
    value = updates_per_sweep / (main_run["ms_per_sweep"] * 1e6)
    # the same form as one launch chain over all replicas, timed the same way
    if main_run["groups"] == 1:
        chain_run = main_run
    else:
        chain_run = run_form(islf, torch, args.form, args.fmt, min(args.steps, 400), min(args.warmup, 100),
                             args.chunk, groups=1)
        print(f"# {args.form}/{args.fmt} one launch chain: {chain_run}", file=sys.stderr, flush=True)

    forms = {}
    if not args.no_extras:
        for form, fmt in (("plain", "bitpack"), ("batched", "int8"), ("plain", "int8"), ("persistent", "bitpack"),
                          ("persistent", "int8")):
            if (form, fmt) == (args.form, args.fmt):
                continue
            r = run_form(islf, torch, form, fmt, min(args.steps, 100), min(args.chunk, 50), min(args.chunk, 50))
            forms[f"{form}_{fmt}"] = round(updates_per_sweep / (r["ms_per_sweep"] * 1e6), 2)
            print(f"# {form}/{fmt}: {r}", file=sys.stderr, flush=True)
        # a batch larger than the 256 MB last-level cache: 8 int8 replicas, 369 MB of spins
        r = run_form(islf, torch, "batched", "int8", min(args.steps, 50), min(args.chunk, 50), min(args.chunk, 50),
                     n_reps=8)
        forms["batched_int8_8x46M_369MB"] = round(8 * N / (r["ms_per_sweep"] * 1e6), 2)
        print(f"# batched/int8 x8: {r}", file=sys.stderr, flush=True)

    # dominant kernel: the sweep kernel.  Its A and B launches of one sweep
    # together update every site of every replica once (A: phase 0 and the
    # previous sweep's phase 3, B: phases 1 and 2), so a launch wave (the A or
    # B dispatches of all concurrent groups) updates half a sweep of every
    # replica; its average duration is the timed region over its 2 x steps
    # waves (the region also holds one closing launch and fold per graph
    # launch, so this slightly overstates the wave time)
    updates_per_wave = n_reps * N / 2
    wave_ms = main_run["ms_per_sweep"] / 2
    achieved_tops = OPS_PER_UPDATE * updates_per_wave / (wave_ms * 1e-3) / 1e12
    # one launch chain over all replicas: its launches run one after another,
    # so the same quotient is the sweep kernel's own per-launch time
    chain_ms = chain_run["ms_per_sweep"] / 2
    chain_tops = OPS_PER_UPDATE * updates_per_wave / (chain_ms * 1e-3) / 1e12
    traffic = committed_traffic(args.fmt)
    alg_gbs = BYTES_PER_UPDATE[args.fmt] * updates_per_wave / (wave_ms * 1e-3) / 1e9
    roofline = {"bound": "alu", "achieved": round(achieved_tops, 2), "peak": round(ALU_PEAK_TOPS, 1),
                "unit": "T int-op/s", "frac": round(achieved_tops / ALU_PEAK_TOPS, 4), "traffic": traffic,
                "kernel": "k_sweep (A and B launches)",
                "peak_basis": f"per update {OPS64} 64-bit products at {VALU64_PEAK / 1e12:.1f} T/s + {OPS32} 32-bit "
                              f"ops at {VALU32_PEAK / 1e12:.1f} T/s = {PEAK_UPDATES / 1e9:.0f} updates/ns",
                "launch_unit": f"wave of {main_run['groups']} concurrent group dispatches of "
                               f"{main_run['grid']} workgroups, half a sweep of every replica",
                "wave_ms": round(wave_ms, 5), "ops_per_update": OPS_PER_UPDATE,
                "single_chain": {"kernel_ms": round(chain_ms, 5), "workgroups": chain_run["grid"],
                                 "achieved": round(chain_tops, 2), "frac": round(chain_tops / ALU_PEAK_TOPS, 4)},
                "single_issue": {"peak": round(SINGLE_ISSUE_PEAK / 1e12, 1),
                                 "frac": round(achieved_tops * 1e12 / SINGLE_ISSUE_PEAK, 4)},
                "hbm_view": {"algorithmic_GBs": round(alg_gbs, 1), "peak_GBs": HBM_PEAK_GBS,
                             "frac": round(alg_gbs / HBM_PEAK_GBS, 4)}}

    prof = layer_profile_rate(islf, torch)
    print(f"# layer profile: {prof}", file=sys.stderr, flush=True)
    hio = host_io_rate(islf, torch, args.fmt, main_run["sweeps_per_launch"], main_run["ms_per_sweep"])
    print(f"# host io: {hio}", file=sys.stderr, flush=True)

    cpu = None if args.no_cpu else cpu_baseline(args.cpu_sweeps)
    line = {
        "metric": "spin updates/ns", "value": round(value, 2), "unit": "spin updates/ns", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(main_run["ms_per_sweep"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32" if args.fmt == "bitpack" else "int8", "data": "synthetic",
        "config": {"workload": f"thin film {Lx}x{Ly}x{Lz} GAPBC, h1=+{H1}/hn=-{H1}, one replica per T in "
                               f"{list(TEMPS)}, {args.fmt} spins, {args.form} form, "
                               f"{main_run['sweeps_per_launch']} sweeps per graph launch",
                   "sites_per_replica": N, "replicas": n_reps, "form": args.form, "spin_format": args.fmt,
                   "groups": main_run["groups"], "workgroups_per_launch": main_run["grid"]},
        "forms": forms,
        "roofline": roofline,
        "layer_profile": prof,
        "host_io": hio,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
