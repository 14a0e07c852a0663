"""Throughput benchmark: spin updates/ns of checkerboard Metropolis sweeps.

Workload: the paper-scale thin film 160 x 480 x 600 (46.08 M sites),
generalized antiperiodic y boundary, J = 1, h1 = +0.55 on x = 0 and
hn = -0.55 on x = Lx-1, random initial state from the seed, one replica per
temperature T in {2, 3, 4} (beta = 1/T), all three swept together by one
graph launch per chunk of sweeps.  A step is one sweep of every replica: four
checkerboard phases with the fused per-sweep observable reductions and the
per-sweep record.  Inputs are synthetic (seeded) and resident in HBM before
timing starts; nothing is copied to the host inside the timed region.

Prints one JSON line.  Besides the headline (batched form) it reports the
other spin format, the plain one-lattice-per-launch and persistent forms on
the same workload, a batch larger than the last-level cache, the batched
thermodynamic-integration batch (64 x 40x120x120 along the surface field),
the uneven autotuned batch (96 replicas of nine shapes) and the serving loop
(Poisson arrivals, p50/p99 latency); the HBM roofline of the dominant kernel
(the sweep kernel) and the CPU oracle timed on a bounded sample of the same
workload.

Roofline: algorithmic bytes (each updated spin read and written once per
sweep: 2 B int8, 0.25 B bit-packed) of one sweep-kernel launch over its
average duration.  A launch (A or B) updates half a sweep of every replica.
The per-launch time is taken from the form run as one launch chain over all
replicas (graph replay, HIP events on the context's stream, timed region
over its launches), the configuration a rocprofv3 kernel trace times the
same way; the batched form's concurrent group dispatches give the
`grouped_wave` figure beside it.
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

# MI355X HBM3E peak, 8 TB/s
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"int8": 2.0, "bitpack": 0.25}   # each spin read and written once per sweep
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_sweep_kernel_160x480x600x3.md")
PROFILE_VALU = os.path.join(ROOT, "profiles", "valu_sweep_kernel_160x480x600x3.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1411_5588_amd", "csrc", "islf_kernels.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--chunk", type=int, default=50, help="sweeps per captured graph launch")
    ap.add_argument("--min-warmup-s", type=float, default=0.5,
                    help="untimed graph replays continue until this many seconds of warm-up have passed")
    ap.add_argument("--groups", type=int, default=0,
                    help="concurrent replica groups of the batched form (0: automatic, 1: one launch chain)")
    ap.add_argument("--grid", type=int, default=0,
                    help="workgroups per launch of the headline form (0: the library's default)")
    ap.add_argument("--tile", type=int, default=-1,
                    help="tile variant of every replica of the headline form (-1: the library's default)")
    ap.add_argument("--taper", type=float, default=None, help="share taper of the headline form's plans")
    ap.add_argument("--barriers", choices=["grid", "team"], default=None, help="barriers of the persistent form")
    ap.add_argument("--form", choices=["persistent", "batched", "plain"], default="batched")
    ap.add_argument("--fmt", choices=["int8", "bitpack"], default="bitpack")
    ap.add_argument("--no-extras", action="store_true", help="skip the other forms and formats")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-aux", action="store_true", help="skip the layer-profile and host hand-over figures")
    ap.add_argument("--cpu-sweeps", type=int, default=10)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the batched-TI, uneven-autotuned and serving configurations")
    ap.add_argument("--serve-requests", type=int, default=100,
                    help="requests of the serving figure in the default run")
    ap.add_argument("--serve", type=int, default=0, metavar="N",
                    help="instead: the serving workload, N Poisson requests (20/s, log-uniform sizes)")
    ap.add_argument("--serve-budget-mib", type=int, default=256)
    ap.add_argument("--full-configs", action="store_true",
                    help="instead: every configuration at its full sweep count, one JSON line of rates")
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


def run_form(islf, torch, form, fmt, steps, warmup, chunk, n_reps=None, groups=0, reps=None, autotune=0, grid=0,
             tile=-1, min_warm_s=0.5, barriers=None, taper=None):
    """Times `steps` sweeps of a batch in one execution form: graph replays of
    `chunk` sweeps (plus eager sweeps for a remainder), after the warm-up:
    at least `warmup` sweeps, at least one untimed replay of the same graph,
    and untimed replays until `min_warm_s` seconds have passed (the GPU
    raises its clocks over the first fraction of a second of work).  HIP
    events on the context's stream bracket the timed region (the group
    streams fork from and join back to it inside it)."""
    mode = {"persistent": islf.EXEC_PERSISTENT, "batched": islf.EXEC_BATCHED, "plain": islf.EXEC_PLAIN}[form]
    f = {"int8": islf.INT8, "bitpack": islf.BITPACK}[fmt]
    reps = replicas(islf, n_reps) if reps is None else reps
    chunk = max(1, min(chunk, steps))
    n_warm = max(1, warmup // chunk)
    warm_rest = max(0, warmup - n_warm * chunk)
    ctx = islf.Context(reps, spin_format=f, obs_capacity=steps + chunk + 64, exec_mode=mode)
    try:
        tuned = 0.0
        if barriers is not None:
            ctx.set_barriers(barriers)
        if taper is not None:
            ctx.set_taper(taper)
        if autotune:
            t = time.perf_counter()
            ctx.autotune(autotune)
            tuned = time.perf_counter() - t
        if groups:
            ctx.set_groups(groups)
        if grid:
            ctx.set_grid(grid)
        if tile >= 0:
            for i in range(len(reps)):
                ctx.set_tile(i, tile)
        ctx.capture(chunk)
        # warm-up: always one untimed replay of the graph (the first replay of
        # a new graph is slower), eager sweeps for the remainder, then replays
        # until the clocks are up
        tw = time.perf_counter()
        ctx.replay(n_warm)
        if warm_rest:
            ctx.sweep(warm_rest)
        torch.cuda.synchronize()
        while time.perf_counter() - tw < min_warm_s:
            ctx.replay(1)
            n_warm += 1
            torch.cuda.synchronize()
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
        done = n_warm * chunk + warm_rest + steps
        for i in range(len(reps)):
            assert ctx.sweep_count(i) == done
        out = dict(ms_per_sweep=total_ms / steps, sweeps_per_launch=chunk, launches=n_launch,
                   warmup_sweeps=done - steps, groups=ctx.get_groups() if form == "batched" else 1,
                   grid=ctx.get_grid(), sites=sum(r.N for r in reps), ctx_means=None)
        if autotune:
            out["autotune_s"] = round(tuned, 2)
            out["tuned"] = {"groups": ctx.get_groups() if form == "batched" else 1, "grid": ctx.get_grid(),
                            "taper": ctx.get_taper(), "tiles": sorted({ctx.get_tile(i) for i in range(len(reps))})}
            if form == "persistent":
                out["tuned"]["barriers"] = "team" if ctx.get_barriers() == islf.BARRIER_TEAM else "grid"
        out["ctx_means"] = ctx.means(done - steps, steps)
        return out
    finally:
        ctx.close()


def rate(run):
    return run["sites"] / (run["ms_per_sweep"] * 1e6)


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


def committed_figure(path, key):
    """A machine-readable figure `key: value` from a committed counter
    summary, or None when the kernel code has changed since it was taken."""
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"kernel_code_sha256_16:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != kernel_code_hash():
        return None
    m = re.search(re.escape(key) + r":\s*([0-9.eE+-]+)", text)
    return float(m.group(1)) if m else None


def committed_traffic(fmt):
    """HBM bytes (FETCH_SIZE + WRITE_SIZE, copy-calibrated) per sweep-kernel
    launch of the one-launch-chain form (half a sweep of every replica)."""
    return committed_figure(PROFILE_TRAFFIC, f"traffic_bytes_per_launch[{fmt}]")


def committed_valu(fmt):
    """Counter-based VALU figures of the same launches: the share of the
    dispatch's SIMD issue slots that issued a VALU instruction
    (SQ_ACTIVE_INST_VALU over GRBM_GUI_ACTIVE cycles), the issue time of a
    launch's VALU instructions (quad-cycles over the 1024 SIMDs at 2.4 GHz)
    and VALU lane-ops per update."""
    f = committed_figure(PROFILE_VALU, f"valu_issue_frac[{fmt}]")
    if f is None:
        return None
    return {"issue_frac": f, "issue_us_per_launch": committed_figure(PROFILE_VALU, f"valu_issue_us_per_launch[{fmt}]"),
            "lane_ops_per_update": committed_figure(PROFILE_VALU, f"valu_lane_ops_per_update[{fmt}]"),
            "source": os.path.relpath(PROFILE_VALU, ROOT)}


def ti_replicas(islf):
    """The batched thermodynamic-integration batch: 64 replicas of
    40 x 120 x 120 along the surface-field path h1 = r/63, hn = -h1, T = 3."""
    return [islf.Replica(40, 120, 120, islf.GAPBC, J=1.0, beta=1.0 / 3.0, H=0.0, h1=r / 63.0, hn=-r / 63.0,
                         seed=SEED + r, replica=r, init=islf.INIT_RANDOM) for r in range(64)]


def uneven_replicas(islf):
    """96 replicas, round-robin over Lx in {20, 40, 80} x Ly = Lz in
    {64, 128, 256}, T in {2, 2.5, 3, 3.5, 4}, |h1| in {0.25, 0.5, 0.75}."""
    out = []
    for r in range(96):
        c = r % 9
        Lx = (20, 40, 80)[c // 3]
        L = (64, 128, 256)[c % 3]
        T = (2.0, 2.5, 3.0, 3.5, 4.0)[(r // 9) % 5]
        h = (0.25, 0.5, 0.75)[(r // 45) % 3]
        out.append(islf.Replica(Lx, L, L, islf.GAPBC, J=1.0, beta=1.0 / T, H=0.0, h1=h, hn=-h,
                                seed=SEED + 1000 + r, replica=r, init=islf.INIT_RANDOM))
    return out


def full_configs(islf, torch):
    """Every configuration at its full sweep count (graph replays of 50
    sweeps after 200 warm-up sweeps): the small film (1,000 sweeps), the
    paper-scale batch in every form and format (2,000), the batched TI batch
    (10^4) and the uneven batch (5,000), default and autotuned."""
    out = {}

    def run(name, *a, **k):
        r = run_form(islf, torch, *a, **k)
        out[name] = {"updates_per_ns": round(rate(r), 2), "ms_per_sweep": round(r["ms_per_sweep"], 6),
                     "groups": r["groups"], "grid": r["grid"]}
        if "tuned" in r:
            out[name]["tuned"] = r["tuned"]
        print("#", name, out[name], file=sys.stderr, flush=True)

    small = [islf.Replica(12, 24, 24, islf.GAPBC, J=1.0, beta=1.0 / 3.0, H=0.0, h1=0.5, hn=-0.5, seed=SEED,
                          replica=0, init=islf.INIT_RANDOM)]
    for fmt in ("int8", "bitpack"):
        run(f"film_12x24x24_plain_{fmt}", "plain", fmt, 1000, 50, 50, reps=small)
    for form in ("batched", "plain", "persistent"):
        for fmt in ("bitpack", "int8"):
            run(f"paper_scale_{form}_{fmt}", form, fmt, 2000, 200, 50)
    for fmt in ("bitpack", "int8"):
        run(f"ti_64_batched_{fmt}", "batched", fmt, 10000, 200, 50, reps=ti_replicas(islf))
        run(f"ti_64_batched_{fmt}_autotuned", "batched", fmt, 10000, 200, 50, reps=ti_replicas(islf), autotune=10)
        run(f"ti_64_persistent_{fmt}_autotuned", "persistent", fmt, 10000, 200, 50, reps=ti_replicas(islf),
            autotune=10)
    run("uneven_96_batched_int8_autotuned", "batched", "int8", 5000, 200, 50, reps=uneven_replicas(islf), autotune=10)
    run("uneven_96_batched_bitpack", "batched", "bitpack", 5000, 200, 50, reps=uneven_replicas(islf))
    return out


def config_figures(islf, torch, steps, warmup, chunk, serve_requests, serve_budget_mib):
    """The batched configurations beside the headline: updates/ns per form
    and format, the field-path integral of the TI batch, serving latency."""
    import numpy as np

    out = {}
    st, wu = min(steps, 100), min(warmup, 50)
    ti = {}
    for form, fmt in (("batched", "bitpack"), ("batched", "int8"), ("persistent", "bitpack"),
                      ("persistent", "int8")):
        r = run_form(islf, torch, form, fmt, st, wu, min(chunk, 50), reps=ti_replicas(islf), min_warm_s=0.2)
        ti[f"{form}_{fmt}"] = round(rate(r), 2)
        print(f"# TI batch {form}/{fmt}: { {k: v for k, v in r.items() if k != 'ctx_means'} }", file=sys.stderr,
              flush=True)
        if (form, fmt) == ("batched", "bitpack"):
            m = r["ctx_means"]
            h = np.arange(64) / 63.0
            cum = islf.integrate(h, m[:, 3], m[:, 4], -1.0, 1.0, 1.0 / (120 * 120))
            ti["delta_f1_at_h1_1"] = float(cum[-1])
    r = run_form(islf, torch, "persistent", "bitpack", st, wu, min(chunk, 50), reps=ti_replicas(islf),
                 min_warm_s=0.2, barriers=islf.BARRIER_TEAM)
    ti["persistent_bitpack_team_barriers"] = round(rate(r), 2)
    for form in ("batched", "persistent"):
        r = run_form(islf, torch, form, "bitpack", st, wu, min(chunk, 50), reps=ti_replicas(islf), autotune=10,
                     min_warm_s=0.2)
        ti[f"{form}_bitpack_autotuned"] = round(rate(r), 2)
        ti[f"{form}_bitpack_tuned"] = r.get("tuned")
        print(f"# TI batch {form}/bitpack autotuned: { {k: v for k, v in r.items() if k != 'ctx_means'} }",
              file=sys.stderr, flush=True)
    ti["workload"] = ("64 replicas of 40x120x120 GAPBC, T=3, h1=r/63, hn=-h1, seeds 14115588+r; "
                      f"timed over {st} sweeps; delta_f1 = trapezoid of -(m1 - mn) over h1 after the timed sweeps "
                      "(short chains: a throughput check, not a physics result)")
    out["ti_64x40x120x120"] = ti
    un = {}
    r = run_form(islf, torch, "batched", "int8", st, wu, min(chunk, 50), reps=uneven_replicas(islf), autotune=10,
                 min_warm_s=0.2)
    un["batched_int8_autotuned"] = round(rate(r), 2)
    un["autotune_s"] = r.get("autotune_s")
    un["tuned"] = r.get("tuned")
    print(f"# uneven batch int8 autotuned: { {k: v for k, v in r.items() if k != 'ctx_means'} }", file=sys.stderr,
          flush=True)
    r = run_form(islf, torch, "batched", "bitpack", st, wu, min(chunk, 50), reps=uneven_replicas(islf), min_warm_s=0.2)
    un["batched_bitpack"] = round(rate(r), 2)
    un["workload"] = (f"96 replicas, Lx in {{20,40,80}} x Ly=Lz in {{64,128,256}}, T in {{2,2.5,3,3.5,4}}, "
                      f"|h1| in {{0.25,0.5,0.75}}, 125,583,360 sites; timed over {st} sweeps")
    out["uneven_96"] = un
    if serve_requests:
        from paper_1411_5588_amd import serving
        reqs = serving.poisson_workload(serve_requests, rate=20.0)
        srv = serving.Server(budget_bytes=serve_budget_mib << 20, max_slots=64, spin_format=islf.BITPACK,
                             max_step=50, obs_capacity=5000, realtime=True)
        try:
            srv.run(reqs)
        finally:
            srv.close()
        sm = serving.summary(reqs, srv.wall_s, srv.busy_s)
        out["serving"] = {k: round(v, 4) for k, v in sm.items()}
        out["serving"]["workload"] = (f"{serve_requests} requests, Poisson 20/s, sites log-uniform on [1e5, 4.6e7], "
                                      f"T~U[2,4.2], h1~U[0.1,1], hn=-h1, sweeps~U{{500..5000}}, bit-packed, "
                                      f"memory budget {serve_budget_mib} MiB, at most 64 slots")
        print(f"# serving: {out['serving']}", file=sys.stderr, flush=True)
    return out


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

    if args.full_configs:
        print(json.dumps({"metric": "spin updates/ns", "full_configs": full_configs(islf, torch),
                          "data": "synthetic"}), flush=True)
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

    def brief(r):
        return {k: v for k, v in r.items() if k != "ctx_means"}

    WARM_S = args.min_warmup_s
    bars = None if args.barriers is None else (islf.BARRIER_TEAM if args.barriers == "team" else islf.BARRIER_GRID)
    main_run = run_form(islf, torch, args.form, args.fmt, args.steps, args.warmup, args.chunk, groups=args.groups,
                        grid=args.grid, tile=args.tile, min_warm_s=WARM_S, barriers=bars, taper=args.taper)
    print(f"# {args.form}/{args.fmt}: {brief(main_run)}", file=sys.stderr, flush=True)
    value = rate(main_run)
    # the same form as one launch chain over all replicas, timed the same way:
    # its launches run one after another, so timed region / launches is the
    # sweep kernel's own average launch duration
    if main_run["groups"] == 1:
        chain_run = main_run
    else:
        chain_run = run_form(islf, torch, args.form, args.fmt, min(args.steps, 400), min(args.warmup, 100),
                             args.chunk, groups=1, tile=args.tile, min_warm_s=WARM_S)
        print(f"# {args.form}/{args.fmt} one launch chain: {brief(chain_run)}", file=sys.stderr, flush=True)

    forms = {}
    if not args.no_extras:
        other = "int8" if args.fmt == "bitpack" else "bitpack"
        for form, fmt in (("batched", other), ("plain", "bitpack"), ("plain", "int8"), ("persistent", "bitpack"),
                          ("persistent", "int8")):
            if (form, fmt) == (args.form, args.fmt):
                continue
            r = run_form(islf, torch, form, fmt, min(args.steps, 100), min(args.warmup, 50), min(args.chunk, 50),
                         min_warm_s=0.2)
            forms[f"{form}_{fmt}"] = round(rate(r), 2)
            print(f"# {form}/{fmt}: {brief(r)}", file=sys.stderr, flush=True)
        r = run_form(islf, torch, "persistent", "bitpack", min(args.steps, 100), min(args.warmup, 50),
                     min(args.chunk, 50), min_warm_s=0.2, barriers=islf.BARRIER_TEAM)
        forms["persistent_bitpack_team_barriers"] = round(rate(r), 2)
        print(f"# persistent/bitpack team barriers: {brief(r)}", file=sys.stderr, flush=True)
        # a batch larger than the 256 MB last-level cache: 8 int8 replicas, 369 MB of spins
        r = run_form(islf, torch, "batched", "int8", min(args.steps, 50), min(args.warmup, 50), min(args.chunk, 50),
                     n_reps=8, min_warm_s=0.2)
        forms["batched_int8_8x46M_369MB"] = round(rate(r), 2)
        print(f"# batched/int8 x8: {brief(r)}", file=sys.stderr, flush=True)

    configs = None
    if not args.no_configs:
        configs = config_figures(islf, torch, args.steps, args.warmup, args.chunk, args.serve_requests,
                                 args.serve_budget_mib)

    # dominant kernel: the sweep kernel.  Its A and B launches of one sweep
    # together update every site of every replica once (A: phase 0 and the
    # previous sweep's phase 3, B: phases 1 and 2), so one launch updates half
    # a sweep of every replica; the one-chain timed region over its 2 x steps
    # launches is the average launch duration (the region also holds one
    # closing launch and fold per graph launch, so this slightly overstates it)
    def roofline_of(fmt, chain, grouped):
        bpu = BYTES_PER_UPDATE[fmt]
        alg_bytes = bpu * n_reps * N / 2
        launch_ms = chain["ms_per_sweep"] / 2
        achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": committed_traffic(fmt),
               "kernel": "k_sweep (A and B launches), one launch over all three replicas",
               "launch_ms": round(launch_ms, 5), "workgroups": chain["grid"],
               "algorithmic_bytes_per_launch": alg_bytes, "bytes_per_update": bpu,
               "roofline_updates_per_ns": HBM_PEAK_GBS / bpu}
        if grouped is not None:
            wave_ms = grouped["ms_per_sweep"] / 2
            gbs = alg_bytes / (wave_ms * 1e-3) / 1e9
            out["grouped_wave"] = {"wave_ms": round(wave_ms, 5), "achieved": round(gbs, 1),
                                   "frac": round(gbs / HBM_PEAK_GBS, 4),
                                   "unit": f"wave of {grouped['groups']} concurrent group dispatches of "
                                           f"{grouped['grid']} workgroups, half a sweep of every replica"}
        out["valu"] = committed_valu(fmt)
        if grouped is not None and out["valu"] and out["valu"].get("issue_us_per_launch"):
            # the same half sweep's VALU issue time over the grouped wave: the
            # share of the wave the SIMDs spend issuing VALU instructions
            out["grouped_wave"]["valu_issue_frac"] = round(
                out["valu"]["issue_us_per_launch"] / (out["grouped_wave"]["wave_ms"] * 1e3), 3)
        out["limiter"] = "VALU issue: Philox4x32-10 costs 5 64-bit products and 5 xors per update"
        return out

    roofline = roofline_of(args.fmt, chain_run, main_run if args.form == "batched" else None)
    roofline["grouped_wave_is_headline_form"] = args.form == "batched"
    if not args.no_extras:
        # the other spin format's sweep kernel, measured the same way
        other = "int8" if args.fmt == "bitpack" else "bitpack"
        oc = run_form(islf, torch, "batched", other, min(args.steps, 400), min(args.warmup, 100), args.chunk,
                      groups=1, min_warm_s=0.2)
        og = run_form(islf, torch, "batched", other, min(args.steps, 400), min(args.warmup, 100), args.chunk,
                      min_warm_s=0.2)
        roofline[f"other_format_{other}"] = roofline_of(other, oc, og)
        roofline[f"other_format_{other}"]["updates_per_ns_batched"] = round(rate(og), 2)
        print(f"# {other} one chain: {brief(oc)}; grouped: {brief(og)}", file=sys.stderr, flush=True)

    prof = hio = None
    if not args.no_aux:
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
                   "groups": main_run["groups"], "workgroups_per_launch": main_run["grid"],
                   "warmup_sweeps_run": main_run["warmup_sweeps"]},
        "roofline": roofline,
        "forms": forms,
        "configs": configs,
        "layer_profile": prof,
        "host_io": hio,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
