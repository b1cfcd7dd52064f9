"""Benchmark of the parallel event-chain sweep on one MI355X.

One step = one full PEC sweep (rebin, four colour phases of simulation-cell
kernels, tallies) of the 1,048,576-disk system at eta = 0.72 in 64 x 64
simulation cells, chain length 20 sigma, isotropic directions, FP64, starting
from the lattice.  The metric is EC collisions (lifts) per second; sweeps per
second and the whole-sweep fraction of HBM bandwidth are reported beside it.

With --workload start-rules it runs the negative control of Sec. 3.4 (Fig. 2-3)
instead: 8 systems with start disks drawn with replacement and 8 with a
shuffled list of distinct disks (N = 16384, eta = 0.70, 16 x 16 cells, seeds
1-8 each), batched, and reports the EC pressure of each rule (mean and
standard error over the seeds) and their difference in units of the combined
error.

With --workload nm-scan it compares the pressure against n_m for both start
rules (Fig. 3 right); --workload serial-ref compares PEC with serial EC of
the same N.

With --workload boundary-rules it compares reflection with rejection at the
cell boundary, each with both start rules (Fig. 3).

With --workload psi6-delaunay it times the Delaunay-neighbour Psi at N = 1M;
with --workload tau it reports the autocorrelation time (eq. tau) of 8
seeded liquid systems from a Psi series.

With --workload batch64 it times the batched form instead: the 64-system
ensemble (N log-uniform in [4096, 262144], eta uniform in [0.30, 0.72], about
64 disks per cell) advanced by shared launches, with the autotuned schedule
and one HIP graph per sweep; the line reports aggregate lifts per second and
the speed-up over running the same sweeps system by system.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                       [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from tests import inputs  # noqa: E402  (seeded workload definitions; no method arithmetic)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VECTOR_PEAK_TF = 78.6     # MI355X FP64 vector, TFLOP/s
# FP64 work of one lift (algorithmic): contact tests of the disks in the
# 3 x 3 neighbourhood of sigma-sized squares (about 8 disks at rho sigma^2 =
# 0.92; 2 sub, 2 mul + 2 fma for r.d and r x d, 1 fma, sqrt, sub = 12 flop
# each) plus the commit (2 fma) = 8 * 12 + 4 = 100 flop.
FLOP_PER_LIFT = 100.0
# HBM bytes per disk of the two rebin kernels (algorithmic): the count kernel
# reads x, y and writes the cell index and the region (one byte); the scatter
# kernel reads both and writes the id into its cell's list.
COUNT_BYTES_PER_DISK = 16 + 4 + 1
SCATTER_BYTES_PER_DISK = 4 + 1 + 4
# simulation cells that can run at once on the chip: one wavefront per SIMD
# (256 CUs x 4 SIMDs), and a 64 x 64 grid admits at most 1024 non-adjacent cells
CONCURRENT_CELLS = 1024
CLOCK_GHZ = 2.4
# HBM bytes of one chain draw: start index (4) and direction (16), written by
# the draw kernel and read by the simulation-cell kernel.
CHAIN_DRAW_BYTES = 4 + 16


def cell_kernel_bytes(n, eta, cells, chains):
    """Algorithmic HBM bytes of one launch of the simulation-cell kernel
    (all four colour phases of one sweep): every disk read once as its own
    (id 4 + position 16) and written back (16), the frozen band -- the disks
    within sigma outside a cell, a fraction ((w + 2 sigma)^2 - w^2) / w^2 of
    all disks -- read again (id + position), and the chain draws read."""
    w = math.sqrt(n * math.pi / (4.0 * eta)) / cells
    band = ((w + 2.0) ** 2 - w * w) / (w * w)
    return (20 + 16 + 20 * band) * n + CHAIN_DRAW_BYTES * chains


def sweep_bytes(n, eta, cells, chains):
    """Algorithmic HBM bytes of a whole sweep: the rebin kernels, the chain
    draws written, and the simulation-cell kernel."""
    return ((COUNT_BYTES_PER_DISK + SCATTER_BYTES_PER_DISK) * n + CHAIN_DRAW_BYTES * chains
            + cell_kernel_bytes(n, eta, cells, chains))


SCHEDULE_FLAGS = {"auto": lambda P: 0,
                  "one-launch": lambda P: P.EC_FLAG_ONE_LAUNCH,
                  "phase-launches": lambda P: P.EC_FLAG_PHASE_LAUNCHES}


def _kernel_source_sha():
    import hashlib
    src = os.path.join(ROOT, "paper_1409_6948_amd", "csrc", "ec_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def _profile_line(name, key):
    """key=value fields of the machine-readable line `key:` of a committed
    profile summary, or None when the file is missing or was taken on another
    kernel source."""
    import re
    prof = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(prof):
        return None
    sha = _kernel_source_sha()
    for line in open(prof):
        if line.startswith(key + ":"):
            f = dict(re.findall(r"(\w+)=(\S+)", line))
            if f.get("source_sha256_prefix") == sha:
                return f
    return None


def measured_traffic(kernel, workload):
    """HBM bytes per launch of the simulation-cell kernel from the committed
    counter summary, or None when the kernel source has changed since the
    counters were taken."""
    f = _profile_line(f"{kernel}_{workload}_counters.md", "traffic")
    if f is None:
        return None
    return float(f["read_bytes_per_launch"]) + float(f["write_bytes_per_launch"])


def measured_cycles_per_event(kernel, workload):
    """Wavefront cycles per event of the simulation-cell kernel from the
    committed SQ counters (same kernel source), or None."""
    f = _profile_line(f"{kernel}_{workload}_sq_counters.md", "tstep")
    return None if f is None else float(f["cycles_per_event"])


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, threads=None):
    """The oracle in its phase-parallel mode (the paper's own scheme: one
    thread per simulation cell of the running colour, Sec. 3.4) on the host's
    cores: one whole sweep of the workload from the lattice -- rebin, the four
    colour phases, write-back -- or, above 4M disks, the first colour phase of
    that sweep (a quarter of the cells)."""
    from oracle import oracle as O
    from oracle import build as OB
    threads = threads or max(1, min(16, os.cpu_count() or 1))
    p = O.params(w["n"], w["eta"], w["ell"], w["cells"], dir_mode=O.DIR_ISO, seed=w["seed"])
    st = O.State(p)
    whole = w["n"] <= (1 << 22)
    O.set_threads(threads)
    try:
        t0 = time.perf_counter()
        if whole:
            st.run(1)
        else:
            C = w["cells"]
            perm = O.sweep_draws(p, 0)[2]
            first = [c for c in range(C * C) if ((c % C) & 1) | (((c // C) & 1) << 1) == perm[0]]
            st.run_cells(0, first, n_phases=1)
        secs = time.perf_counter() - t0
    finally:
        O.set_threads(1)
    lifts = int(st.acc_cnt[:, O.CNT_LIFTS].sum())
    what = "one whole sweep" if whole else "the first colour phase of sweep 0"
    return {"value": lifts / secs, "unit": "lifts/s", "cores": threads, "kind": "oracle",
            "sample": f"{what} of {w['n']} disks from the lattice: {lifts} lifts in {secs:.1f} s, "
                      f"rebin and staging included; phase-parallel oracle on {threads} threads",
            "host": {"nproc": os.cpu_count(), "cpu_model": _cpu_model(),
                     "compiler": "gcc " + " ".join(OB.FLAGS)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="pec_1m")
    ap.add_argument("--cells-per-block", type=int, default=0)
    ap.add_argument("--schedule", choices=("auto", "one-launch", "phase-launches"), default="auto",
                    help="all four colour phases of a sweep in one launch with per-cell "
                         "dependencies, or one launch per phase; auto = the library's default "
                         "(one launch for a system alone, a ready queue for a batch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=("fp64", "fp32-screen"), default=None,
                    help="fp32-screen: FP32 screening of candidates, FP64 for the survivors "
                         "and every commit (identical events); default: the workload's own "
                         "(FP64 for pec_1m, FP32 screen for pec_16m and batch64)")
    ap.add_argument("--other-precision", action="store_true",
                    help="walled cells: also run the same sweeps from the same start in the "
                         "other precision (FP64 or FP32 screen), compare the per-sweep digests "
                         "and report its time")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU "
              f"decomposition is described, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1409_6948_amd as P

    if args.workload == "batch64":
        return bench_batch(args, torch, P)
    if args.workload == "start-rules":
        return bench_start_rules(args, torch, P)
    if args.workload == "boundary-rules":
        return bench_boundary_rules(args, torch, P)
    if args.workload == "serial-ref":
        return bench_serial_ref(args, torch, P)
    if args.workload == "nm-scan":
        return bench_nm_scan(args, torch, P)
    if args.workload == "psi6-delaunay":
        return bench_psi6_delaunay(args, torch, P)
    if args.workload == "tau":
        return bench_tau(args, torch, P)
    w = dict(inputs.WORKLOADS[args.workload])
    torch.cuda.set_device(0)
    precision = args.precision or w.get("precision", "fp64")
    prec = P.EC_PREC_FP64 if precision == "fp64" else P.EC_PREC_FP32_SCREEN
    flags = SCHEDULE_FLAGS[args.schedule](P)
    kernel = "k_phase" if args.schedule == "phase-launches" else "k_sweep_cells"
    if w["cells"] == 1:
        # one periodic cell: N serial chains in one wavefront, on the bin grid
        # where the box holds at least 12 bins below 0.7 sigma per side (the
        # library's rule; the label only names the kernel that is timed)
        box = math.sqrt(w["n"] * math.pi / (4.0 * w["eta"]))
        kernel = "k_periodic_bins" if math.floor(box / 0.7) + 1 >= 12 else "k_periodic"
    p = P.make_params(w["n"], w["eta"], w["ell"], w["cells"], dir_mode=w["dir_mode"],
                      seed=w["seed"], cells_per_block=args.cells_per_block, precision=prec,
                      flags=flags)
    g = P.System(p, device="cuda:0")
    if args.copy_probe_mb > 0:
        nbytes = args.copy_probe_mb << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy probe: {nbytes} bytes read and written", file=sys.stderr, flush=True)
        del src, dst
    print(f"# workload {args.workload} ({precision}): warmup {args.warmup} sweeps", file=sys.stderr,
          flush=True)
    g.sweep(args.warmup)
    torch.cuda.synchronize()
    g.reset_tallies()
    # the library records HIP events around its kernels on its own stream and
    # reads them after the timed region: the sweeps run free, back to back
    g.set_timing(True)
    stream = g.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    print(f"# timing {args.steps} sweeps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    e0.record(stream)
    g.sweep(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    phase_ms, launches = g.get_timing()
    count_ms, scatter_ms, rebins = g.get_rebin_timing()
    g.set_timing(False)
    z, bp, counts = g.measure_pressure()
    digests = g.get_digests(args.warmup + args.steps) if args.warmup + args.steps <= 1024 else None
    psi = None
    if w.get("psi6"):
        psi6, nb = g.measure_psi6()
        psi = {"abs": abs(psi6), "re": psi6.real, "im": psi6.imag, "mean_neighbours": nb,
               "neighbours": "disks within 1.4 sigma"}
    secs = gpu_ms / 1e3
    lifts = counts["lifts"]
    events = counts["lifts"] + counts["frozen"] + counts["walls"] + counts["chains"]
    value = lifts / secs
    sweeps_s = args.steps / secs
    chains_per_sweep = counts["chains"] / args.steps
    hbm_frac = (sweep_bytes(w["n"], w["eta"], w["cells"], chains_per_sweep) * sweeps_s
                / (HBM_PEAK_GBS * 1e9))
    avg_launch_s = phase_ms / 1e3 / max(launches, 1)
    # algorithmic FP64 work per launch: 100 flop per lift, the lifts of the
    # timed sweeps spread over the launches
    flop_per_launch = FLOP_PER_LIFT * lifts / max(launches, 1)
    achieved_tf = flop_per_launch / avg_launch_s / 1e12
    traffic = measured_traffic(kernel, args.workload)
    # latency bound of the one-wave-per-cell design: at most CONCURRENT_CELLS
    # cells run at once, each an event after the other
    cyc = measured_cycles_per_event(kernel, args.workload)
    latency = None
    if cyc is not None:
        t_step = cyc / (CLOCK_GHZ * 1e9)
        bound = CONCURRENT_CELLS / t_step * lifts / events
        latency = {"cycles_per_event": cyc, "t_step_us": t_step * 1e6,
                   "concurrent_cells": CONCURRENT_CELLS, "lifts_per_s_bound": bound,
                   "frac": value / bound, "source": f"profiles/{kernel}_{args.workload}_sq_counters.md"}
    rebin = None
    if rebins > 0:
        c_s, s_s = count_ms / 1e3 / rebins, scatter_ms / 1e3 / rebins
        rebin = {"k_count": {"avg_ms": c_s * 1e3, "bytes": COUNT_BYTES_PER_DISK * w["n"],
                             "gb_s": COUNT_BYTES_PER_DISK * w["n"] / c_s / 1e9,
                             "hbm_frac": COUNT_BYTES_PER_DISK * w["n"] / c_s / (HBM_PEAK_GBS * 1e9)},
                 "k_scatter": {"avg_ms": s_s * 1e3, "bytes": SCATTER_BYTES_PER_DISK * w["n"],
                               "gb_s": SCATTER_BYTES_PER_DISK * w["n"] / s_s / 1e9,
                               "hbm_frac": SCATTER_BYTES_PER_DISK * w["n"] / s_s / (HBM_PEAK_GBS * 1e9)}}
    line = {
        "metric": "EC collisions (lifts)/sec, 1 MI355X, " + w["label"],
        "value": value,
        "unit": "lifts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32-screen+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_disks": w["n"], "eta": w["eta"],
                   "cells_per_side": w["cells"], "ell": w["ell"],
                   "directions": "isotropic" if w["dir_mode"] == 1 else "+x/+y alternating",
                   "precision": precision,
                   "schedule": {"k_phase": "phase-launches", "k_periodic": "one periodic cell",
                                "k_periodic_bins": "one periodic cell"}.get(
                       kernel, "one-launch"),
                   "start": "lattice",
                   "sweeps_before_timing": args.warmup},
        "sweeps_per_s": sweeps_s,
        "events_per_s": events / secs,
        "counts": counts,
        "z_timed_sweeps": z,
        "beta_p_sigma2_timed_sweeps": bp,
        "psi6": psi,
        "hbm_frac_whole_sweep": hbm_frac,
        "wall_s": wall,
        "roofline": {"bound": "alu", "kernel": kernel, "achieved": achieved_tf,
                     "peak": FP64_VECTOR_PEAK_TF, "unit": "TFLOP/s",
                     "frac": achieved_tf / FP64_VECTOR_PEAK_TF,
                     "traffic": traffic,
                     "traffic_over_algorithmic": (
                         traffic / cell_kernel_bytes(w["n"], w["eta"], w["cells"], chains_per_sweep)
                         if traffic is not None and kernel == "k_sweep_cells" else None),
                     "flop_per_lift": FLOP_PER_LIFT,
                     "lifts_per_launch": lifts / max(launches, 1),
                     "avg_launch_ms": avg_launch_s * 1e3, "launches": launches,
                     "kernel_share_of_sweep": phase_ms / gpu_ms},
        "latency_bound": latency,
        "rebin": rebin,
    }
    if w["cells"] > 1 and args.other_precision and digests is not None:
        # the same sweeps from the same start in the other form; identical
        # collision sequences give identical per-sweep digests
        g.close()
        other = "fp64" if precision == "fp32-screen" else "fp32-screen"
        po = P.make_params(w["n"], w["eta"], w["ell"], w["cells"], dir_mode=w["dir_mode"],
                           seed=w["seed"], cells_per_block=args.cells_per_block,
                           precision=P.EC_PREC_FP64 if other == "fp64" else P.EC_PREC_FP32_SCREEN,
                           flags=flags)
        print(f"# the same sweeps in {other}", file=sys.stderr, flush=True)
        go = P.System(po, device="cuda:0")
        go.sweep(args.warmup)
        torch.cuda.synchronize()
        go.reset_tallies()
        f0 = torch.cuda.Event(enable_timing=True)
        f1 = torch.cuda.Event(enable_timing=True)
        f0.record(go.stream)
        go.sweep(args.steps)
        f1.record(go.stream)
        torch.cuda.synchronize()
        ms_o = f0.elapsed_time(f1) / args.steps
        dig_o = go.get_digests(args.warmup + args.steps)
        _, _, counts_o = go.measure_pressure()
        go.close()
        line["other_precision"] = {
            "precision": other, "ms_per_step": ms_o,
            "value": counts_o["lifts"] / (ms_o * args.steps / 1e3),
            "sweeps_compared": args.warmup + args.steps,
            "digests_identical": bool(np.array_equal(digests, dig_o)),
            "speedup_of_this_precision": ms_o / (gpu_ms / args.steps)}
    if not args.no_cpu_baseline:
        print("# CPU oracle baseline (phase-parallel)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


def _batch_run(P, torch, ps, args, schedule_tune=True):
    """Build the batch, autotune its schedule, warm up, time args.steps sweeps;
    returns (lifts/s, events/s, ms/sweep, digests of every system, tuning)."""
    b = P.Batch(ps)
    b.sweep(1)
    tuned = b.autotune(trial_sweeps=2) if schedule_tune else None
    b.set_graph(True)
    b.sweep(max(args.warmup - 1, 0))
    b.stream.synchronize()
    for s in b.systems:
        s.reset_tallies()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.sweep(args.steps)
    e1.record(b.stream)
    b.stream.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    lifts = events = 0
    digs = []
    for s in b.systems:
        _, _, c = s.measure_pressure()
        lifts += c["lifts"]
        events += c["lifts"] + c["frozen"] + c["walls"] + c["chains"]
        digs.append(s.get_digests(args.steps))
    b.close()
    return lifts / secs, events / secs, secs * 1e3 / args.steps, digs, tuned


def bench_batch(args, torch, P):
    """Aggregate lifts/s of the 64-system ensemble in the batched form, in the
    requested precision (default: FP32 screening with FP64 commits), the same
    sweeps in the other precision (digests compared system by system), and the
    same sweeps run system by system (solo launches, one after another)."""
    cfgs = inputs.batch_systems(64, seed=0)
    flags = SCHEDULE_FLAGS[args.schedule](P)
    precision = args.precision or "fp32-screen"
    other = "fp64" if precision == "fp32-screen" else "fp32-screen"
    code = {"fp64": P.EC_PREC_FP64, "fp32-screen": P.EC_PREC_FP32_SCREEN}

    def params(prec):
        return [P.make_params(c["n"], c["eta"], c["ell"], c["cells"], dir_mode=c["dir_mode"],
                              seed=c["seed"], system=i, flags=flags, precision=code[prec])
                for i, c in enumerate(cfgs)]

    torch.cuda.set_device(0)
    ps = params(precision)
    print(f"# batch64: {len(ps)} systems, sum N = {sum(c['n'] for c in cfgs)}, {precision}",
          file=sys.stderr, flush=True)
    value, ev_s, ms, digs, (sched, cpb, trials) = _batch_run(P, torch, ps, args)
    print(f"# batch64: {other} for the same sweeps", file=sys.stderr, flush=True)
    value_o, _, ms_o, digs_o, _ = _batch_run(P, torch, params(other), args)
    same = all(np.array_equal(a, b) for a, b in zip(digs, digs_o))
    # the same sweeps, system by system
    print("# batch64: solo runs", file=sys.stderr, flush=True)
    solo_secs = 0.0
    st = torch.cuda.Stream()
    for p in ps:
        g = P.System(p, stream=st)
        g.sweep(args.warmup)
        st.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(st)
        g.sweep(args.steps)
        t1.record(st)
        st.synchronize()
        solo_secs += t0.elapsed_time(t1) / 1e3
        g.close()
    line = {
        "metric": "EC collisions (lifts)/sec, 1 MI355X, 64-system batch (aggregate)",
        "value": value,
        "unit": "lifts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32-screen+f64",
        "data": "synthetic",
        "config": {"workload": "batch64", "n_systems": len(ps),
                   "sum_n": int(sum(c["n"] for c in cfgs)), "eta_range": [0.30, 0.72],
                   "ell": 20.0, "precision": precision, "schedule": sched, "cells_per_block": cpb,
                   "hip_graph": True},
        "events_per_s": ev_s,
        "autotune_trial_ms": trials,
        "other_precision": {"precision": other, "value": value_o, "ms_per_step": ms_o,
                            "digests_identical": same,
                            "speedup_of_this_precision": ms_o / ms},
        "solo_sequential_s": solo_secs,
        "speedup_vs_solo_sequential": solo_secs / (ms * args.steps / 1e3),
    }
    print(json.dumps(line), flush=True)


def bench_start_rules(args, torch, P):
    """Negative control: pressure with starts drawn with replacement (the
    correct rule, Fig. 2) against shuffled distinct starts (Fig. 3), n_m = n_c.
    Both pressure routes are reported: the lift tallies (eq. EC pressure) and
    g(r) extrapolated to contact (eq. pressure), the route of Fig. 3."""
    import math
    n, eta, C, ell, sigma = 16384, 0.70, 16, 20.0, 1.0
    r_max, n_bins, fit = 1.5, 100, 0.05
    box = math.sqrt(n * math.pi * sigma * sigma / (4.0 * eta))
    ps = []
    for rule in (P.EC_START_REPLACE, P.EC_START_DISTINCT):
        for seed in range(1, 9):
            ps.append(P.make_params(n, eta, ell, C, seed=seed, start_mode=rule, system=len(ps)))
    b = P.Batch(ps)
    b.set_graph(True)
    b.sweep(args.warmup)
    b.stream.synchronize()
    for s in b.systems:
        s.reset_tallies()
        s.gr_reset()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.sweep(1)
        for s in b.systems:
            s.gr_accumulate(r_max, n_bins)
    b.stream.synchronize()
    secs = time.perf_counter() - t0
    z_ec, z_gr = [], []
    for s in b.systems:
        z_ec.append(s.measure_pressure()[0])
        counts, samples, _ = s.gr_counts()
        z_gr.append(P.gr_normalize(n, box, sigma, r_max, counts, samples, fit)[3])

    def stats(v):
        m = sum(v) / len(v)
        return m, math.sqrt(sum((x - m) ** 2 for x in v) / (len(v) - 1) / len(v))

    out, diffs = {}, {}
    for route, zs in (("ec", z_ec), ("gr_contact", z_gr)):
        out[route] = {}
        for name, part in (("replacement", zs[:8]), ("distinct", zs[8:])):
            m, se = stats(part)
            out[route][name] = {"z_mean": m, "z_stderr": se, "z_per_seed": part}
        d = out[route]["distinct"]["z_mean"] - out[route]["replacement"]["z_mean"]
        comb = math.hypot(out[route]["distinct"]["z_stderr"], out[route]["replacement"]["z_stderr"])
        diffs[route] = {"z_difference": d, "in_combined_stderr": d / comb if comb > 0 else None}
    line = {"workload": "start-rules", "n_disks": n, "eta": eta, "cells_per_side": C, "ell": ell,
            "warmup": args.warmup, "sweeps": args.steps, "seconds": secs, "routes": out,
            "distinct_minus_replacement": diffs}
    print(json.dumps(line), flush=True)

def bench_psi6_delaunay(args, torch, P):
    """Psi with Delaunay neighbours (eq. Psi) on the 1M-disk workload after one
    sweep: time of one measurement (rebin, neighbour kernel, reduction, result
    copy) with HIP events on the system's stream."""
    w = dict(inputs.WORKLOADS["pec_1m"])
    g = P.System(P.make_params(w["n"], w["eta"], w["ell"], w["cells"], dir_mode=w["dir_mode"],
                               seed=w["seed"]), device="cuda:0")
    g.sweep(1)
    g.measure_psi6_delaunay()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = max(args.steps, 1)
    e0.record(g.stream)
    for _ in range(reps):
        psi, nb = g.measure_psi6_delaunay()
    e1.record(g.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    line = {"workload": "psi6-delaunay", "n_disks": w["n"], "eta": w["eta"], "measurements": reps,
            "ms_per_measurement": ms, "disks_per_s": w["n"] / (ms / 1e3),
            "psi_abs": abs(psi), "mean_neighbours": nb}
    print(json.dumps(line), flush=True)


def bench_tau(args, torch, P):
    """The autocorrelation time tau of eq. (tau) in sweeps: 8 seeded liquid
    systems (N = 16384, eta = 0.60, 16 x 16 cells) in one batch, Psi with
    Delaunay neighbours after every sweep of the series."""
    n, eta, C, seeds = 16384, 0.60, 16, 8
    warm, series = max(args.warmup, 1) * 10, max(args.steps, 20) * 10
    ps = [P.make_params(n, eta, 20.0, C, seed=sd + 1, system=sd) for sd in range(seeds)]
    b = P.Batch(ps)
    b.set_graph(True)
    b.sweep(warm)
    psis = np.zeros((seeds, series), dtype=np.complex128)
    for t in range(series):
        b.sweep(1)
        for i, sy in enumerate(b.systems):
            psis[i, t] = sy.measure_psi6_delaunay()[0]
    b.close()
    out = [P.psi_autocorrelation(psis[i], min(60, series - 1)) for i in range(seeds)]
    line = {"workload": "tau", "n_disks": n, "eta": eta, "cells_per_side": C, "ell": 20.0,
            "seeds": seeds, "warmup_sweeps": warm, "series_sweeps": series,
            "tau_sweeps_per_seed": [t for _, t in out],
            "c_lag1_per_seed": [float(c[1]) for c, _ in out],
            "psi_abs_mean": float(np.mean(np.abs(psis)))}
    print(json.dumps(line), flush=True)

def _z_routes(P, sysm, n, box, r_max=1.5, n_bins=100, fit=0.05):
    counts, samples, _ = sysm.gr_counts()
    return sysm.measure_pressure()[0], P.gr_normalize(n, box, 1.0, r_max, counts, samples, fit)[3]


def bench_serial_ref(args, torch, P):
    """PEC against serial EC in one periodic cell of the same N (the exact
    reference): N = 256, eta = 0.70, 4 x 4 cells (16 disks each), both start
    rules at n_m = 1, 4, 16, 16 seeds per case, both pressure routes.  Every
    case runs about the same number of chains: 16 / n_m times as many sweeps
    as n_m = 16."""
    import math
    n, eta, ell, seeds = 256, 0.70, 20.0, 16
    box = math.sqrt(n * math.pi / (4.0 * eta))
    base_warm, base_sweeps = max(args.warmup, 1) * 2, max(args.steps, 1) * 5

    def stats(v):
        m = sum(v) / len(v)
        return m, math.sqrt(sum((x - m) ** 2 for x in v) / (len(v) - 1) / len(v))

    t0 = time.perf_counter()
    # serial reference: one periodic cell, every disk starts one chain per sweep
    serial = []
    for sd in range(seeds):
        st = torch.cuda.Stream()
        g = P.System(P.make_params(n, eta, ell, 1, dir_mode=P.EC_DIR_ISOTROPIC, seed=sd + 1), stream=st)
        serial.append(g)
    for g in serial:
        g.sweep(base_warm)
    torch.cuda.synchronize()
    for g in serial:
        g.reset_tallies()
        g.gr_reset()
    for t in range(base_sweeps):
        for g in serial:
            g.sweep(1)
            g.gr_accumulate(1.5, 100)
        if t % 50 == 49:
            torch.cuda.synchronize()
            print(f"# serial-ref: serial sweep {t + 1} ({time.perf_counter() - t0:.1f} s)",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    zs = [_z_routes(P, g, n, box) for g in serial]
    ref = {"ec": stats([z[0] for z in zs]), "gr_contact": stats([z[1] for z in zs])}
    print(f"# serial-ref: serial reference done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
          flush=True)
    cases = []
    for nm in (1, 4, 16):
        scale = 16 // nm
        ps = []
        for rule in (P.EC_START_REPLACE, P.EC_START_DISTINCT):
            for sd in range(seeds):
                ps.append(P.make_params(n, eta, ell, 4, seed=sd + 1, chains_per_cell=nm, start_mode=rule,
                                        system=len(ps)))
        b = P.Batch(ps)
        b.set_graph(True)
        b.sweep(base_warm * scale)
        b.stream.synchronize()
        for sy in b.systems:
            sy.reset_tallies()
            sy.gr_reset()
        for _ in range(base_sweeps * scale):
            b.sweep(1)
            for sy in b.systems:
                sy.gr_accumulate(1.5, 100)
        b.stream.synchronize()
        zs = [_z_routes(P, sy, n, box) for sy in b.systems]
        b.close()
        for r, rule in enumerate(("replacement", "distinct")):
            part = zs[r * seeds:(r + 1) * seeds]
            c = {"n_m": nm, "rule": rule, "sweeps": base_sweeps * scale}
            for k, route in enumerate(("ec", "gr_contact")):
                m, se = stats([z[k] for z in part])
                rm, rse = ref[route]
                c[route] = {"z_mean": m, "z_stderr": se,
                            "minus_serial_in_stderr": (m - rm) / math.hypot(se, rse)}
            cases.append(c)
        print(f"# serial-ref: n_m = {nm} done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
              flush=True)
    line = {"workload": "serial-ref", "n_disks": n, "eta": eta, "cells_per_side": 4, "ell": ell,
            "seeds": seeds, "serial_sweeps": base_sweeps, "warmup_sweeps_per_n_m_16": base_warm,
            "serial": {r: {"z_mean": v[0], "z_stderr": v[1]} for r, v in ref.items()},
            "pec": cases, "seconds": time.perf_counter() - t0}
    print(json.dumps(line), flush=True)

def bench_nm_scan(args, torch, P):
    """Pressure against the list length n_m for both start rules (Sec. 3.4,
    Fig. 3 right): N = 16384, eta = 0.70, 16 x 16 cells (about 64 disks each),
    n_m = 1, 4, 16, 64, 8 seeds per case, both pressure routes.  At n_m = 1 the
    two rules draw from the same distribution, the paper's reference.  Every
    case runs the same number of chains (64 / n_m times the sweeps of
    n_m = 64) and the same number of g(r) samples."""
    import math
    n, eta, ell, C, seeds = 16384, 0.70, 20.0, 16, 8
    box = math.sqrt(n * math.pi / (4.0 * eta))
    warm, meas = max(args.warmup, 1) * 10, max(args.steps, 1) * 5

    def stats(v):
        m = sum(v) / len(v)
        return m, math.sqrt(sum((x - m) ** 2 for x in v) / (len(v) - 1) / len(v))

    t0 = time.perf_counter()
    cases = {}
    for nm in (1, 4, 16, 64):
        scale = 64 // nm
        ps = []
        for rule in (P.EC_START_REPLACE, P.EC_START_DISTINCT):
            for sd in range(seeds):
                ps.append(P.make_params(n, eta, ell, C, seed=sd + 1, chains_per_cell=nm, start_mode=rule,
                                        system=len(ps)))
        b = P.Batch(ps)
        b.set_graph(True)
        b.sweep(warm * scale)
        b.stream.synchronize()
        for sy in b.systems:
            sy.reset_tallies()
            sy.gr_reset()
        for _ in range(meas):
            b.sweep(scale)
            for sy in b.systems:
                sy.gr_accumulate(1.5, 100)
        b.stream.synchronize()
        zs = [_z_routes(P, sy, n, box) for sy in b.systems]
        b.close()
        for r, rule in enumerate(("replacement", "distinct")):
            part = zs[r * seeds:(r + 1) * seeds]
            cases[(nm, rule)] = {route: stats([z[k] for z in part])
                                 for k, route in enumerate(("ec", "gr_contact"))}
        print(f"# nm-scan: n_m = {nm} done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
              flush=True)
    # reference: n_m = 1, both rules pooled (the same distribution)
    out = []
    for (nm, rule), v in sorted(cases.items()):
        c = {"n_m": nm, "rule": rule, "sweeps": meas * 64 // nm}
        for route in ("ec", "gr_contact"):
            m, se = v[route]
            r1, r2 = cases[(1, "replacement")][route], cases[(1, "distinct")][route]
            rm = 0.5 * (r1[0] + r2[0])
            rse = 0.5 * math.hypot(r1[1], r2[1])
            c[route] = {"z_mean": m, "z_stderr": se,
                        "minus_n_m_1_in_stderr": (m - rm) / math.hypot(se, rse) if nm > 1 else None}
        out.append(c)
    line = {"workload": "nm-scan", "n_disks": n, "eta": eta, "cells_per_side": C, "ell": ell,
            "seeds": seeds, "warmup_sweeps_at_n_m_64": warm, "sweeps_at_n_m_64": meas,
            "cases": out, "seconds": time.perf_counter() - t0}
    print(json.dumps(line), flush=True)

def bench_boundary_rules(args, torch, P):
    """Reflection (the paper's rule) against rejection at the cell boundary
    (Sec. 3.4), each with starts drawn with replacement and with shuffled
    distinct starts (Fig. 3 left and right): N = 16384, eta = 0.70, 16 x 16
    cells, ell = 0.2 sigma (the front of a straight chain advances by about
    sigma per lift, some 10 ell here, and rejection needs it to stay inside
    the cell), n_m = n_c, 8 seeds per case, g(r) sampled every 10 sweeps;
    pressure from g(r) at contact (the EC estimator does not apply to
    rejected chains) and, for reflection, from the lift tallies."""
    import math
    n, eta, ell, C, seeds = 16384, 0.70, 0.2, 16, 8
    box = math.sqrt(n * math.pi / (4.0 * eta))
    warm, meas = max(args.warmup, 1) * 300, max(args.steps, 1) * 15

    def stats(v):
        m = sum(v) / len(v)
        return m, math.sqrt(sum((x - m) ** 2 for x in v) / (len(v) - 1) / len(v))

    t0 = time.perf_counter()
    res = {}
    for bname, bflag in (("reflect", 0), ("reject", P.EC_FLAG_REJECT)):
        ps = []
        for rule in (P.EC_START_REPLACE, P.EC_START_DISTINCT):
            for sd in range(seeds):
                ps.append(P.make_params(n, eta, ell, C, seed=sd + 1, start_mode=rule, system=len(ps),
                                        flags=bflag))
        b = P.Batch(ps)
        b.set_graph(True)
        b.sweep(warm)
        b.stream.synchronize()
        for sy in b.systems:
            sy.reset_tallies()
            sy.gr_reset()
        for _ in range(meas):
            b.sweep(10)
            for sy in b.systems:
                sy.gr_accumulate(1.5, 100)
        b.stream.synchronize()
        zs = [_z_routes(P, sy, n, box) for sy in b.systems]
        counts = [sy.measure_pressure()[2] for sy in b.systems]
        b.close()
        for r, rule in enumerate(("replacement", "distinct")):
            part = zs[r * seeds:(r + 1) * seeds]
            cnt = counts[r * seeds:(r + 1) * seeds]
            chains = sum(c["chains"] for c in cnt)
            rejected = sum(c["walls"] + c["frozen"] for c in cnt) if bflag else 0
            res[(bname, rule)] = {"gr_contact": stats([z[1] for z in part]),
                                  "ec": stats([z[0] for z in part]) if not bflag else None,
                                  "rejected_fraction": rejected / chains if chains else None}
        print(f"# boundary-rules: {bname} done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
              flush=True)
    ref = res[("reflect", "replacement")]["gr_contact"]
    cases = []
    for (bname, rule), v in res.items():
        m, se = v["gr_contact"]
        c = {"boundary": bname, "rule": rule, "rejected_fraction": v["rejected_fraction"],
             "gr_contact": {"z_mean": m, "z_stderr": se,
                            "minus_reflect_replacement_in_stderr":
                                (m - ref[0]) / math.hypot(se, ref[1]) if (bname, rule) != ("reflect", "replacement") else None}}
        if v["ec"] is not None:
            c["ec"] = {"z_mean": v["ec"][0], "z_stderr": v["ec"][1]}
        cases.append(c)
    line = {"workload": "boundary-rules", "n_disks": n, "eta": eta, "cells_per_side": C, "ell": ell,
            "seeds": seeds, "warmup_sweeps": warm, "sweeps": meas * 10, "gr_samples": meas,
            "cases": cases,
            "seconds": time.perf_counter() - t0}
    print(json.dumps(line), flush=True)

if __name__ == "__main__":
    main()
