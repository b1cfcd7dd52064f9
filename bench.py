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
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from tests import inputs  # noqa: E402  (seeded workload definitions; no method arithmetic)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VECTOR_PEAK_TF = 78.6     # MI355X FP64 vector, TFLOP/s
# FP64 work of one event (algorithmic): contact tests of the disks in the
# 3 x 3 neighbourhood of sigma-sized squares (about 8 disks at rho sigma^2 =
# 0.92; 2 sub, 2 mul + 2 fma for r.d and r x d, 1 fma, sqrt, sub = 12 flop
# each) plus the commit (2 fma) = 8 * 12 + 4 = 100 flop.
FLOP_PER_EVENT = 100.0
# HBM bytes of one sweep per disk (algorithmic): rebin reads x, y (16) and
# writes/reads the cell index (8) and the id list (8); the four phases read
# every disk once as its own (16 + 4 id) and write it back (16), and read the
# frozen halo (about a quarter of the disks again, 20).
HBM_BYTES_PER_DISK = 16 + 8 + 8 + 20 + 16 + 20


SCHEDULE_FLAGS = {"auto": lambda P: 0,
                  "one-launch": lambda P: P.EC_FLAG_ONE_LAUNCH,
                  "phase-launches": lambda P: P.EC_FLAG_PHASE_LAUNCHES}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of the simulation-cell kernel from the committed
    counter summary, or None when the kernel source has changed since the
    counters were taken."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_1409_6948_amd", "csrc", "ec_kernels.hip")
    prof = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.md")
    if not os.path.exists(prof):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(prof):
        m = re.match(r"traffic: .*source_sha256_prefix=(\w+) read_bytes_per_launch=(\S+) "
                     r"write_bytes_per_launch=(\S+)", line)
        if m and m.group(1) == sha:
            return float(m.group(2)) + float(m.group(3))
    return None


def cpu_baseline(w, budget_s=15.0):
    """Time the CPU oracle on first-phase cells of sweep 0 from the lattice."""
    from oracle import oracle as O
    p = O.params(w["n"], w["eta"], w["ell"], w["cells"], dir_mode=O.DIR_ISO, seed=w["seed"])
    st = O.State(p)
    C = w["cells"]
    _, _, perm = O.sweep_draws(p, 0)
    first = [c for c in range(C * C) if ((c % C) & 1) | (((c // C) & 1) << 1) == perm[0]]
    done, lifts, t_cells = 0, 0, 0.0
    for c in first:
        t0 = time.perf_counter()
        st.run_cells(0, [c], n_phases=1)
        t_cells += time.perf_counter() - t0
        done += 1
        if t_cells >= budget_s:
            break
    lifts = int(st.acc_cnt[:, O.CNT_LIFTS].sum())
    return {"value": lifts / t_cells, "unit": "lifts/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} first-phase cells of sweep 0 of {w['n']} disks from the lattice "
                      f"({lifts} lifts in {t_cells:.1f} s; rebin and halo scan excluded)"}


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
                         "(one launch for a system alone, phase launches for a batch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=("fp64", "fp32-screen"), default="fp64",
                    help="fp32-screen: FP32 screening of candidates, FP64 for the survivors "
                         "and every commit (identical events)")
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
    prec = P.EC_PREC_FP64 if args.precision == "fp64" else P.EC_PREC_FP32_SCREEN
    flags = SCHEDULE_FLAGS[args.schedule](P)
    kernel = "k_phase" if args.schedule == "phase-launches" else "k_sweep_cells"
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
    print(f"# workload {args.workload}: warmup {args.warmup} sweeps", file=sys.stderr, flush=True)
    g.sweep(args.warmup)
    torch.cuda.synchronize()
    g.reset_tallies()
    g.set_timing(True)
    stream = g.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for k in range(args.steps):
        g.sweep(1)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    phase_ms, launches = g.get_timing()
    g.set_timing(False)
    z, bp, counts = g.measure_pressure()
    secs = gpu_ms / 1e3
    lifts = counts["lifts"]
    events = counts["lifts"] + counts["frozen"] + counts["walls"] + counts["chains"]
    value = lifts / secs
    sweeps_s = args.steps / secs
    hbm_frac = (HBM_BYTES_PER_DISK * w["n"] * sweeps_s) / (HBM_PEAK_GBS * 1e9)
    avg_phase_s = phase_ms / 1e3 / max(launches, 1)
    flop_per_launch = FLOP_PER_EVENT * events / max(launches, 1)
    achieved_tf = flop_per_launch / avg_phase_s / 1e12
    line = {
        "metric": "EC collisions (lifts)/sec, 1 MI355X, N=1M eta=0.72",
        "value": value,
        "unit": "lifts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_disks": w["n"], "eta": w["eta"],
                   "cells_per_side": w["cells"], "ell": w["ell"], "directions": "isotropic",
                   "precision": args.precision,
                   "schedule": "phase-launches" if kernel == "k_phase" else "one-launch",
                   "start": "lattice",
                   "sweeps_before_timing": args.warmup},
        "sweeps_per_s": sweeps_s,
        "events_per_s": events / secs,
        "counts": counts,
        "z_timed_sweeps": z,
        "hbm_frac_whole_sweep": hbm_frac,
        "wall_s": wall,
        "roofline": {"bound": "alu", "kernel": kernel, "achieved": achieved_tf,
                     "peak": FP64_VECTOR_PEAK_TF, "unit": "TFLOP/s",
                     "frac": achieved_tf / FP64_VECTOR_PEAK_TF,
                     "traffic": measured_traffic(kernel, args.workload),
                     "avg_launch_ms": avg_phase_s * 1e3, "launches": launches,
                     "kernel_share_of_sweep": phase_ms / gpu_ms},
    }
    if not args.no_cpu_baseline:
        print("# CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


def bench_batch(args, torch, P):
    """Aggregate lifts/s of the 64-system ensemble in the batched form, and the
    same sweeps run system by system (solo launches, one system after another)."""
    cfgs = inputs.batch_systems(64, seed=0)
    flags = SCHEDULE_FLAGS[args.schedule](P)
    ps = [P.make_params(c["n"], c["eta"], c["ell"], c["cells"], dir_mode=c["dir_mode"],
                        seed=c["seed"], system=i, flags=flags) for i, c in enumerate(cfgs)]
    torch.cuda.set_device(0)
    b = P.Batch(ps)
    print(f"# batch64: {len(ps)} systems, sum N = {sum(c['n'] for c in cfgs)}", file=sys.stderr,
          flush=True)
    b.sweep(1)
    cpb, trials = b.autotune(trial_sweeps=2)
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
    lifts = 0
    events = 0
    for s in b.systems:
        _, _, c = s.measure_pressure()
        lifts += c["lifts"]
        events += c["lifts"] + c["frozen"] + c["walls"] + c["chains"]
    # the same sweeps, system by system
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
        "value": lifts / secs,
        "unit": "lifts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batch64", "n_systems": len(ps),
                   "sum_n": int(sum(c["n"] for c in cfgs)), "eta_range": [0.30, 0.72],
                   "ell": 20.0, "cells_per_block": cpb,
                   "schedule": "one-launch" if args.schedule == "one-launch" else "phase-launches",
                   "hip_graph": True},
        "events_per_s": events / secs,
        "autotune_trial_ms": trials,
        "solo_sequential_s": solo_secs,
        "speedup_vs_solo_sequential": solo_secs / secs,
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
