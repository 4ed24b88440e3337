#!/usr/bin/env python3
"""Throughput of the MPMC hard-disk sweep on one MI355X.

Workload: N = 1,048,576 hard disks (1024 x 1024 triangular lattice) at
packing fraction 0.70, cells narrower than sqrt(2) sigma (826 x 714 cells,
capacity 4), n_M = 4 trial moves per active cell, square trial moves with
delta tuned to about 30 % acceptance by the plain tuner during warm-up and
frozen for the timed sweeps.  One step = one sweep (four checkerboard
sub-sweeps, the random grid shift and the rebuild of the cell lists).

Prints one JSON line: trial moves per second over the timed sweeps, the
sub-sweep kernel's achieved bandwidth against the HBM peak, and the CPU
oracle timed on a bounded sample of the same workload.  Two more objects
compare the batched and learned-controller forms with the plain form:
  batched -- 64 replicas of uneven N (64^2 .. 512^2) and packing fraction
             (0.65 .. 0.73), all from one equilibrated batch state, in one
             handle against the same 64 systems run one after another (same
             chain, bit for bit); with n_M from the autotuner; and
             learned+batched: the trained network sets delta, n_M
             autotuned; P* per replica of each form against the plain batch
             next to a seed control;
  learned -- a move-size network trained on windows the sweeps log (256^2
             systems, phi 0.65 .. 0.73), then at phi = 0.700, 0.716 and
             0.720 both arms start from one equilibrated 1M-disk state: 20
             windows of the network or the plain tuner, delta frozen, then
             mean-square displacement per second of production sweeps and
             beta P sigma^2 with its block error (the plain arm's P* is the
             equilibrated equation of state, checked against Table 2);
  eos     -- (with --eos) a short lattice-start P* at the three phi;
  table3  -- the paper's own throughput benchmark like for like: phi 0.698,
             in-circle moves of radius 0.16, n_M = 4, N = 253^2 .. 3040^2,
             median eta of 11 runs next to the paper's K20 figures;
  spheres -- the same chain in three dimensions: 100^3 hard spheres at
             eta = 0.45, n_M = 4, delta tuned to about 30 % acceptance during
             warm-up, trial moves per second and the sub-sweep kernel against
             the HBM peak.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed sweeps (>= 1)")
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed sweeps after the fixed set-up (tuner, launch shape); < 0 reads as 0")
    ap.add_argument("--phi", type=float, default=0.70)
    ap.add_argument("--lattice", type=int, default=1024)
    ap.add_argument("--n-moves", type=int, default=4)
    ap.add_argument("--block", type=int, default=0,
                    help="sub-sweep workgroup size; 0 = pick the shape with the autotuner")
    ap.add_argument("--lanes", type=int, default=1, help="lanes per cell when --block is given")
    ap.add_argument("--separate", action="store_true",
                    help="four sub-sweep launches and a rebuild per sweep instead of the fused sweep "
                         "(the same chain; for profiling the separate kernels)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the all-core oracle run (0 = every host core)")
    ap.add_argument("--kernel-samples", type=int, default=200,
                    help="sub-sweep launches timed one by one with HIP events")
    ap.add_argument("--cpu-sweeps", type=int, default=0,
                    help="oracle sweeps for the CPU baseline (0 = sized to ~15 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-sweeps", type=int, default=160)
    ap.add_argument("--batched-equilibration", type=int, default=100000,
                    help="sweeps from the lattices before the batched comparisons")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-equilibration", type=int, default=200000,
                    help="sweeps from the lattice before the learned-vs-plain comparison")
    ap.add_argument("--learned-production", type=int, default=4000)
    ap.add_argument("--train-lattice", type=int, default=256,
                    help="side of the lattices the controller's training windows come from")
    ap.add_argument("--train-windows", type=int, default=300)
    ap.add_argument("--no-eos", action="store_true",
                    help="(kept for old command lines; the short EOS leg runs only with --eos)")
    ap.add_argument("--eos", action="store_true",
                    help="also run the short lattice-start EOS leg (equilibrated P* at the three "
                         "phi comes from the learned leg's plain arms)")
    ap.add_argument("--no-table3", action="store_true",
                    help="skip the paper's Table 3 benchmark (in-circle moves, N = 253^2 .. 3040^2)")
    ap.add_argument("--table3-runs", type=int, default=11)
    ap.add_argument("--no-spheres", action="store_true", help="skip the 3D hard-sphere leg")
    ap.add_argument("--eos-equilibration", type=int, default=8000)
    ap.add_argument("--eos-blocks", type=int, default=20)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this size (a known byte count "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def host_cpu():
    """Model name and logical core count of the host CPU."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def cpu_baseline(args, geo):
    """The CPU oracle on the same workload: a bounded number of sweeps from
    the lattice, timed with a monotonic clock, once on one thread and once
    with OpenMP over the active cells of each sub-sweep on every host core
    (the cells of a set are independent, so the chain is the same)."""
    import oracle
    model, ncores = host_cpu()
    threads = args.cpu_threads if args.cpu_threads > 0 else ncores

    def timed(nthreads, budget_s):
        O = oracle.OracleSystem.lattice(args.lattice, args.lattice, args.phi, w_max=math.sqrt(2.0),
                                        delta=0.1, n_moves=args.n_moves, seed=1)
        used = O.set_threads(nthreads)
        O.sweep(1)                                   # touch memory once
        n = args.cpu_sweeps
        if n <= 0:
            t0 = time.perf_counter()
            O.sweep(2)
            per = (time.perf_counter() - t0) / 2
            n = max(3, min(400, int(budget_s / max(per, 1e-6))))
        tr0, _ = O.counters()
        t0 = time.perf_counter()
        O.sweep(n)
        dt = time.perf_counter() - t0
        tr1, _ = O.counters()
        return (tr1 - tr0) / dt, n, tr1 - tr0, dt, used

    v1, n1, t1, d1, _ = timed(1, 12.0)
    vall, nall, tall, dall, used = timed(threads, 8.0)
    return {"value": vall, "unit": "trial moves/s", "cores": used, "kind": "oracle",
            "sample": "%d sweeps of the %d-disk workload from the lattice (%d trial moves, %.1f s), "
                      "C oracle with OpenMP over the active cells of each sub-sweep on %d threads"
                      % (nall, geo["n_particles"], tall, dall, used),
            "host_cpu": model, "host_logical_cores": ncores,
            "one_thread": {"value": v1, "unit": "trial moves/s", "cores": 1,
                           "sample": "%d sweeps (%d trial moves, %.1f s), serial C oracle"
                                     % (n1, t1, d1)}}


def traffic_from_profile(kernel_src, kernel_name, key="hbm bytes per launch",
                         profile="subsweep_1M_phi070_counters.md"):
    """A figure of a committed counter summary (HBM bytes per sub-sweep
    launch by default), if it was taken on the current kernel source and the
    same kernel (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()[:16]
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            vals[k.strip()] = v.strip().split()[0]
    if vals.get("kernel source sha256/16") != digest or vals.get("kernel") != kernel_name.split("<")[0]:
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


VALU_PEAK_WAVE_INSTR = 256 * 4 * 2.4e9 / 4   # 1,024 SIMDs, one wave64 VALU instruction per 4 cycles


def alu_roofline(src, kernel_name, profile, k_avg_ms):
    """The same kernel against the VALU issue ceiling: wave64 VALU
    instructions per launch (committed counter summary of the same kernel
    source, else None) over this run's launch time, against 1,024 SIMDs
    issuing one wave64 VALU instruction per 4 cycles at 2.4 GHz."""
    n = traffic_from_profile(src, kernel_name, "valu wave instructions per launch", profile=profile)
    if n is None:
        return None
    achieved = n / (k_avg_ms * 1e-3)
    return {"unit": "wave64 VALU instructions/s", "achieved": achieved,
            "peak": VALU_PEAK_WAVE_INSTR, "frac": achieved / VALU_PEAK_WAVE_INSTR,
            "instructions_per_launch": n}


def spheres_leg(args):
    """The 3D chain: 100^3 spheres at eta = 0.45 (see sphere_throughput.py)."""
    from paper_1211_1646_amd import sphere_throughput as ST
    r = ST.measure(side=100, eta=0.45, n_moves=4, delta=0.05, warmup=100, steps=500,
                   kernel_samples=64)
    src = os.path.join(ROOT, "paper_1211_1646_amd", "csrc", "sphere_kernels.hip")
    prof = "sphere_subsweep_1M_eta045_counters.md"
    k = r["roofline"]["kernel"]
    r["roofline"]["traffic"] = traffic_from_profile(src, k, profile=prof)
    r["roofline"]["valu_busy"] = traffic_from_profile(src, k, "valu busy fraction", profile=prof)
    r["roofline"]["alu"] = alu_roofline(src, k, prof, r["roofline"]["kernel_avg_us"] * 1e-3)
    return r


def cpu_baseline_spheres(delta):
    """The 3D oracle on three sweeps of the same 100^3-sphere workload (the
    GPU leg's tuned delta, from the lattice)."""
    from oracle.spheres import SphereOracle
    O = SphereOracle.lattice(100, 100, 100, 0.45, delta=delta, n_moves=4, seed=1)
    t0 = time.perf_counter()
    O.sweep(3)
    dt = time.perf_counter() - t0
    tr, _ = O.counters()
    return {"value": tr / dt, "unit": "trial moves/s", "cores": 1, "kind": "oracle",
            "sample": "3 sweeps of the 1,000,000-sphere workload from the lattice (%d trial moves, "
                      "%.1f s, serial C oracle, one thread)" % (tr, dt)}


def batched_leg(args, pkg, torch, net=None):
    """64 replicas of uneven N and packing fraction, all started from one
    equilibrated batch state (plain tuner, then --batched-equilibration
    sweeps from the lattices): the batched form against the same 64 systems
    run one after another (bit for bit the same chain), the batched form
    with n_M picked by the n_M autotuner, and with a trained network the
    learned+batched form (network-set delta, autotuned n_M).  Each form's P*
    per replica is compared with the plain batch's, next to a seed control."""
    from paper_1211_1646_amd import workloads as W
    from paper_1211_1646_amd import controller as ctl
    specs = W.replicas(64, seed=1)
    lat = [pkg.SystemConfig(lattice_nx=s["nx"], lattice_ny=s["ny"], phi=s["phi"], w_min=s["w_min"],
                            w_max=s["w_max"], delta=0.1, n_moves=args.n_moves, seed=1, replica=r)
           for r, s in enumerate(specs)]
    t0 = time.perf_counter()
    Beq = pkg.HardDiskBatch(lat)
    Beq.tune(10, 20)
    Beq.sweep(args.batched_equilibration)
    states = [Beq.get_state(r) for r in range(Beq.R)]
    geos = Beq.geometries
    deltas = np.array([float(Beq.delta(r)) for r in range(Beq.R)], np.float32)
    Beq.close()
    eq_s = time.perf_counter() - t0

    def grid_cfgs(seed=1):
        return [pkg.SystemConfig(cells_x=g["cells_x"], cells_y=g["cells_y"], cell_w_x=g["w_x"],
                                 cell_w_y=g["w_y"], n_particles=g["n_particles"],
                                 delta=float(deltas[r]), n_moves=args.n_moves, seed=seed,
                                 replica=r, flags=pkg.FLAG_ACC) for r, g in enumerate(geos)]

    def loaded_batch(seed=1):
        B = pkg.HardDiskBatch(grid_cfgs(seed))
        for r, st in enumerate(states):
            B.set_state(r, *st)
        return B

    def timed(B, n):
        B.reset_acc()
        tr0 = B.counters()[0]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        B.prepare_sweeps(n)
        B.synchronize()
        e0.record(B.stream)
        B.sweep(n)
        e1.record(B.stream)
        e1.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3
        _, _, dl, msd = B.stats(with_msd=True)
        return sec, B.counters()[0] - tr0, dl, msd

    cfgs = grid_cfgs()
    Ns = np.array([g["n_particles"] for g in geos], np.float64)
    n = args.batched_sweeps
    n_candidates = pkg.HardDiskBatch.AUTOTUNE_CANDIDATES
    B = loaded_batch()
    lanes, blk, _ = B.autotune(16)
    bsec, btr, _, msd = timed(B, n)
    b_msd_sum = float((Ns * msd).sum())
    eos_plain = eos_window(B, torch)
    B.close()
    # the batched form with trials per cell from the n_M autotuner
    B2 = loaded_batch()
    B2.set_launch(lanes, blk)
    best_nm, rates = ctl.autotune_moves(B2, (2, 4, 8, 16), window_sweeps=64)
    B2.sweep(16)                      # graph re-captured for the chosen n_M
    a_sec, _, _, msd2 = timed(B2, n)
    a_msd_sum = float((Ns * msd2).sum())
    eos_auto = eos_window(B2, torch)
    B2.close()
    z = np.abs(eos_auto[0] - eos_plain[0]) / np.sqrt(eos_auto[1] ** 2 + eos_plain[1] ** 2)
    lb = None
    if net is not None:
        B4 = loaded_batch()
        B4.control(net, 10, 4)
        B4.set_launch(lanes, blk)
        B4.set_n_moves(best_nm)
        B4.sweep(16)
        l_sec, _, l_deltas, msd4 = timed(B4, n)
        l_msd_sum = float((Ns * msd4).sum())
        eos_lb = eos_window(B4, torch)
        B4.close()
        z4 = np.abs(eos_lb[0] - eos_plain[0]) / np.sqrt(eos_lb[1] ** 2 + eos_plain[1] ** 2)
        lb = (l_msd_sum / l_sec, l_deltas, z4)
    # control: the plain batch from the same states with another seed
    B3 = loaded_batch(seed=2)
    B3.set_launch(lanes, blk)
    B3.sweep(n_candidates * 32 + n)
    eos_ctrl = eos_window(B3, torch)
    B3.close()
    z0 = np.abs(eos_ctrl[0] - eos_plain[0]) / np.sqrt(eos_ctrl[1] ** 2 + eos_plain[1] ** 2)
    # the same replicas, one handle each, one after another, through the same
    # chain as the plain batch (the autotuner's sweeps, then the timed window)
    seq_sec, seq_tr, seq_msd = 0.0, 0, 0.0
    for r, c in enumerate(cfgs):
        S = pkg.HardDiskSystem(c)
        S.set_state(*states[r])
        S.set_launch(lanes, blk)
        S.sweep(n_candidates * 32)
        t0 = S.counters()[0]
        S.reset_acc()
        S.prepare_sweeps(n)
        S.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(S.stream)
        S.sweep(n)
        e1.record(S.stream)
        e1.synchronize()
        seq_sec += e0.elapsed_time(e1) * 1e-3
        seq_tr += S.counters()[0] - t0
        seq_msd += float(Ns[r]) * S.msd()
        S.close()

    def zsum(v):
        return {"mean": float(v.mean()), "max": float(v.max()),
                "frac_above_2": float((v > 2).mean()), "frac_above_3": float((v > 3).mean())}

    out = {"replicas": len(cfgs), "disks": int(Ns.sum()), "sweeps": n,
           "equilibration_sweeps": args.batched_equilibration + 200,
           "equilibration_seconds": eq_s,
           "trial_moves_per_s": btr / bsec, "sequential_trial_moves_per_s": seq_tr / seq_sec,
           "speedup": (btr / bsec) / (seq_tr / seq_sec),
           "msd_sum_per_s": b_msd_sum / bsec, "sequential_msd_sum_per_s": seq_msd / seq_sec,
           "subsweep_lanes_per_cell": lanes, "subsweep_block": blk,
           "autotuned_n_moves": best_nm,
           "autotune_msd_per_s_by_n_moves": {str(k): v for k, v in rates.items()},
           "autotuned_msd_sum_per_s": a_msd_sum / a_sec,
           "autotuned_vs_sequential_msd_per_s": (a_msd_sum / a_sec) / (seq_msd / seq_sec),
           "eos_check": "P* per replica over 8 blocks of 256 sweeps after the timed window, from "
                        "equilibrated states: autotuned n_M vs n_M = %d, |dP| / combined SE"
                        % args.n_moves,
           "eos_z": zsum(z),
           "eos_z_control": zsum(z0),
           "eos_control": "the n_M = %d batch with seed 2 against seed 1, same check" % args.n_moves}
    if lb is not None:
        out["learned_batched"] = {
            "msd_sum_per_s": lb[0],
            "vs_sequential_plain_msd_per_s": lb[0] / (seq_msd / seq_sec),
            "vs_batched_plain_msd_per_s": lb[0] / (b_msd_sum / bsec),
            "n_moves": best_nm,
            "delta_range": [float(np.min(lb[1])), float(np.max(lb[1]))],
            "plain_delta_range": [float(np.min(deltas)), float(np.max(deltas))],
            "eos_z": zsum(lb[2])}
    return out


def eos_window(B, torch, blocks=8, per_block=256, sample_every=16):
    """P* of every replica of a batch: `blocks` blocks of `per_block` sweeps,
    a contact histogram every `sample_every` sweeps; returns (mean, SE) per
    replica over the blocks."""
    P = np.zeros((blocks, B.R))
    for b in range(blocks):
        for k in range(per_block // sample_every):
            B.sweep(sample_every)
            B.pair_histogram(reset=(k == 0))
        for r in range(B.R):
            P[b, r] = B.pressure_from_contact(r)[0]
    return P.mean(axis=0), P.std(axis=0, ddof=1) / math.sqrt(blocks)


PAPER_TABLE3_K20 = {"253": 6.23e8, "760": 9.83e8, "1520": 1.09e9, "3040": 1.09e9}  # eta, Table 3


def table3_leg(args, pkg, torch):
    """The paper's throughput benchmark (Table 3) like for like: phi = 0.698,
    in-circle moves of radius 0.16, n_M = 4, cells as wide as the paper's,
    N = 253^2 .. 3040^2.  Per N: the launch shape from the autotuner, then
    11 runs from the lattice, each 100 warm-up and 100 timed sweeps (HIP
    events on the system's stream); the median eta = trial moves / s."""
    from paper_1211_1646_amd import workloads as W
    out = {}
    for side in W.PAPER_TABLE3_SIDES:
        w = W.paper_benchmark(side)
        cfg = pkg.SystemConfig(lattice_nx=w["nx"], lattice_ny=w["ny"], phi=w["phi"], w_min=1.0,
                               w_max=w["w_max"], delta=w["delta"], n_moves=w["n_moves"], seed=1,
                               flags=pkg.FLAG_DISK)
        S = pkg.HardDiskSystem(cfg)
        lanes, block, _ = S.autotune(16)
        geo = S.geometry
        S.close()
        etas, accs = [], []
        for run in range(args.table3_runs):
            cfg.seed = 1 + run
            S = pkg.HardDiskSystem(cfg)
            S.set_launch(lanes, block)
            S.sweep(100)
            S.synchronize()
            t0, a0 = S.counters()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(S.stream)
            S.sweep(100)
            e1.record(S.stream)
            e1.synchronize()
            t1, a1 = S.counters()
            etas.append((t1 - t0) / (e0.elapsed_time(e1) * 1e-3))
            accs.append((a1 - a0) / max(t1 - t0, 1))
            S.close()
        etas.sort()
        med = etas[len(etas) // 2]
        out[str(side)] = {
            "N": geo["n_particles"], "cells": [geo["cells_x"], geo["cells_y"]],
            "w": [geo["w_x"], geo["w_y"]], "mean_occupancy": geo["n_particles"] / (geo["cells_x"] * geo["cells_y"]),
            "lanes": lanes, "block": block, "runs": len(etas),
            "eta_median": med, "eta_min": etas[0], "eta_max": etas[-1],
            "acceptance": float(np.median(accs)),
            "paper_k20_eta": PAPER_TABLE3_K20[str(side)], "vs_paper_k20": med / PAPER_TABLE3_K20[str(side)]}
        print("[bench] table 3, N=%d: eta %.4g (K20 %.3g, x%.1f)" % (
            geo["n_particles"], med, PAPER_TABLE3_K20[str(side)], med / PAPER_TABLE3_K20[str(side)]),
            file=sys.stderr, flush=True)
    top = max(v["eta_median"] for v in out.values())
    for v in out.values():
        v["eta_over_max"] = v["eta_median"] / top
    out["note"] = ("phi 0.698, in-circle moves d = 0.16, n_M = 4, cell width ~1.399 (the paper's grid "
                   "rule on its square box); 253^2 is run as a 254 x 252 lattice")
    return out


PAPER_TABLE2_1024 = {"0.698": 9.16934, "0.702": 9.1882, "0.706": 9.1859, "0.710": 9.1842,
                     "0.714": 9.1819, "0.718": 9.1951}   # Table 2, N = 1024^2, MPMC


def eos_leg(args, pkg, torch, lanes, block):
    """beta P sigma^2 of the 1M-disk system at each packing fraction of the
    large workload: plain tuner, equilibration, then production sweeps with a
    contact histogram every 20 sweeps, P* per block of 200 sweeps."""
    out = {}
    for phi in (0.700, 0.716, 0.720):
        cfg = pkg.SystemConfig(lattice_nx=args.lattice, lattice_ny=args.lattice, phi=phi,
                               w_max=math.sqrt(2.0), delta=0.1, n_moves=args.n_moves, seed=1)
        S = pkg.HardDiskSystem(cfg)
        S.set_launch(lanes, block)
        S.tune(10, 20)
        S.sweep(args.eos_equilibration)
        S.synchronize()
        P = []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = S.counters()[0]
        ms = 0.0
        for b in range(args.eos_blocks):
            for k in range(10):
                e0.record(S.stream)
                S.sweep(20)
                e1.record(S.stream)
                S.pair_histogram(reset=(k == 0))
                e1.synchronize()
                ms += e0.elapsed_time(e1)
            P.append(S.pressure_from_contact()[0])
        trials = S.counters()[0] - t0
        P = np.array(P)
        out["%.3f" % phi] = {"P": float(P.mean()), "P_se": float(P.std(ddof=1) / math.sqrt(len(P))),
                             "blocks": len(P), "delta": float(S.delta),
                             "trial_moves_per_s": trials / (ms * 1e-3)}
        S.close()
    out["equilibration_sweeps"] = args.eos_equilibration + 200
    out["paper_table2_N1024sq"] = PAPER_TABLE2_1024
    out["note"] = ("lattice start and ~1e4 sweeps, so P* reads 1-3 % below the equilibrium "
                   "value; python -m paper_1211_1646_amd.eos with 4e5 + 4e5 sweeps per phi "
                   "(about a minute each) lands within 0.1 % of the paper's table")
    return out


PAPER_TABLE2_INTERP = {"0.700": (9.16934 + 9.1882) / 2,      # Table 2, N = 1024^2, linear
                       "0.716": (9.1819 + 9.1951) / 2}        # between the neighbouring phi


def equilibrated_state(pkg, args, phi, sweeps, lanes, block):
    """The 1M-disk system at phi after the plain tuner (20 windows of 10
    sweeps) and `sweeps` more sweeps from the lattice: (cells, widths,
    state).  Both arms of a comparison start from this same state."""
    cfg = pkg.SystemConfig(lattice_nx=args.lattice, lattice_ny=args.lattice, phi=phi,
                           w_max=math.sqrt(2.0), delta=0.1, n_moves=args.n_moves, seed=1)
    S = pkg.HardDiskSystem(cfg)
    S.set_launch(lanes, block)
    S.tune(10, 20)
    S.sweep(sweeps)
    xy, st, sw = S.get_state()
    geo = S.geometry
    S.close()
    return geo, (xy, st, sw)


def arm_from_state(pkg, args, geo, state, lanes, block, seed):
    """A fresh handle on the grid of `geo`, loaded with `state`, keeping
    displacement accumulators."""
    cfg = pkg.SystemConfig(cells_x=geo["cells_x"], cells_y=geo["cells_y"],
                           cell_w_x=geo["w_x"], cell_w_y=geo["w_y"],
                           n_particles=geo["n_particles"], delta=0.1, n_moves=args.n_moves,
                           seed=seed, flags=pkg.FLAG_ACC)
    S = pkg.HardDiskSystem(cfg)
    S.set_state(*state)
    S.set_launch(lanes, block)
    return S


def learned_leg(args, pkg, torch, lanes_main, block_main):
    """Train the controller on windows logged from 256^2-disk systems (the
    medium workload's size) over phi 0.65 .. 0.73, then compare it with the
    plain tuner on the 1M-disk workload at phi 0.700, 0.716 and 0.720, both
    arms starting from one equilibrated state: 20 windows of 10 sweeps with
    the tuner or the network, delta frozen, then production sweeps with
    mean-square displacement per second and P* with its block error."""
    from paper_1211_1646_amd import controller as ctl
    phis = [0.65, 0.66, 0.67, 0.68, 0.69, 0.70, 0.71, 0.72, 0.73]
    deltas = [0.02, 0.04, 0.06, 0.08, 0.10, 0.12, 0.14, 0.16, 0.18, 0.20, 0.22, 0.24, 0.26,
              0.28, 0.30]
    base = [pkg.SystemConfig(lattice_nx=args.train_lattice, lattice_ny=args.train_lattice, phi=p,
                             w_max=math.sqrt(2.0), n_moves=args.n_moves, seed=1) for p in phis]
    t0 = time.perf_counter()
    net, info = ctl.train_controller(base, deltas, windows=args.train_windows, window_sweeps=10,
                                     skip=20, steps=2000)
    train_s = time.perf_counter() - t0
    out = {"training": {"systems": "%d x %d disks, phi %.2f .. %.2f, %d deltas"
                                   % (args.train_lattice, args.train_lattice, phis[0], phis[-1],
                                      len(deltas)),
                        "samples": info["samples"], "seconds": train_s,
                        "loss_first": info["loss_first"], "loss_last": info["loss_last"],
                        "labels": {"%.2f" % k: v for k, v in sorted(info["labels"].items())}},
           "equilibration_sweeps": args.learned_equilibration + 200,
           "production_sweeps": args.learned_production}
    for phi in (0.700, 0.716, 0.720):
        geo, state = equilibrated_state(pkg, args, phi, args.learned_equilibration, lanes_main,
                                        block_main)
        res = {}
        for mode in ("plain", "learned"):
            S = arm_from_state(pkg, args, geo, state, lanes_main, block_main, seed=11)
            res[mode] = ctl.equilibrate_and_measure(S, mode, net, eq_windows=20, window_sweeps=10,
                                                    prod_sweeps=args.learned_production,
                                                    sample_every=10, blocks=10)
            S.close()
        pl, le = res["plain"], res["learned"]
        comb = math.hypot(pl["P_se"], le["P_se"])
        key = "%.3f" % phi
        entry = {"plain": pl, "learned": le,
                 "msd_per_s_ratio": le["msd_per_s"] / pl["msd_per_s"],
                 "P_diff_in_combined_se": abs(le["P"] - pl["P"]) / comb if comb > 0 else None,
                 "equal_eos_accuracy": bool(comb > 0 and abs(le["P"] - pl["P"]) <= 3 * comb
                                            and le["P_se"] <= 1.25 * pl["P_se"])}
        if key in PAPER_TABLE2_INTERP:
            ref = PAPER_TABLE2_INTERP[key]
            entry["plain_P_vs_table2_interp"] = {"table2": ref, "rel": pl["P"] / ref - 1.0,
                                                 "within_0.2pct": abs(pl["P"] / ref - 1.0) <= 2e-3}
        out[key] = entry
        print("[bench] learned phi=%.3f: MSD/s x%.3f, P* %.4f (%.4f) vs %.4f (%.4f)"
              % (phi, entry["msd_per_s_ratio"], le["P"], le["P_se"], pl["P"], pl["P_se"]),
              file=sys.stderr, flush=True)
    return out, net


TUNER_WINDOWS = 20          # plain tuner during set-up: 20 windows ...
TUNER_WINDOW_SWEEPS = 10    # ... of 10 sweeps (delta to ~30 % acceptance, then frozen)
GRAPH_SWEEPS = 16           # sweeps per captured graph in the library


def warmup_plan(warmup: int, steps: int) -> dict:
    """Untimed work before the timed sweeps.  A fixed set-up -- the plain
    tuner over TUNER_WINDOWS windows, then (unless a launch shape is given)
    the launch-shape autotuner -- and then `warmup` extra sweeps, read as 0
    when negative.  The timed `steps` sweeps are graph launches only: the
    library's 16-sweep graph steps // 16 times and one graph of the rest."""
    if steps < 1:
        raise ValueError("--steps must be at least 1")
    return {"tuner_windows": TUNER_WINDOWS, "tuner_window_sweeps": TUNER_WINDOW_SWEEPS,
            "tuner_sweeps": TUNER_WINDOWS * TUNER_WINDOW_SWEEPS,
            "extra_sweeps": max(0, int(warmup)),
            "timed_graph_launches": steps // GRAPH_SWEEPS + (1 if steps % GRAPH_SWEEPS else 0)}


def kernel_time(S, torch, launches):
    """Mean duration of one sub-sweep launch: `launches` launches (the four
    sets in turn, as inside a sweep) captured into one graph on the system's
    stream and replayed between two HIP events on that stream, after one
    untimed replay.  Each launch's share includes the graph's gap before the
    next node, so this is an upper bound on the kernel's own duration."""
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=S.stream):
        for i in range(launches):
            S.subsweep(i % 4)
    with torch.cuda.stream(S.stream):
        g.replay()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(S.stream)
        g.replay()
        e1.record(S.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / launches
    del g
    return ms


def side_leg(name, out, fn):
    """Run one optional leg; a failure is recorded in the line, not raised,
    so that the headline figure is always printed."""
    print("[bench] %s leg" % name, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    try:
        out[name] = fn()
    except Exception as e:  # noqa: BLE001 -- reported in the JSON line
        out[name] = {"error": "%s: %s" % (type(e).__name__, e)}
    print("[bench] %s leg done in %.1f s" % (name, time.perf_counter() - t0), file=sys.stderr,
          flush=True)
    return out[name]


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    plan = warmup_plan(args.warmup, args.steps)
    import torch
    import paper_1211_1646_amd as pkg

    cfg = pkg.SystemConfig(lattice_nx=args.lattice, lattice_ny=args.lattice, phi=args.phi,
                           w_max=math.sqrt(2.0), delta=0.1, n_moves=args.n_moves, seed=1, flags=0)
    print("[bench] building system N=%d phi=%.3f" % (args.lattice ** 2, args.phi), file=sys.stderr,
          flush=True)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    S = pkg.HardDiskSystem(cfg)
    if args.separate:
        S.set_fused(False)
    geo = S.geometry
    N, C = geo["n_particles"], geo["cells_x"] * geo["cells_y"]

    # set-up: delta tuned to ~30 % acceptance, then frozen; launch shape
    S.tune(plan["tuner_window_sweeps"], plan["tuner_windows"])
    S.synchronize()
    delta = float(S.delta)
    if args.block > 0:
        S.set_launch(args.lanes, args.block)
        tuned = None
    else:
        tuned = S.autotune(16)
    if plan["extra_sweeps"]:
        S.sweep(plan["extra_sweeps"])
    S.prepare_sweeps(args.steps)   # capture now: the timed region only launches graphs
    S.synchronize()
    print("[bench] set-up done: delta=%.5f after %d tuner sweeps, sub-sweep %d lanes per cell, "
          "block %d%s, %d more warm-up sweeps" % (
              delta, plan["tuner_sweeps"], S.lanes, S.block,
              " (autotuned, %.1f us/sweep)" % tuned[2] if tuned else "", plan["extra_sweeps"]),
          file=sys.stderr, flush=True)

    # timed sweeps: graph launches only, HIP events on the system's stream,
    # synchronised on both sides
    t0_trials, t0_acc = S.counters()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(S.stream)
    S.sweep(args.steps)
    ev1.record(S.stream)
    ev1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    gpu_ms = ev0.elapsed_time(ev1)
    t1_trials, t1_acc = S.counters()
    trials = t1_trials - t0_trials
    secs = gpu_ms / 1e3
    value = trials / secs
    print("[bench] %d sweeps in %.3f ms (wall %.3f s), %.4g trial moves/s, acceptance %.3f"
          % (args.steps, gpu_ms, wall, value, (t1_acc - t0_acc) / max(trials, 1)),
          file=sys.stderr, flush=True)

    cap = geo["capacity"]
    fused = S.fused
    if fused:
        # dominant kernel: the fused sweep, one launch per sweep, so its mean
        # launch time is the timed region's per sweep (graph gaps included);
        # algorithmic bytes of a sweep: four sub-sweeps reading every
        # position and count (4 (8 N + 4 C)), the active cells' write-backs
        # (8 N), the rebuild reading and writing positions and counts
        # (16 N + 8 C): 56 N + 24 C
        ks = args.steps
        k_avg_ms = gpu_ms / args.steps
        bytes_per_launch = 56.0 * N + 24.0 * C
        # template arguments: capacity, proposal (0 = square), one system, largest
        # tile side, accumulators, tags
        tile, ftx, fty = S.fused_tile
        kernel_name = "k_sweep_fused<%d, 0, true, %d, false, false>" % (cap, tile)
        timing = ("the timed region: %d sweeps, one launch each, HIP events on the system's "
                  "stream (graph gaps included)" % args.steps)
    else:
        # dominant kernel: the sub-sweep (four launches per sweep); bytes per
        # launch: every position read once (8 N), every cell count read once
        # (4 C), the active quarter of positions written back (8 N / 4)
        ks = max(4, args.kernel_samples)
        k_avg_ms = kernel_time(S, torch, ks)
        bytes_per_launch = 8.0 * N + 4.0 * C + 2.0 * N
        # template arguments: capacity, [lanes per cell,] proposal (0 = square), one system
        kernel_name = ("k_subsweep<%d, 0, true>" % cap if S.lanes == 1
                       else "k_subsweep_mc<%d, %d, 0, true>" % (cap, S.lanes))
        timing = ("%d launches in one captured graph, HIP events around the replay on the "
                  "system's stream (graph gaps included)" % ks)
    achieved = bytes_per_launch / (k_avg_ms * 1e-3) / 1e9
    S.synchronize()
    src = os.path.join(ROOT, "paper_1211_1646_amd", "csrc", "mpmc_kernels.hip")
    prof = "sweep_fused_1M_phi070_counters.md" if fused else "subsweep_1M_phi070_counters.md"

    out = {
        "metric": "trial moves/sec at 1M disks phi=0.70; MSD/sec learned+batched vs plain",
        "value": value,
        "unit": "trial moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: triangular-lattice start, Philox streams seed 1",
        "config": {"workload": "hard disks N=%d (%dx%d lattice), phi=%.3f, cells %dx%d (w=%.5f x %.5f, "
                               "capacity %d), n_M=%d, delta=%.5f tuned to ~30%% acceptance"
                               % (N, args.lattice, args.lattice, args.phi, geo["cells_x"], geo["cells_y"],
                                  geo["w_x"], geo["w_y"], geo["capacity"], args.n_moves, delta),
                   "sweeps_per_s": args.steps / secs,
                   "acceptance": (t1_acc - t0_acc) / max(trials, 1),
                   "trial_moves_per_sweep": trials / args.steps,
                   "sweep_kernel": ("fused (one tiled launch per sweep, tiles of %dx%d cells)"
                                    % S.fused_tile[1:]) if fused
                                   else "four sub-sweep launches and a rebuild",
                   "subsweep_lanes_per_cell": S.lanes,
                   "subsweep_block": S.block,
                   "tuner_sweeps": plan["tuner_sweeps"],
                   "autotune_sweeps": 2 * 16 * S.AUTOTUNE_CANDIDATES if tuned else 0,
                   "extra_warmup_sweeps": plan["extra_sweeps"],
                   "timed_graph_launches": plan["timed_graph_launches"],
                   "wall_s_timed": wall,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_from_profile(src, kernel_name, profile=prof),
                     "valu_busy": traffic_from_profile(src, kernel_name, "valu busy fraction",
                                                       profile=prof),
                     "alu": alu_roofline(src, kernel_name, prof, k_avg_ms),
                     "kernel": kernel_name, "kernel_avg_us": k_avg_ms * 1e3,
                     "kernel_timing": timing,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
    }
    S.close()
    lanes_main, block_main = out["config"]["subsweep_lanes_per_cell"], out["config"]["subsweep_block"]
    net = None
    if not args.no_learned:
        res = side_leg("learned", out, lambda: learned_leg(args, pkg, torch, lanes_main, block_main))
        if isinstance(res, tuple):
            out["learned"], net = res
    if not args.no_batched:
        side_leg("batched", out, lambda: batched_leg(args, pkg, torch, net))
    if args.eos and not args.no_eos:
        side_leg("eos", out, lambda: eos_leg(args, pkg, torch, lanes_main, block_main))
    if not args.no_table3:
        side_leg("table3", out, lambda: table3_leg(args, pkg, torch))
    if not args.no_spheres:
        side_leg("spheres", out, lambda: spheres_leg(args))
    if not args.no_cpu_baseline:
        cb = side_leg("cpu_baseline", out, lambda: cpu_baseline(args, geo))
        if not args.no_spheres and "error" not in cb and "delta" in out.get("spheres", {}):
            try:
                cb["spheres"] = cpu_baseline_spheres(out["spheres"]["delta"])
            except Exception as e:  # noqa: BLE001
                cb["spheres"] = {"error": "%s: %s" % (type(e).__name__, e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
