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
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed sweeps")
    ap.add_argument("--warmup", type=int, default=200, help="untimed sweeps (tuner runs here)")
    ap.add_argument("--phi", type=float, default=0.70)
    ap.add_argument("--lattice", type=int, default=1024)
    ap.add_argument("--n-moves", type=int, default=4)
    ap.add_argument("--block", type=int, default=0,
                    help="sub-sweep workgroup size; 0 = pick with the autotuner during warm-up")
    ap.add_argument("--kernel-samples", type=int, default=200,
                    help="sub-sweep launches timed one by one with HIP events")
    ap.add_argument("--cpu-sweeps", type=int, default=0,
                    help="oracle sweeps for the CPU baseline (0 = sized to ~15 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this size (a known byte count "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def cpu_baseline(args, geo, trials_per_sweep_gpu):
    """The CPU oracle (serial C, one thread) on the same workload: a bounded
    number of sweeps from the same lattice, timed with a monotonic clock."""
    import oracle
    O = oracle.OracleSystem.lattice(args.lattice, args.lattice, args.phi, w_max=math.sqrt(2.0),
                                    delta=0.1, n_moves=args.n_moves, seed=1)
    O.sweep(1)                                   # touch memory once
    n = args.cpu_sweeps
    if n <= 0:
        t0 = time.perf_counter()
        O.sweep(2)
        per = (time.perf_counter() - t0) / 2
        n = max(3, min(200, int(15.0 / max(per, 1e-6))))
    tr0, _ = O.counters()
    t0 = time.perf_counter()
    O.sweep(n)
    dt = time.perf_counter() - t0
    tr1, _ = O.counters()
    return {"value": (tr1 - tr0) / dt, "unit": "trial moves/s", "cores": 1, "kind": "oracle",
            "sample": "%d sweeps of the %d-disk workload from the lattice (%d trial moves, %.1f s, "
                      "serial C oracle, one thread)" % (n, geo["n_particles"], tr1 - tr0, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
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
    geo = S.geometry
    N, C = geo["n_particles"], geo["cells_x"] * geo["cells_y"]

    # warm-up: tune delta to ~30 % acceptance in windows of 10 sweeps, then freeze
    windows = max(1, args.warmup // 10)
    S.tune(10, windows)
    S.sweep(args.warmup - 10 * windows)
    S.synchronize()
    delta = float(S.delta)
    # launch shape: autotuned (shape never changes results), or as given
    if args.block > 0:
        S.set_launch(1, args.block)
        tuned = None
    else:
        tuned = S.autotune(16)
    print("[bench] warm-up done, delta=%.5f, sub-sweep block %d%s" % (
        delta, S.block, " (autotuned, %.1f us/sweep)" % tuned[1] if tuned else ""),
        file=sys.stderr, flush=True)

    # timed sweeps: one captured graph per 16 sweeps, events on the system's stream
    t0_trials, t0_acc = S.counters()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(S.stream)
    S.sweep(args.steps)
    ev1.record(S.stream)
    ev1.synchronize()
    wall = time.perf_counter() - wall0
    gpu_ms = ev0.elapsed_time(ev1)
    t1_trials, t1_acc = S.counters()
    trials = t1_trials - t0_trials
    secs = gpu_ms / 1e3
    value = trials / secs
    print("[bench] %d sweeps in %.3f ms (wall %.3f s), %.4g trial moves/s, acceptance %.3f"
          % (args.steps, gpu_ms, wall, value, (t1_acc - t0_acc) / max(trials, 1)),
          file=sys.stderr, flush=True)

    # dominant kernel: the sub-sweep, one launch at a time between HIP events
    # on the stream it runs on
    ks = max(4, args.kernel_samples)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(ks)]
    for i in range(ks):
        evs[i][0].record(S.stream)
        S.subsweep(i % 4)
        evs[i][1].record(S.stream)
    evs[-1][1].synchronize()
    kms = sorted(a.elapsed_time(b) for a, b in evs)
    k_avg_ms = sum(kms) / len(kms)
    # algorithmic bytes per sub-sweep launch: every position read once (8 N),
    # every offset read once (4 (C + 1)), the active quarter of positions
    # written back (8 N / 4)
    bytes_per_launch = 8.0 * N + 4.0 * (C + 1) + 2.0 * N
    achieved = bytes_per_launch / (k_avg_ms * 1e-3) / 1e9
    S.synchronize()

    out = {
        "metric": "trial moves/sec at 1M disks phi=0.70",
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
                   "subsweep_block": S.block,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_subsweep<4>", "kernel_avg_us": k_avg_ms * 1e3,
                     "kernel_median_us": kms[len(kms) // 2] * 1e3,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args, geo, trials / args.steps)
    S.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
