"""Throughput of the hard-sphere sweep (the method in d = 3) on one GPU.

Workload: side^3 spheres from the simple cubic lattice at packing fraction
eta (default 100^3 = 1,000,000 at eta = 0.45, a fluid), cells narrower than
2/sqrt(3) (92^3 cells, capacity 8), n_M = 4 trial moves per active cell.
The `warmup` sweeps run the plain tuner in windows of 10 sweeps (delta
towards 30 % acceptance from the given start), then delta is frozen and
`steps` sweeps are timed with HIP events on the system's stream (trial
moves per second); then the sub-sweep kernel alone: `kernel_samples`
launches (the eight sets in turn) captured into one graph and replayed
between two events.

    python -m paper_1211_1646_amd.sphere_throughput --side 100 --eta 0.45

prints one JSON line.
"""
from __future__ import annotations

import argparse
import json

from .spheres import HardSphereSystem, SphereConfig

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def algorithmic_bytes(N: int, C: int) -> float:
    """Bytes one sub-sweep launch must move at least: every sphere's three
    FP32 coordinates read once (each is in an active cell or a neighbour of
    one), every cell count read once, the active eighth written back."""
    return 12.0 * N + 4.0 * C + 12.0 * N / 8.0


def measure(side: int = 100, eta: float = 0.45, n_moves: int = 4, delta: float = 0.05,
            warmup: int = 100, steps: int = 500, kernel_samples: int = 64, seed: int = 1,
            copy_calibration_mib: int = 0, lanes: int = 0) -> dict:
    import torch
    if copy_calibration_mib > 0:
        n = copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    S = HardSphereSystem(SphereConfig(lattice_nx=side, lattice_ny=side, lattice_nz=side, eta=eta,
                                      delta=delta, n_moves=n_moves, seed=seed))
    N, C = S.N, S.C
    if lanes:
        S.set_launch(lanes)
    windows = warmup // 10
    S.tune(10, windows)
    S.sweep(warmup - 10 * windows)
    S.synchronize()
    delta = float(S.delta())
    tr0, ac0 = S.counters()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(S.stream)
    S.sweep(steps)
    e1.record(S.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    tr1, ac1 = S.counters()
    trials = tr1 - tr0
    ks = max(8, kernel_samples)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=S.stream):
        for i in range(ks):
            S.subsweep(i % 8)
    with torch.cuda.stream(S.stream):
        g.replay()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record(S.stream)
        g.replay()
        g1.record(S.stream)
    g1.synchronize()
    k_ms = g0.elapsed_time(g1) / ks
    del g
    overlaps = S.count_overlaps()
    S.close()
    bpl = algorithmic_bytes(N, C)
    achieved = bpl / (k_ms * 1e-3) / 1e9
    return {"workload": "hard spheres N=%d (%d^3 simple cubic lattice), eta=%.3f, cells %dx%dx%d "
                        "(w=%.5f, capacity 8), n_M=%d, delta=%.5f tuned to ~30%% acceptance"
                        % (N, side, eta, S.m[0], S.m[1], S.m[2], S.w[0], n_moves, delta),
            "trial_moves_per_s": trials / (ms * 1e-3), "us_per_sweep": ms * 1e3 / steps,
            "steps": steps, "warmup": warmup, "delta": delta,
            "acceptance": (ac1 - ac0) / max(trials, 1),
            "trial_moves_per_sweep": trials / steps, "overlaps_after": overlaps,
            "lanes_per_cell": lanes or "library default",
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "kernel": ("k_subsweep3b<false>" if lanes in (0, 1)
                                    else "k_subsweep3<%d, false>" % lanes),
                         "kernel_avg_us": k_ms * 1e3,
                         "kernel_timing": "%d launches in one captured graph, HIP events around "
                                          "the replay on the system's stream" % ks,
                         "algorithmic_bytes_per_launch": bpl}}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--side", type=int, default=100)
    ap.add_argument("--eta", type=float, default=0.45)
    ap.add_argument("--n-moves", type=int, default=4)
    ap.add_argument("--delta", type=float, default=0.05, help="starting delta of the tuner")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--kernel-samples", type=int, default=64)
    ap.add_argument("--lanes", type=int, default=0, help="sub-sweep lanes per cell (0: default)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="copy this many MiB device to device first (counter calibration)")
    a = ap.parse_args()
    print(json.dumps(measure(a.side, a.eta, a.n_moves, a.delta, a.warmup, a.steps,
                             a.kernel_samples, copy_calibration_mib=a.copy_calibration_mib,
                             lanes=a.lanes)),
          flush=True)


if __name__ == "__main__":
    main()
