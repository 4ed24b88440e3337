"""Throughput against system size, as in the paper's Fig. 4(a) and Table 3:
eta = trial moves per second at phi = 0.698 with the paper's proposal
(in-circle moves of radius 0.16, n_M = 4), for a list of lattice sides, with
cells narrower than sqrt(2).  Per side: the launch shape from the autotuner,
then `runs` runs from the lattice of 100 warm-up and 100 timed sweeps (HIP
events on the handle's stream), and the median.  With --batch-disks B, the
same sweep is also timed for a batch of max(1, B // N) replicas of that
size, whose aggregate eta shows what batching recovers for small systems.

    python -m paper_1211_1646_amd.throughput --sides 64 128 253 512 1024 2048

prints one JSON line per side.
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

from . import workloads as W
from ._lib import FLAG_DISK
from .system import HardDiskBatch, HardDiskSystem, SystemConfig


def _eta(make, runs: int, warm: int = 100, timed: int = 100):
    import torch
    lanes, block, _ = make(1).autotune(16)
    etas = []
    for run in range(runs):
        S = make(1 + run)
        S.set_launch(lanes, block)
        S.sweep(warm)
        S.synchronize()
        t0 = S.counters()[0]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(S.stream)
        S.sweep(timed)
        e1.record(S.stream)
        e1.synchronize()
        etas.append((S.counters()[0] - t0) / (e0.elapsed_time(e1) * 1e-3))
        S.close()
    return float(np.median(etas)), lanes, block


def eta_against_size(side: int, runs: int = 11, batch_disks: int = 0) -> dict:
    # the paper's proposal and packing fraction; cells narrower than sqrt(2),
    # the paper's width criterion, at every size (its rounding of the cell
    # count to multiples of 64 would give small systems cells narrower than 1)
    w = W.paper_benchmark(side)

    def cfg(seed, replica=0):
        return SystemConfig(lattice_nx=w["nx"], lattice_ny=w["ny"], phi=w["phi"], w_min=1.0,
                            w_max=math.sqrt(2.0), delta=w["delta"], n_moves=w["n_moves"],
                            seed=seed, replica=replica, flags=FLAG_DISK)

    N = w["nx"] * w["ny"]
    eta, lanes, block = _eta(lambda seed: HardDiskSystem(cfg(seed)), runs)
    out = {"side": side, "N": N, "eta": eta, "runs": runs, "lanes": lanes, "block": block}
    if batch_disks > 0:
        R = max(1, batch_disks // N)
        beta, _, _ = _eta(lambda seed: HardDiskBatch([cfg(seed, r) for r in range(R)]),
                          max(3, runs // 4))
        out.update({"batch_replicas": R, "batch_eta": beta})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--sides", type=int, nargs="+", default=[64, 128, 253, 512, 760, 1024])
    ap.add_argument("--runs", type=int, default=11)
    ap.add_argument("--batch-disks", type=int, default=0,
                    help="also time batches of about this many disks in all")
    a = ap.parse_args()
    for side in a.sides:
        print(json.dumps(eta_against_size(side, a.runs, a.batch_disks)), flush=True)


if __name__ == "__main__":
    main()
