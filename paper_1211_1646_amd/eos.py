"""Equation of state P*(phi) of hard disks on the GPU (Sec. 4): a triangular
lattice at packing fraction phi, the plain tuner, equilibration sweeps, then
production sweeps with a contact histogram every `sample_every` sweeps and
P* from the contact value per block (Eqs. gR, R, P); the result is the block
mean with its standard error.

    python -m paper_1211_1646_amd.eos --phi 0.698 0.718 --nx 1024

prints one JSON line per packing fraction.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from .system import HardDiskSystem, SystemConfig


def equation_of_state(phi: float, nx: int = 1024, equilibration: int = 400_000,
                      production: int = 400_000, sample_every: int = 100, blocks: int = 20,
                      n_moves: int = 4, seed: int = 1, w_max: float = math.sqrt(2.0),
                      progress=None) -> dict:
    S = HardDiskSystem(SystemConfig(lattice_nx=nx, lattice_ny=nx, phi=phi, w_max=w_max,
                                    delta=0.1, n_moves=n_moves, seed=seed))
    t0 = time.time()
    S.autotune(16)
    S.tune(10, 30)
    chunk = 50_000
    done = 0
    while done < equilibration:
        k = min(chunk, equilibration - done)
        S.sweep(k)
        S.synchronize()
        done += k
        if progress:
            progress("phi %.3f equilibration %d / %d (%.0f s)" % (phi, done, equilibration,
                                                                 time.time() - t0))
    per_block = production // blocks
    samples = max(1, per_block // sample_every)
    P = []
    for b in range(blocks):
        for k in range(samples):
            S.sweep(sample_every)
            S.pair_histogram(reset=(k == 0))
        P.append(S.pressure_from_contact()[0])
        if progress and (b + 1) % 5 == 0:
            progress("phi %.3f block %d / %d: P* %.5f (%.0f s)" % (phi, b + 1, blocks, P[-1],
                                                                  time.time() - t0))
    P = np.array(P)
    out = {"phi": phi, "N": nx * nx, "P": float(P.mean()),
           "P_se": float(P.std(ddof=1) / math.sqrt(len(P))), "blocks": len(P),
           "equilibration_sweeps": equilibration + 300 + 24 * 16, "production_sweeps": production,
           "samples_per_block": samples, "delta": float(S.delta), "seconds": time.time() - t0}
    S.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--phi", type=float, nargs="+", default=[0.698, 0.718])
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--equilibration", type=int, default=400_000)
    ap.add_argument("--production", type=int, default=400_000)
    ap.add_argument("--sample-every", type=int, default=100)
    ap.add_argument("--blocks", type=int, default=20)
    ap.add_argument("--seed", type=int, default=1)
    a = ap.parse_args()
    for phi in a.phi:
        r = equation_of_state(phi, a.nx, a.equilibration, a.production, a.sample_every, a.blocks,
                              seed=a.seed, progress=lambda m: print("[eos] " + m, flush=True))
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
