"""Equation of state P*(phi) of hard disks on the GPU (Sec. 4): a triangular
lattice at packing fraction phi, the plain tuner, equilibration sweeps, then
production sweeps with a contact histogram every `sample_every` sweeps and
P* from the contact value per block (Eqs. gR, R, P); the result is the block
mean with its standard error.

    python -m paper_1211_1646_amd.eos --phi 0.698 0.718 --nx 1024
    python -m paper_1211_1646_amd.eos --phi 0.698 0.702 --nx 256 --replicas 8

prints one JSON line per packing fraction (the second form runs all of them
as one batch of independent replicas).
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


# Table 2, MPMC rows: P* at N = 256^2, 512^2, 1024^2
PAPER_TABLE2 = {
    256: {0.698: 9.1709, 0.702: 9.1920, 0.706: 9.1854, 0.710: 9.1792, 0.714: 9.1758, 0.718: 9.187},
    512: {0.698: 9.1699, 0.702: 9.1900, 0.706: 9.1861, 0.710: 9.1828, 0.714: 9.1800, 0.718: 9.1930},
    1024: {0.698: 9.16934, 0.702: 9.1882, 0.706: 9.1859, 0.710: 9.1842, 0.714: 9.1819,
           0.718: 9.1951}}


def equation_of_state_batch(phis, nx: int = 256, replicas: int = 8,
                            equilibration: int = 400_000, production: int = 400_000,
                            sample_every: int = 100, blocks: int = 10, n_moves: int = 4,
                            seed: int = 1, w_max: float = math.sqrt(2.0), progress=None) -> list:
    """P*(phi) for several packing fractions at once: one batch of
    len(phis) x `replicas` independent systems (replica r runs phis[r % P]
    with Philox key (seed, r)), each tuned, equilibrated and sampled as in
    equation_of_state.  A packing fraction's P* is the mean over its replicas
    of their time averages; its standard error comes from the spread between
    those independent replicas."""
    from .system import HardDiskBatch
    P = len(phis)
    cfgs = [SystemConfig(lattice_nx=nx, lattice_ny=nx, phi=phis[r % P], w_max=w_max, delta=0.1,
                         n_moves=n_moves, seed=seed, replica=r) for r in range(P * replicas)]
    B = HardDiskBatch(cfgs)
    t0 = time.time()
    B.autotune(16)
    B.tune(10, 30)
    chunk = 50_000
    done = 0
    while done < equilibration:
        k = min(chunk, equilibration - done)
        B.sweep(k)
        B.synchronize()
        done += k
        if progress:
            progress("N %d^2 x %d replicas: equilibration %d / %d (%.0f s)" % (
                nx, len(cfgs), done, equilibration, time.time() - t0))
    samples = max(1, (production // blocks) // sample_every)
    Pb = np.zeros((blocks, len(cfgs)))
    for b in range(blocks):
        for k in range(samples):
            B.sweep(sample_every)
            B.pair_histogram(reset=(k == 0))
        for r in range(len(cfgs)):
            Pb[b, r] = B.pressure_from_contact(r)[0]
        if progress:
            progress("N %d^2: block %d / %d (%.0f s)" % (nx, b + 1, blocks, time.time() - t0))
    _, _, deltas, _ = B.stats()
    B.close()
    per_rep = Pb.mean(axis=0)
    out = []
    for i, phi in enumerate(phis):
        v = per_rep[i::P]
        row = {"phi": phi, "N": nx * nx, "replicas": replicas, "P": float(v.mean()),
               "P_se": float(v.std(ddof=1) / math.sqrt(len(v))),
               "equilibration_sweeps": equilibration, "production_sweeps": production,
               "delta": float(np.mean(deltas[i::P])), "seconds": time.time() - t0}
        ref = PAPER_TABLE2.get(nx, {}).get(round(phi, 3))
        if ref is not None:
            row["paper_P"] = ref
            row["relative_difference"] = row["P"] / ref - 1.0
        out.append(row)
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
    ap.add_argument("--replicas", type=int, default=0,
                    help="> 0: run every phi at once in one batch with this many replicas each")
    a = ap.parse_args()
    if a.replicas > 0:
        for row in equation_of_state_batch(a.phi, a.nx, a.replicas, a.equilibration, a.production,
                                           a.sample_every, a.blocks, seed=a.seed,
                                           progress=lambda m: print("[eos] " + m, flush=True)):
            print(json.dumps(row), flush=True)
        return
    for phi in a.phi:
        r = equation_of_state(phi, a.nx, a.equilibration, a.production, a.sample_every, a.blocks,
                              seed=a.seed, progress=lambda m: print("[eos] " + m, flush=True))
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
