"""The balance test of Table 1 on the GPU: P* of hard disks with the particle
shuffle and the checkerboard-set shuffle switched on or off (Sec. 2.4).

One batch holds `per_case` independent replicas of each of the four cases,
interleaved (replica r runs case r mod 4 with Philox key (seed, r)), all at
the same N, packing fraction, proposal (in-circle, d = 0.16, n_M = 4 by
default: the paper's tuned values) and cells narrower than sqrt(2).  After
`equilibration` sweeps from the lattice, every replica takes a contact
histogram every `sample_every` sweeps for `production` sweeps, with P* per
block; a case's P* is the mean over its replicas of their time averages, and
its standard error comes from the spread between those independent replicas.

    python -m paper_1211_1646_amd.ablation --phi 0.708 --side 256
    python -m paper_1211_1646_amd.ablation --phi 0.708 --leave --deltas 0.08 0.16

prints one JSON line per packing fraction.  With --leave the cases are
the plain chain and the two cell-leaving pitfalls of Sec. 2.4 at each move
radius, with each replica's final hexatic order and its orientation.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from ._lib import FLAG_DISK, FLAG_LEAVE, FLAG_LEAVE_ONCE, FLAG_NO_PARTICLE_SHUFFLE, FLAG_NO_SET_SHUFFLE
from .system import HardDiskBatch, SystemConfig

# (particle shuffle, set shuffle) -> flags; Table 1's row order
CASES = (("yes", "yes", 0),
         ("yes", "no", FLAG_NO_SET_SHUFFLE),
         ("no", "yes", FLAG_NO_PARTICLE_SHUFFLE),
         ("no", "no", FLAG_NO_PARTICLE_SHUFFLE | FLAG_NO_SET_SHUFFLE))

# Table 1 (N = 256^2): P* for the four cases at phi = 0.698, 0.708, 0.716
PAPER_TABLE1 = {"0.698": (9.17079, 9.1707, 9.1716, 9.1715),
                "0.708": (9.18214, 9.1821, 9.1876, 9.1873),
                "0.716": (9.1774, 9.1775, 9.1831, 9.1823)}


def shuffle_ablation(phi: float, side: int = 256, per_case: int = 16,
                     equilibration: int = 400_000, production: int = 400_000,
                     sample_every: int = 100, blocks: int = 10, n_moves: int = 4,
                     delta: float = 0.16, in_circle: bool = True, seed: int = 1,
                     cases=(0, 1, 2, 3), progress=None) -> dict:
    """`cases` picks rows of CASES (the first is the reference of the z
    scores; Table 1's reference is both shuffles on, case 0)."""
    K = len(cases)
    R = K * per_case
    disk = FLAG_DISK if in_circle else 0
    cfgs = [SystemConfig(lattice_nx=side, lattice_ny=side, phi=phi, w_min=1.0,
                         w_max=math.sqrt(2.0), delta=delta, n_moves=n_moves, seed=seed,
                         replica=r, flags=CASES[cases[r % K]][2] | disk) for r in range(R)]
    B = HardDiskBatch(cfgs)
    t0 = time.time()
    chunk = 50_000
    done = 0
    while done < equilibration:
        k = min(chunk, equilibration - done)
        B.sweep(k)
        B.synchronize()
        done += k
        if progress:
            progress("phi %.3f equilibration %d / %d (%.0f s)" % (phi, done, equilibration,
                                                                 time.time() - t0))
    per_block = production // blocks
    samples = max(1, per_block // sample_every)
    P = np.zeros((blocks, R))
    for b in range(blocks):
        for k in range(samples):
            B.sweep(sample_every)
            B.pair_histogram(reset=(k == 0))
        for r in range(R):
            P[b, r] = B.pressure_from_contact(r)[0]
        if progress:
            progress("phi %.3f block %d / %d (%.0f s)" % (phi, b + 1, blocks, time.time() - t0))
    tr, ac, _, _ = B.stats()
    B.close()
    per_replica = P.mean(axis=0)
    key = "%.3f" % phi
    out = {"phi": phi, "N": side * side, "replicas_per_case": per_case,
           "equilibration_sweeps": equilibration, "production_sweeps": production,
           "proposal": "in-circle" if in_circle else "square", "delta": delta,
           "n_moves": n_moves, "seconds": time.time() - t0, "cases": []}
    for i, ci in enumerate(cases):
        ps, cs, _ = CASES[ci]
        v = per_replica[i::K]
        case = {"particle_shuffle": ps, "set_shuffle": cs, "P": float(v.mean()),
                "P_se": float(v.std(ddof=1) / math.sqrt(len(v))),
                "acceptance": float(ac[i::K].sum() / max(tr[i::K].sum(), 1))}
        if key in PAPER_TABLE1:
            case["paper_P"] = PAPER_TABLE1[key][ci]
        out["cases"].append(case)
    ref = out["cases"][0]
    for c in out["cases"][1:]:
        d = c["P"] - ref["P"]
        c["minus_both_shuffled"] = d
        c["z"] = d / math.sqrt(c["P_se"] ** 2 + ref["P_se"] ** 2)
        if "paper_P" in c:
            c["paper_minus_both_shuffled"] = c["paper_P"] - ref["paper_P"]
    return out


LEAVE_CASES = (("plain", 0), ("leave", FLAG_LEAVE), ("leave_once", FLAG_LEAVE_ONCE))


def orientation(xy_global, box, rc=1.35):
    """Global hexatic order of a configuration: psi6 = mean over disks of
    the mean over their neighbours (closer than rc) of exp(6 i theta), with
    theta the bond angle against the x axis (periodic box).  Returns
    (|psi6|, its angle / 6 in degrees): the mean lattice orientation."""
    from scipy.spatial import cKDTree
    Lx, Ly = box
    pts = np.mod(xy_global, [Lx, Ly])
    tree = cKDTree(pts, boxsize=[Lx, Ly])
    pairs = tree.query_pairs(rc, output_type="ndarray")
    d = pts[pairs[:, 1]] - pts[pairs[:, 0]]
    d[:, 0] -= Lx * np.round(d[:, 0] / Lx)
    d[:, 1] -= Ly * np.round(d[:, 1] / Ly)
    z = np.exp(6j * np.arctan2(d[:, 1], d[:, 0]))
    acc = np.zeros(len(pts), complex)
    cnt = np.zeros(len(pts))
    np.add.at(acc, pairs[:, 0], z)
    np.add.at(acc, pairs[:, 1], z)
    np.add.at(cnt, pairs[:, 0], 1)
    np.add.at(cnt, pairs[:, 1], 1)
    psi = np.mean(acc[cnt > 0] / cnt[cnt > 0])
    return float(abs(psi)), float(np.degrees(np.angle(psi)) / 6.0)


def leave_ablation(phi: float, side: int = 256, per_case: int = 8, deltas=(0.08, 0.16),
                   equilibration: int = 200_000, production: int = 200_000,
                   sample_every: int = 100, blocks: int = 10, n_moves: int = 4,
                   in_circle: bool = True, seed: int = 1, progress=None) -> dict:
    """The cell-leaving pitfalls of Sec. 2.4 against the plain chain: for
    each move radius d, `per_case` independent replicas of the plain chain,
    of "leaving allowed" and of "leave, each disk once per sweep", in one
    batch; P* per case (spread between replicas) and each replica's final
    global hexatic order and its orientation."""
    nc = len(LEAVE_CASES)
    cases = [(d, name, fl) for d in deltas for name, fl in LEAVE_CASES]
    R = len(cases) * per_case
    disk = FLAG_DISK if in_circle else 0
    cfgs = [SystemConfig(lattice_nx=side, lattice_ny=side, phi=phi, w_min=1.0,
                         w_max=math.sqrt(2.0), delta=cases[r % len(cases)][0], n_moves=n_moves,
                         seed=seed, replica=r, flags=cases[r % len(cases)][2] | disk)
            for r in range(R)]
    B = HardDiskBatch(cfgs)
    t0 = time.time()
    chunk = 50_000
    done = 0
    while done < equilibration:
        k = min(chunk, equilibration - done)
        B.sweep(k)
        B.synchronize()
        done += k
        if progress:
            progress("phi %.3f equilibration %d / %d (%.0f s)" % (phi, done, equilibration,
                                                                 time.time() - t0))
    per_block = production // blocks
    samples = max(1, per_block // sample_every)
    P = np.zeros((blocks, R))
    for b in range(blocks):
        for k in range(samples):
            B.sweep(sample_every)
            B.pair_histogram(reset=(k == 0))
        for r in range(R):
            P[b, r] = B.pressure_from_contact(r)[0]
        if progress:
            progress("phi %.3f block %d / %d (%.0f s)" % (phi, b + 1, blocks, time.time() - t0))
    tr, ac, _, _ = B.stats()
    orient = []
    for r in range(R):
        g = B.geometries[r]
        xy, st, _ = B.get_state(r)
        cell = np.repeat(np.arange(len(st) - 1), np.diff(st.astype(np.int64)))
        cx, cy = cell % g["cells_x"], cell // g["cells_x"]
        glob = np.stack([cx * np.float64(g["w_x"]) + xy[:, 0], cy * np.float64(g["w_y"]) + xy[:, 1]], 1)
        orient.append(orientation(glob, (g["box_x"], g["box_y"])))
    B.close()
    per_replica = P.mean(axis=0)
    out = {"phi": phi, "N": side * side, "replicas_per_case": per_case,
           "equilibration_sweeps": equilibration, "production_sweeps": production,
           "proposal": "in-circle" if in_circle else "square", "n_moves": n_moves,
           "seconds": time.time() - t0, "cases": []}
    for i, (d, name, _) in enumerate(cases):
        v = per_replica[i::len(cases)]
        o = np.array(orient[i::len(cases)])
        out["cases"].append({"delta": d, "case": name, "P": float(v.mean()),
                             "P_se": float(v.std(ddof=1) / math.sqrt(len(v))),
                             "acceptance": float(ac[i::len(cases)].sum() / max(tr[i::len(cases)].sum(), 1)),
                             "psi6": [float(x) for x in o[:, 0]],
                             "psi6_angle_deg": [float(x) for x in o[:, 1]]})
    for c in out["cases"]:
        ref = next(x for x in out["cases"] if x["delta"] == c["delta"] and x["case"] == "plain")
        if c is not ref:
            c["minus_plain"] = c["P"] - ref["P"]
            c["z"] = c["minus_plain"] / math.sqrt(c["P_se"] ** 2 + ref["P_se"] ** 2)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--phi", type=float, nargs="+", default=[0.708])
    ap.add_argument("--side", type=int, default=256)
    ap.add_argument("--per-case", type=int, default=16)
    ap.add_argument("--equilibration", type=int, default=400_000)
    ap.add_argument("--production", type=int, default=400_000)
    ap.add_argument("--sample-every", type=int, default=100)
    ap.add_argument("--blocks", type=int, default=10)
    ap.add_argument("--square", action="store_true", help="square trial moves instead of in-circle")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--leave", action="store_true",
                    help="the cell-leaving pitfalls against the plain chain instead of the shuffles")
    ap.add_argument("--deltas", type=float, nargs="+", default=[0.08, 0.16])
    ap.add_argument("--cases", type=int, nargs="+", default=[0, 1, 2, 3],
                    help="rows of Table 1 to run (0: both shuffles, 1: no set shuffle, 2: no "
                         "particle shuffle, 3: neither); the first is the z reference")
    a = ap.parse_args()
    if a.leave:
        for phi in a.phi:
            r = leave_ablation(phi, a.side, a.per_case, a.deltas, a.equilibration, a.production,
                               a.sample_every, a.blocks, in_circle=not a.square, seed=a.seed,
                               progress=lambda m: print("[ablation] " + m, flush=True))
            print(json.dumps(r), flush=True)
        return
    for phi in a.phi:
        r = shuffle_ablation(phi, a.side, a.per_case, a.equilibration, a.production,
                             a.sample_every, a.blocks, in_circle=not a.square, seed=a.seed,
                             cases=tuple(a.cases),
                             progress=lambda m: print("[ablation] " + m, flush=True))
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
