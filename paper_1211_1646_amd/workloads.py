"""Seeded synthetic workloads (inputs only: no step of the method lives here).

The paper's measurements use synthetic hard-disk systems started from
triangular lattices (Sec. 4, Tables 2 and 3); these recipes produce the
parameters of such systems.  Both the HIP path's tests and the oracle's side
of them take their inputs from here.
"""
from __future__ import annotations

import math

import numpy as np


def large(phi: float = 0.70) -> dict:
    """1024 x 1024 lattice (N = 1,048,576) with cells narrower than sqrt(2)
    (capacity 4, about two disks per cell)."""
    return dict(nx=1024, ny=1024, phi=phi, w_min=1.0, w_max=math.sqrt(2.0))


def medium() -> dict:
    """256 x 256 lattice (N = 65,536) at phi = 0.70, cells of width >= 1."""
    return dict(nx=256, ny=256, phi=0.70, w_min=1.0, w_max=0.0)


def small() -> dict:
    """64 x 64 lattice (N = 4096) at phi = 0.60, cells of width >= 1."""
    return dict(nx=64, ny=64, phi=0.60, w_min=1.0, w_max=0.0)


PAPER_TABLE3_SIDES = (253, 760, 1520, 3040)


def paper_benchmark(side: int, phi: float = 0.698) -> dict:
    """The throughput benchmark of Table 3: N = side^2 disks at phi = 0.698,
    in-circle trial moves of radius d = 0.16 and n_M = 4 (the tuned values of
    Sec. 3.3).

    The paper's box is square, and its grid has m = floor(L / sqrt 2) cells per
    side rounded up to a multiple of 64 (Sec. 3.1), i.e. cells of width
    w_p = L / m (about 1.399 for these N).  Here the box is the lattice's
    rectangle, so each axis takes the smallest even cell count with w < w_p:
    cells as wide and as full as the paper's.  A triangular lattice needs an
    even number of rows, so an odd side becomes (side + 1) x (side - 1)
    (N one less)."""
    L = math.sqrt(side * side * math.pi / (4.0 * phi))
    m = -(-math.floor(L / math.sqrt(2.0)) // 64) * 64
    nx, ny = (side, side) if side % 2 == 0 else (side + 1, side - 1)
    return dict(nx=nx, ny=ny, phi=phi, w_min=1.0, w_max=L / m, delta=0.16, n_moves=4,
                in_circle=True, paper_cells=m, paper_w=L / m)


def replicas(R: int = 64, seed: int = 1, n_min: int = 64, n_max: int = 512,
             phi_lo: float = 0.65, phi_hi: float = 0.73) -> list[dict]:
    """R square lattices n_r x n_r, N_r = n_r^2 log-uniform between n_min^2 and
    n_max^2 (n_r even), packing fractions evenly spaced over [phi_lo, phi_hi],
    cells narrower than sqrt(2) (the paper's choice, capacity 4, about 1.7
    disks per cell).  Sizes come from numpy's PCG64 seeded with `seed`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(R)
    half_lo, half_hi = n_min // 2, n_max // 2
    out = []
    for r in range(R):
        k = int(round(half_lo * (half_hi / half_lo) ** float(u[r])))
        n = 2 * min(max(k, half_lo), half_hi)
        phi = phi_lo + (phi_hi - phi_lo) * (r / (R - 1) if R > 1 else 0.0)
        out.append(dict(nx=n, ny=n, phi=phi, w_min=1.0, w_max=math.sqrt(2.0)))
    return out
