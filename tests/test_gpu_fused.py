"""The fused sweep (the four sub-sweeps and the rebuild of a sweep in one
tiled launch, halo updates recomputed in LDS) against the CPU oracle and
against the separate launches, bit for bit, through the C ABI.  Grids
smaller than one tile (every cell loaded several times), ragged edge tiles,
both proposals, the particle-shuffle ablation, accept bits, and the
benchmark's full size.  Needs an MI355X."""
import math
import sys

import numpy as np
import pytest

from oracle import OracleSystem

pytestmark = pytest.mark.gpu
FLAG_ACCEPT_LOG = 4


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1211_1646_amd as pkg
    pkg.load()
    return pkg


def pair(pkg, nx, ny, phi, delta=0.15, n_moves=4, seed=1, flags=0, w_max=math.sqrt(2.0)):
    log("  pair nx=%d ny=%d phi=%.3f n_moves=%d flags=%d" % (nx, ny, phi, n_moves, flags))
    cfg = pkg.SystemConfig(lattice_nx=nx, lattice_ny=ny, phi=phi, w_max=w_max, delta=delta,
                           n_moves=n_moves, seed=seed, flags=flags)
    G = pkg.HardDiskSystem(cfg)
    O = OracleSystem.lattice(nx, ny, phi, w_max=w_max, delta=delta, n_moves=n_moves, seed=seed,
                             flags=flags)
    assert G.geometry["capacity"] == 4
    return G, O


def same(G, O, what):
    gx, gs, gsw = G.get_state()
    ox, os_, osw = O.get_state()
    assert gsw == osw, (what, gsw, osw)
    assert np.array_equal(gs, os_), (what, "cell lists differ")
    assert np.array_equal(gx.view(np.uint32), ox.view(np.uint32)), (what, "positions differ")
    assert G.counters() == O.counters(), (what, G.counters(), O.counters())


# (nx, ny, phi): grids of 14 x 12 cells (smaller than a tile and its halo:
# cells appear several times in the loaded region), 40 x 34 (second tiles
# of 8 and 2 cells) and 64 x 54 (a second row of 22)
SIZES = [(16, 16, 0.70), (48, 48, 0.69), (80, 78, 0.71)]


@pytest.mark.parametrize("nx,ny,phi", SIZES)
def test_fused_sweeps_match_oracle_every_sweep(gpu, nx, ny, phi):
    G, O = pair(gpu, nx, ny, phi, flags=FLAG_ACCEPT_LOG)
    assert G.fused, "this system should sweep in the fused form"
    for k in range(24):
        G.sweep(1)
        O.sweep(1)
        assert np.array_equal(G.accept_log(), O.accept_log()), k
        assert G.counters() == O.counters(), k
    same(G, O, "24 single sweeps")
    G.sweep(40)
    O.sweep(40)
    same(G, O, "40 more in graphs")
    assert G.count_overlaps() == 0


@pytest.mark.parametrize("n_moves", [1, 3, 4, 9])
def test_fused_n_moves(gpu, n_moves):
    G, O = pair(gpu, 40, 40, 0.70, n_moves=n_moves, seed=3)
    G.sweep(19)
    O.sweep(19)
    same(G, O, "n_M %d" % n_moves)


def test_fused_in_circle_and_ablation(gpu):
    for flags in (8, 16, 32, 8 | 16):
        G, O = pair(gpu, 40, 44, 0.70, delta=0.16, seed=5, flags=flags)
        assert G.fused
        G.sweep(21)
        O.sweep(21)
        same(G, O, "flags %d" % flags)


def test_fused_equals_separate_launches(gpu):
    """The same system swept fused and with the four sub-sweeps and the
    rebuild launched separately: identical states, counters and accept
    bits after every sweep."""
    kw = dict(lattice_nx=64, lattice_ny=64, phi=0.70, w_max=math.sqrt(2.0), delta=0.15,
              n_moves=4, seed=9, flags=FLAG_ACCEPT_LOG)
    A = gpu.HardDiskSystem(gpu.SystemConfig(**kw))
    B = gpu.HardDiskSystem(gpu.SystemConfig(**kw))
    B.set_fused(False)
    assert A.fused and not B.fused
    for k in range(10):
        A.sweep(3)
        B.sweep(3)
        assert np.array_equal(A.accept_log(), B.accept_log()), k
        ax, ast, asw = A.get_state()
        bx, bst, bsw = B.get_state()
        assert asw == bsw and np.array_equal(ast, bst)
        assert np.array_equal(ax.view(np.uint32), bx.view(np.uint32)), k
        assert A.counters() == B.counters()
    # switching forms in the middle of a run continues the same chain
    A.set_fused(False)
    B.set_fused(True)
    A.sweep(17)
    B.sweep(17)
    ax, _, _ = A.get_state()
    bx, _, _ = B.get_state()
    assert np.array_equal(ax.view(np.uint32), bx.view(np.uint32))


def test_fused_not_used_where_unsupported(gpu):
    cfg = gpu.SystemConfig(lattice_nx=16, lattice_ny=16, phi=0.7, w_max=1.932, delta=0.1,
                           n_moves=4, seed=1, flags=0)
    S = gpu.HardDiskSystem(cfg)
    assert S.geometry["capacity"] > 4 and not S.fused


@pytest.mark.parametrize("flags", [1, 2, 3, 7])
@pytest.mark.parametrize("nx,ny,phi", [(16, 16, 0.70), (72, 70, 0.70)])
def test_fused_with_accumulators_and_tags(gpu, flags, nx, ny, phi):
    """Accumulators (tile 24) and tags (tile 20) travel with their disks
    through the fused sub-sweeps and the rebuild, bit for bit."""
    G, O = pair(gpu, nx, ny, phi, flags=flags, seed=7)
    assert G.fused
    for k in range(3):
        G.sweep(7)
        O.sweep(7)
        same(G, O, "flags %d block %d" % (flags, k))
        ga, gt = G.aux()
        oa, ot = O.aux()
        if flags & 2:
            assert np.array_equal(gt, ot), k
        if flags & 1:
            assert np.array_equal(ga.view(np.uint32), oa.view(np.uint32)), k
            ref = float(np.mean((oa.astype(np.float64) ** 2).sum(axis=1)))
            assert abs(G.msd() - ref) <= 1e-12 * max(ref, 1e-30), k


def test_fused_batch_matches_single_runs(gpu):
    """A batch of uneven replicas (capacity 4 each, one with in-circle moves,
    one without the particle shuffle) in fused sweeps: each replica equals
    its own oracle run, bit for bit, with accumulators and tags."""
    specs = [(16, 16, 0.66, 0), (40, 36, 0.70, 8), (24, 26, 0.72, 16), (64, 60, 0.69, 0)]
    cfgs = [gpu.SystemConfig(lattice_nx=a, lattice_ny=b, phi=ph, w_max=math.sqrt(2.0), delta=0.14,
                             n_moves=4, seed=3, replica=r, flags=3 | fl)
            for r, (a, b, ph, fl) in enumerate(specs)]
    B = gpu.HardDiskBatch(cfgs)
    assert B.fused
    B.sweep(23)
    for r, (a, b, ph, fl) in enumerate(specs):
        O = OracleSystem.lattice(a, b, ph, w_max=math.sqrt(2.0), delta=0.14, n_moves=4, seed=3,
                                 replica=r, flags=3 | fl)
        O.sweep(23)
        bx, bs, bsw = B.get_state(r)
        ox, os_, osw = O.get_state()
        assert bsw == osw == 23 and np.array_equal(bs, os_), r
        assert np.array_equal(bx.view(np.uint32), ox.view(np.uint32)), r
        ba, bt = B.aux(r)
        oa, ot = O.aux()
        assert np.array_equal(bt, ot) and np.array_equal(ba.view(np.uint32), oa.view(np.uint32)), r
        assert B.replica_counters(r) == O.counters(), r


@pytest.mark.timeout(900)
@pytest.mark.parametrize("phi", [0.700, 0.716, 0.720])
def test_fused_full_size(gpu, phi):
    """1,048,576 disks at the benchmark's geometry: 16 fused sweeps (one
    captured graph) from the lattice equal the oracle's whole state."""
    import os
    G, O = pair(gpu, 1024, 1024, phi, delta=0.1, seed=1)
    O.set_threads(max(1, min(16, len(os.sched_getaffinity(0)))))
    assert G.fused
    G.sweep(16)
    O.sweep(16)
    same(G, O, "16 sweeps")
    assert G.count_overlaps() == 0
