"""Parity of the HIP path (through the C ABI) with the CPU oracle: bit-exact
cell lists, positions, accumulators, tags and counters; the contact fit
within FP64 rounding.  Needs an MI355X."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import OracleSystem
from oracle import estimator as E

pytestmark = pytest.mark.gpu

FLAGS = 3  # accumulators + tags on both sides


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


def lattice_pair(pkg, nx, ny, phi, w_max=0.0, delta=0.1, n_moves=4, seed=1, replica=0,
                 flags=FLAGS, w_min=1.0):
    log("  lattice pair nx=%d ny=%d phi=%.3f w_max=%.4f n_moves=%d" % (nx, ny, phi, w_max, n_moves))
    cfg = pkg.SystemConfig(lattice_nx=nx, lattice_ny=ny, phi=phi, w_min=w_min, w_max=w_max,
                           delta=delta, n_moves=n_moves, seed=seed, replica=replica, flags=flags)
    G = pkg.HardDiskSystem(cfg)
    O = OracleSystem.lattice(nx, ny, phi, w_min=w_min, w_max=w_max, delta=delta, n_moves=n_moves,
                             seed=seed, replica=replica, flags=flags)
    return G, O


def grid_pair(pkg, O, n_moves=None, seed=1, replica=0, flags=FLAGS, delta=None):
    """A GPU system and a fresh oracle, both loaded with the oracle's current
    state (loading clears accumulators and counters on both sides)."""
    xy, start, sweep = O.get_state()
    _, tag = O.aux()
    n_moves = n_moves if n_moves is not None else 4
    delta = np.float32(O.delta if delta is None else delta)
    cfg = pkg.SystemConfig(cells_x=O.mx, cells_y=O.my, cell_w_x=float(O.wx), cell_w_y=float(O.wy),
                           n_particles=len(xy), delta=float(delta), n_moves=n_moves, seed=seed,
                           replica=replica, flags=flags)
    G = pkg.HardDiskSystem(cfg)
    G.set_state(xy, start, sweep, tag)
    O2 = OracleSystem.grid(O.mx, O.my, O.wx, O.wy, delta=delta, n_moves=n_moves, seed=seed,
                           replica=replica, flags=flags)
    O2.set_state(xy, start, sweep, tag)
    return G, O2


def assert_same(G, O, what=""):
    gx, gs, gsw = G.get_state()
    ox, os_, osw = O.get_state()
    assert gsw == osw, (what, gsw, osw)
    assert np.array_equal(gs, os_), (what, "cell lists differ", int(np.argmax(gs != os_)))
    bad = np.nonzero(np.any(gx.view(np.uint32) != ox.view(np.uint32), axis=1))[0]
    assert bad.size == 0, (what, "positions differ", bad[:5], gx[bad[:3]], ox[bad[:3]])
    ga, gt = G.aux()
    oa, ot = O.aux()
    if gt is not None:
        assert np.array_equal(gt, ot), (what, "tags differ")
    if ga is not None:
        assert np.array_equal(ga.view(np.uint32), oa.view(np.uint32)), (what, "accumulators differ")
    assert G.counters() == O.counters(), (what, G.counters(), O.counters())


CONFIGS = [
    (64, 64, 0.60, 0.0),             # small workload, w >= 1
    (24, 24, 0.70, math.sqrt(2.0)),  # w < sqrt(2), capacity 4
    (20, 20, 0.72, 1.932),           # capacity 7
    (16, 18, 0.45, 1.664),           # rectangular lattice, capacity 5
    (30, 30, 0.50, 1.8),             # capacity 6
]


@pytest.mark.parametrize("nx,ny,phi,w_max", CONFIGS)
def test_initial_state_matches(gpu, nx, ny, phi, w_max):
    G, O = lattice_pair(gpu, nx, ny, phi, w_max)
    assert_same(G, O, "init")
    assert G.count_overlaps() == 0


@pytest.mark.parametrize("nx,ny,phi,w_max", CONFIGS)
def test_single_subsweeps_match(gpu, nx, ny, phi, w_max):
    G, O = lattice_pair(gpu, nx, ny, phi, w_max, delta=0.2)
    O.sweep(7)
    G, O = grid_pair(gpu, O, delta=0.2)
    for Q in (2, 0, 3, 1, 1):
        log("  subsweep Q=%d" % Q)
        G.subsweep(Q)
        O.subsweep(Q)
        assert_same(G, O, "subsweep %d" % Q)


@pytest.mark.parametrize("nx,ny,phi,w_max", CONFIGS)
def test_explicit_shifts_match(gpu, nx, ny, phi, w_max):
    G, O = lattice_pair(gpu, nx, ny, phi, w_max, delta=0.2)
    O.sweep(5)
    G, O = grid_pair(gpu, O, delta=0.2)
    rng = np.random.default_rng(nx)
    for f in (0, 1, 2, 3, 2, 0, 3, 1):
        w = O.wx if f < 2 else O.wy
        for d in (np.float32(0.0), np.float32(rng.uniform(0, 0.5)) * np.float32(0.5) * w,
                  np.float32(0.5) * w):
            log("  shift f=%d d=%r" % (f, float(d)))
            G.shift_and_rebin(f, d)
            O.shift(f, d)
            assert_same(G, O, "shift %d %r" % (f, d))


@pytest.mark.parametrize("n_moves", [0, 1, 3, 4, 6, 9])
def test_sweeps_match_for_any_n_moves(gpu, n_moves):
    G, O = lattice_pair(gpu, 20, 20, 0.70, math.sqrt(2.0), delta=0.15, n_moves=n_moves, seed=5)
    for k in range(12):
        G.sweep(1)
        O.sweep(1)
        assert_same(G, O, "sweep %d" % k)


def test_small_workload_1000_sweeps(gpu):
    """N = 4096 at phi = 0.60, w >= 1, delta = 0.1, n_M = 4, seed 1:
    counters after every sweep of the first hundred, the whole state every
    hundred sweeps, including accept counts."""
    G, O = lattice_pair(gpu, 64, 64, 0.60, 0.0, delta=0.1, n_moves=4, seed=1)
    for k in range(100):
        G.sweep(1)
        O.sweep(1)
        assert G.counters() == O.counters(), k
    assert_same(G, O, "sweep 100")
    for block in range(9):
        G.sweep(100)
        O.sweep(100)
        log("  sweeps %d" % (200 + 100 * block))
        assert_same(G, O, "sweep %d" % (200 + 100 * block))
    assert G.count_overlaps() == 0


def test_graph_path_matches_eager_path(gpu):
    G1, O = lattice_pair(gpu, 32, 32, 0.70, math.sqrt(2.0), delta=0.12, seed=3)
    G2, _ = lattice_pair(gpu, 32, 32, 0.70, math.sqrt(2.0), delta=0.12, seed=3)
    G1.sweep(48)            # three captured graphs of 16 sweeps
    for _ in range(48):
        G2.sweep(1)        # one sweep at a time, no graph
    O.sweep(48)
    assert_same(G1, O, "graph")
    assert_same(G2, O, "eager")
    G1.sweep(17)           # graph + one eager sweep, then graphs on the other half
    G1.sweep(16)
    O.sweep(33)
    assert_same(G1, O, "graph odd")


@pytest.mark.parametrize("lanes", [1, 2, 4, 64])
@pytest.mark.parametrize("block", [64, 128, 192, 256])
def test_launch_shape_does_not_change_results(gpu, lanes, block):
    """The separate sub-sweep launches (the fused sweep switched off) at every
    launch shape, one wavefront per cell (64 lanes) included."""
    G, O = lattice_pair(gpu, 40, 40, 0.70, math.sqrt(2.0), delta=0.15, seed=9)
    G.set_fused(False)
    G.set_launch(lanes, block)
    G.sweep(20)
    O.sweep(20)
    assert_same(G, O, "lanes %d block %d" % (lanes, block))


@pytest.mark.parametrize("lanes", [2, 4, 64])
@pytest.mark.parametrize("nx,ny,phi,w_max", CONFIGS)
def test_lane_groups_match_for_every_capacity(gpu, lanes, nx, ny, phi, w_max):
    """Lane groups on capacities 4-7 and n_M from 0 to 9: single sub-sweeps
    and whole sweeps bit-exact."""
    G, O = lattice_pair(gpu, nx, ny, phi, w_max, delta=0.2)
    O.sweep(5)
    G, O = grid_pair(gpu, O, delta=0.2)
    G.set_launch(lanes, 128)
    for Q in (3, 1, 0, 2):
        G.subsweep(Q)
        O.subsweep(Q)
        assert_same(G, O, "lanes %d subsweep %d" % (lanes, Q))
    for n_moves in (0, 1, 6, 9):
        Gm, Om = lattice_pair(gpu, nx, ny, phi, w_max, delta=0.17, n_moves=n_moves, seed=n_moves + 2)
        Gm.set_fused(False)
        Gm.set_launch(lanes, 64)
        Gm.sweep(17)
        Om.sweep(17)
        assert_same(Gm, Om, "lanes %d n_M %d" % (lanes, n_moves))


@pytest.mark.parametrize("lanes", [1, 2, 4, 64])
@pytest.mark.parametrize("nx,ny,phi,w_max", CONFIGS)
def test_in_circle_moves_match(gpu, lanes, nx, ny, phi, w_max):
    """In-circle trial moves (the paper's proposal, MPMC_FLAG_DISK) on every
    capacity and lane count: sweeps bit-exact, accumulators included (they
    hold the sum of the accepted moves' FP32 components), with n_M = 4 and
    n_M = 7 and delta up to w/2."""
    flags = FLAGS | gpu.FLAG_DISK
    for n_moves, delta in ((4, 0.16), (7, 0.45)):
        G, O = lattice_pair(gpu, nx, ny, phi, w_max, delta=delta, n_moves=n_moves, seed=11,
                            flags=flags)
        G.set_fused(False)
        G.set_launch(lanes, 128)
        G.sweep(19)
        O.sweep(19)
        assert_same(G, O, "in-circle lanes %d n_M %d" % (lanes, n_moves))
        assert G.count_overlaps() == 0


@pytest.mark.parametrize("lanes", [1, 2, 4, 64])
@pytest.mark.parametrize("ablate", ["particle", "set", "both"])
def test_shuffle_ablations_match(gpu, lanes, ablate):
    """The balance-test switches of Table 1 (no particle shuffle, no set
    shuffle, both off), with square and in-circle moves, on capacities 4 and
    7: sweeps bit-exact."""
    bits = {"particle": gpu.FLAG_NO_PARTICLE_SHUFFLE, "set": gpu.FLAG_NO_SET_SHUFFLE,
            "both": gpu.FLAG_NO_PARTICLE_SHUFFLE | gpu.FLAG_NO_SET_SHUFFLE}[ablate]
    for extra in (0, gpu.FLAG_DISK):
        for nx, ny, phi, w_max in ((24, 24, 0.70, math.sqrt(2.0)), (20, 20, 0.72, 1.932)):
            G, O = lattice_pair(gpu, nx, ny, phi, w_max, delta=0.15, n_moves=5, seed=21,
                                flags=FLAGS | bits | extra)
            G.set_fused(False)
            G.set_launch(lanes, 128)
            G.sweep(17)
            O.sweep(17)
            assert_same(G, O, "ablation %s lanes %d flags %d" % (ablate, lanes, bits | extra))


def test_in_circle_and_square_moves_differ(gpu):
    """The flag really switches the proposal: same key, same start, the two
    chains part after the first sweep (and each matches its own oracle)."""
    Gs, Os = lattice_pair(gpu, 24, 24, 0.70, math.sqrt(2.0), delta=0.16, seed=4)
    Gd, Od = lattice_pair(gpu, 24, 24, 0.70, math.sqrt(2.0), delta=0.16, seed=4,
                          flags=FLAGS | gpu.FLAG_DISK)
    for G, O in ((Gs, Os), (Gd, Od)):
        G.sweep(3)
        O.sweep(3)
        assert_same(G, O)
    assert not np.array_equal(Gs.get_state()[0], Gd.get_state()[0])


def test_autotune_leaves_the_chain_alone(gpu):
    G, O = lattice_pair(gpu, 64, 64, 0.70, math.sqrt(2.0), delta=0.12, seed=6)
    lanes, block, us = G.autotune(16)
    assert lanes in (1, 2, 4) and block in (64, 128, 192, 256) and us > 0
    O.sweep(G.AUTOTUNE_CANDIDATES * 2 * 16)
    assert_same(G, O, "autotuned")
    G.sweep(20)
    O.sweep(20)
    assert_same(G, O, "after autotune")


def test_seed_change_and_delta_change(gpu):
    G, O = lattice_pair(gpu, 24, 24, 0.65, 0.0, delta=0.1, seed=1)
    G.sweep(5)
    O.sweep(5)
    G.sweep(5, seed=77)
    O.set_seed(77)
    O.sweep(5)
    assert_same(G, O, "seed")
    G.set_delta(0.25)
    O.set_delta(np.float32(0.25))
    G.sweep(5, seed=77)
    O.sweep(5)
    assert_same(G, O, "delta")
    assert G.delta == np.float32(0.25)


def test_tuner_matches_oracle(gpu):
    G, O = lattice_pair(gpu, 48, 48, 0.70, 0.0, delta=0.02, seed=4)
    window, n = 10, 8
    G.tune(window, n)
    for _ in range(n):
        t0, a0 = O.counters()
        O.sweep(window)
        t1, a1 = O.counters()
        O.set_delta(oracle.tuned_delta(O.delta, t1 - t0, a1 - a0, O.wx, O.wy))
    assert G.delta == O.delta
    assert_same(G, O, "tuned")
    log("  tuned delta %r" % float(G.delta))


@pytest.mark.parametrize("nx,ny,phi,w_max", [(40, 40, 0.70, 0.0), (40, 40, 0.70, math.sqrt(2.0)),
                                             (30, 30, 0.60, 1.932)])
def test_pair_histogram_and_pressure(gpu, nx, ny, phi, w_max):
    G, O = lattice_pair(gpu, nx, ny, phi, w_max, delta=0.15, seed=8)
    hist_o = np.zeros(200, np.uint64)
    G.pair_histogram(reset=True)
    for k in range(6):
        G.sweep(3)
        O.sweep(3)
        G.pair_histogram()
        hist_o += O.pair_histogram()
    # the first GPU sample was the lattice; add it on the oracle side too
    O0 = OracleSystem.lattice(nx, ny, phi, w_max=w_max, delta=0.15, seed=8, flags=FLAGS)
    hist_o += O0.pair_histogram()
    p, g0, hist_g, ns = G.pressure_from_contact()
    assert ns == 7
    assert np.array_equal(hist_g, hist_o)
    Lx, Ly = O.box
    rho = O.N / (Lx * Ly)
    p_ref, g_ref = E.pressure_from_histogram(hist_o, 7, O.N, rho)
    assert abs(g0 - g_ref) <= 1e-9 * abs(g_ref) + 1e-12, (g0, g_ref)
    assert abs(p - p_ref) <= 1e-9 * abs(p_ref), (p, p_ref)
    # single configuration when nothing is accumulated
    G2, O2 = lattice_pair(gpu, nx, ny, phi, w_max, delta=0.15, seed=8)
    G2.sweep(4)
    O2.sweep(4)
    p2, _, h2, n2 = G2.pressure_from_contact()
    assert n2 == 1 and np.array_equal(h2, O2.pair_histogram())


def test_msd_matches(gpu):
    G, O = lattice_pair(gpu, 32, 32, 0.68, 0.0, delta=0.2, seed=12)
    G.sweep(30)
    O.sweep(30)
    acc, _ = O.aux()
    ref = float(np.mean((acc.astype(np.float64) ** 2).sum(axis=1)))
    assert abs(G.msd() - ref) <= 1e-12 * ref
    G.reset_acc()
    O.reset_acc()
    G.sweep(3)
    O.sweep(3)
    assert_same(G, O, "after reset")


def test_tiny_systems(gpu):
    """One and two disks, an empty cell grid apart from them."""
    w = np.float32(1.25)
    for pts in ([[0.6, 0.7]], [[0.3, 0.3], [1.2, 1.1]]):
        xy = np.array(pts, np.float32)
        start = np.zeros(37, np.uint32)
        start[1:] = len(pts)
        O = OracleSystem.grid(6, 6, w, w, delta=np.float32(0.6), n_moves=4, seed=29, flags=FLAGS)
        O.set_state(xy, start)
        G, O = grid_pair(gpu, O, n_moves=4, seed=29, delta=np.float32(0.6))
        G.sweep(40)
        O.sweep(40)
        assert_same(G, O, "tiny %d" % len(pts))


def test_state_errors(gpu):
    from paper_1211_1646_amd import _lib as L
    O = OracleSystem.grid(4, 4, np.float32(1.2), np.float32(1.2), flags=FLAGS)
    cfg = gpu.SystemConfig(cells_x=4, cells_y=4, cell_w_x=1.2, cell_w_y=1.2, n_particles=2,
                           delta=0.1, flags=FLAGS)
    G = gpu.HardDiskSystem(cfg)
    start = np.zeros(17, np.uint32)
    start[1:] = 2
    with pytest.raises(L.MPMCError) as e:      # overlapping pair
        G.set_state(np.array([[0.5, 0.5], [0.9, 0.5]], np.float32), start)
    assert e.value.status == L.MPMC_EOVERLAP
    with pytest.raises(L.MPMCError) as e:      # outside (0, w]
        G.set_state(np.array([[0.0, 0.5], [1.1, 1.1]], np.float32), start)
    assert e.value.status == L.MPMC_ESTATE
    with pytest.raises(L.MPMCError) as e:
        G.subsweep(4)
    assert e.value.status == L.MPMC_EINVAL
    with pytest.raises(L.MPMCError) as e:
        G.shift_and_rebin(0, 0.7)              # d > w/2
    assert e.value.status == L.MPMC_EINVAL
    with pytest.raises(L.MPMCError) as e:
        G.set_delta(0.61)
    assert e.value.status == L.MPMC_EINVAL
    G.set_state(np.array([[0.5, 0.1], [0.5, 1.1]], np.float32), start)   # touching allowed
    assert G.count_overlaps() == 0


def test_medium_workload(gpu):
    """N = 65,536 at phi = 0.70, w in [1, 1.2): 300 sweeps, whole state every
    hundred sweeps, counters every ten."""
    G, O = lattice_pair(gpu, 256, 256, 0.70, 0.0, delta=0.1, seed=1)
    for k in range(30):
        G.sweep(10)
        O.sweep(10)
        assert G.counters() == O.counters(), k
        if (k + 1) % 10 == 0:
            log("  medium sweep %d" % (10 * (k + 1)))
            assert_same(G, O, "medium %d" % (10 * (k + 1)))
    assert G.count_overlaps() == 0


@pytest.mark.parametrize("phi", [0.70, 0.716, 0.720])
def test_large_workload_full_size(gpu, phi):
    """N = 1,048,576 at the benchmark's geometry (w < sqrt(2), capacity 4),
    launched as the benchmark launches it (captured graphs of 16 sweeps):
    the whole state after 16 sweeps equals the oracle's."""
    G, O = lattice_pair(gpu, 1024, 1024, phi, math.sqrt(2.0), delta=0.1, seed=1, flags=0)
    assert_same(G, O, "init")
    G.sweep(16)
    O.sweep(16)
    assert_same(G, O, "16 sweeps")
    assert G.count_overlaps() == O.count_overlaps() == 0


def _paper_pair(gpu, side, seed=1):
    from paper_1211_1646_amd import workloads as W
    w = W.paper_benchmark(side)
    return lattice_pair(gpu, w["nx"], w["ny"], w["phi"], w["w_max"], delta=w["delta"],
                        n_moves=w["n_moves"], seed=seed, flags=gpu.FLAG_DISK)


def test_long_run_loses_nothing(gpu):
    """Sec. 3.2: with each disk's leave/stay decision taken once from one
    rounded value, no disk is lost or duplicated however many shifts run.
    65,536 disks at phi = 0.70 through 100,000 sweeps (100,000 random grid
    shifts, in captured graphs): every identity tag still present exactly
    once, every coordinate inside its cell, every cell within capacity, and
    no overlapping pair."""
    cfg = gpu.SystemConfig(lattice_nx=256, lattice_ny=256, phi=0.70, w_max=math.sqrt(2.0),
                           delta=0.15, n_moves=4, seed=31, flags=gpu.FLAG_TAG)
    G = gpu.HardDiskSystem(cfg)
    G.sweep(100_000)
    xy, st, sw = G.get_state()
    assert sw == 100_000
    _, tags = G.aux()
    N = 256 * 256
    assert len(xy) == N and st[-1] == N
    assert np.array_equal(np.sort(tags), np.arange(N, dtype=np.uint32))
    wx, wy = np.float32(G.geometry["w_x"]), np.float32(G.geometry["w_y"])
    assert np.all(xy[:, 0] > 0) and np.all(xy[:, 0] <= wx)
    assert np.all(xy[:, 1] > 0) and np.all(xy[:, 1] <= wy)
    assert np.all(np.diff(st.astype(np.int64)) <= G.geometry["capacity"])
    assert G.count_overlaps() == 0
    t, a = G.counters()
    assert 0 < a < t
    # the margin of the overlap invariant, measured: the smallest r^2 of any
    # neighbour pair (in the first disk's frame) after 1e5 shifts
    O = oracle.OracleSystem.grid(G.mx, G.my, wx, wy, delta=0.15, n_moves=4, seed=31)
    O.set_state(xy, st, sw)
    r2 = O.min_pair_r2()
    log("  smallest r^2 after 1e5 shifts: 1 - %.3g" % (1.0 - r2))
    assert r2 >= np.float32(1.0) - np.float32(2.0 ** -20)


def test_paper_benchmark_smallest_matches(gpu):
    """The paper's Table 3 benchmark at its smallest N (253^2, run as a
    254 x 252 lattice; in-circle moves of radius 0.16, n_M = 4): 100 warm-up
    sweeps as the benchmark runs them, in the autotuned launch shape, equal
    the oracle's whole state; so do 100 more."""
    G, O = _paper_pair(gpu, 253)
    lanes, block, _ = G.autotune(16)
    O.sweep(G.AUTOTUNE_CANDIDATES * 2 * 16)
    assert_same(G, O, "autotune")
    for k in range(2):
        G.sweep(100)
        O.sweep(100)
        assert_same(G, O, "paper benchmark %d00 sweeps, lanes %d block %d" % (k + 1, lanes, block))
    assert G.count_overlaps() == 0


def test_paper_benchmark_largest_full_size(gpu):
    """N = 9,241,600 (3040^2), the largest Table 3 size, with the paper's
    proposal: the whole state after 8 sweeps (captured graph path) equals the
    oracle's."""
    G, O = _paper_pair(gpu, 3040, seed=2)
    G.sweep(8)
    O.sweep(8)
    assert_same(G, O, "3040^2, 8 sweeps")
    assert G.count_overlaps() == 0


@pytest.mark.parametrize("lanes", [1, 2, 64])
@pytest.mark.parametrize("nx,ny,phi,w_max", [(64, 64, 0.60, 0.0), (20, 20, 0.72, 1.932)])
def test_accept_log_matches_every_sweep(gpu, lanes, nx, ny, phi, w_max):
    """The accept/reject sequence of every cell, sweep after sweep, equals
    the oracle's bit for bit (n_M = 4 and 9)."""
    for n_moves in (4, 9):
        G, O = lattice_pair(gpu, nx, ny, phi, w_max, delta=0.12, n_moves=n_moves, seed=5,
                            flags=FLAGS | 4)
        G.set_fused(False)
        G.set_launch(lanes, 128)
        for k in range(12):
            G.sweep(1)
            O.sweep(1)
            gl, ol = G.accept_log(), O.accept_log()
            assert np.array_equal(gl, ol), (k, int(np.argmax(gl != ol)))
        assert_same(G, O, "accept log run")


def test_n_moves_change_mid_run(gpu):
    """n_M changed between sweeps (graphs re-captured) on both sides."""
    G, O = lattice_pair(gpu, 32, 32, 0.70, math.sqrt(2.0), delta=0.15, n_moves=4, seed=13)
    G.sweep(17)
    O.sweep(17)
    for n in (1, 7, 4):
        G.set_n_moves(n)
        O.set_n_moves(n)
        G.sweep(18)
        O.sweep(18)
        assert_same(G, O, "n_M %d" % n)
