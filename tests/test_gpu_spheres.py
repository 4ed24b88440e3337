"""Parity of the hard-sphere HIP path (through the C ABI) with the 3D CPU
oracle: bit-exact cell lists, positions, tags and counters after sub-sweeps,
shifts and whole sweeps; the contact histogram exactly and the pressure fit
within FP64 rounding.  Needs an MI355X."""
import math
import sys

import numpy as np
import pytest

from oracle import estimator as E
from oracle.spheres import SphereOracle

pytestmark = pytest.mark.gpu


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


def lattice_pair(pkg, n, eta, delta=0.1, n_moves=4, seed=1, replica=0, w_max=0.0, lanes=4,
                 tags=True):
    log("  sphere lattice pair n=%s eta=%.3f delta=%.3f n_moves=%d seed=%d lanes=%d tags=%d"
        % (n, eta, delta, n_moves, seed, lanes, tags))
    cfg = pkg.SphereConfig(lattice_nx=n[0], lattice_ny=n[1], lattice_nz=n[2], eta=eta,
                           w_max=w_max, delta=delta, n_moves=n_moves, seed=seed,
                           replica=replica, flags=pkg.FLAG_TAG if tags else 0)
    G = pkg.HardSphereSystem(cfg)
    G.set_launch(lanes)
    O = SphereOracle.lattice(*n, eta, w_max=w_max, delta=delta, n_moves=n_moves, seed=seed,
                             replica=replica)
    return G, O


def grid_pair(pkg, m, w, xyz, start, tags, sweep=0, delta=0.1, n_moves=4, seed=1, replica=0,
              lanes=4, tagged=True):
    log("  sphere grid pair m=%s N=%d delta=%.3f n_moves=%d lanes=%d"
        % (m, len(xyz), delta, n_moves, lanes))
    cfg = pkg.SphereConfig(cells_x=m[0], cells_y=m[1], cells_z=m[2], cell_w_x=float(w[0]),
                           cell_w_y=float(w[1]), cell_w_z=float(w[2]), n_particles=len(xyz),
                           delta=delta, n_moves=n_moves, seed=seed, replica=replica,
                           flags=pkg.FLAG_TAG if tagged else 0)
    G = pkg.HardSphereSystem(cfg)
    G.set_launch(lanes)
    G.set_state(xyz, start, sweep, tags if tagged else None)
    O = SphereOracle.grid(m, w, len(xyz), delta=delta, n_moves=n_moves, seed=seed,
                          replica=replica)
    O.set_state(xyz, start, tags, sweep)
    return G, O


def assert_same(G, O, what=""):
    gx, gs, gsw, gt = G.get_state(with_tags=True)
    ox, os_, ot, osw = O.get_state()
    assert gsw == osw, (what, gsw, osw)
    assert np.array_equal(gs, os_), "cell lists differ " + what
    assert np.array_equal(gt, ot), "tags differ " + what
    bad = np.nonzero(gx.view(np.uint32) != ox.view(np.uint32))[0]
    assert bad.size == 0, "positions differ %s at %s" % (what, bad[:5])
    assert G.counters() == tuple(O.counters()), (what, G.counters(), O.counters())


def test_lattice_start_matches(gpu):
    for n, eta in [((10, 10, 10), 0.3), ((8, 10, 12), 0.45), ((6, 6, 6), math.pi / 6)]:
        G, O = lattice_pair(gpu, n, eta)
        assert_same(G, O, "start %s" % (n,))
        assert G.count_overlaps() == 0
        G.close()


@pytest.mark.parametrize("eta,n_moves,lanes", [(0.3, 4, 4), (0.45, 7, 1), (0.5, 1, 2), (0.45, 0, 4)])
def test_each_subsweep_and_shift(gpu, eta, n_moves, lanes):
    G, O = lattice_pair(gpu, (12, 10, 14), eta, delta=0.15, n_moves=n_moves, seed=7, lanes=lanes)
    for Q in (5, 0, 3, 6, 1, 7, 2, 4):
        G.subsweep(Q)
        O.subsweep(Q)
        assert_same(G, O, "after set %d" % Q)
    for f in range(6):
        d = np.float32(0.5 * O.w[f // 2] * (0.1 + 0.15 * f))
        G.shift(f, float(d))
        O.shift(f, d)
        assert_same(G, O, "after shift f=%d" % f)
        G.subsweep(f)
        O.subsweep(f)
        assert_same(G, O, "after set %d following shift %d" % (f, f))
    G.close()


def test_shift_by_zero_and_half_a_cell(gpu):
    G, O = lattice_pair(gpu, (10, 10, 10), 0.4, seed=3)
    G.sweep(3)
    O.sweep(3)
    for f, frac in [(0, 0.0), (1, 0.5), (4, 0.5), (5, 0.0), (2, 0.5)]:
        d = np.float32(frac * 0.5 * O.w[f // 2])
        G.shift(f, float(d))
        O.shift(f, d)
        assert_same(G, O, "shift f=%d d=%r" % (f, d))
    G.close()


@pytest.mark.parametrize("n,eta,delta,n_moves,seed,sweeps,lanes", [
    ((10, 10, 10), 0.3, 0.1, 4, 1, 5, 4),
    ((12, 8, 16), 0.45, 0.12, 4, 2, 37, 4),     # 37 = two captured graphs + 5 direct sweeps
    ((12, 8, 16), 0.45, 0.12, 4, 2, 37, 1),
    ((14, 14, 14), 0.5, 0.05, 9, 3, 20, 2),
    ((16, 16, 16), 0.2, 0.3, 3, 4, 17, 4),
    ((10, 10, 10), 0.1, 0.4, 1, 5, 40, 2)])
def test_sweeps_match(gpu, n, eta, delta, n_moves, seed, sweeps, lanes):
    G, O = lattice_pair(gpu, n, eta, delta=delta, n_moves=n_moves, seed=seed, lanes=lanes)
    G.sweep(sweeps)
    O.sweep(sweeps)
    assert_same(G, O, "after %d sweeps" % sweeps)
    assert G.count_overlaps() == 0
    G.close()


def test_set_state_then_continue(gpu):
    G0, O = lattice_pair(gpu, (10, 12, 10), 0.45, delta=0.1, n_moves=4, seed=11)
    G0.close()
    O.sweep(13)
    xyz, start, tags, sweep = O.get_state()
    G, O2 = grid_pair(gpu, O.m, O.w, xyz, start, tags, sweep, delta=0.1, n_moves=4, seed=11)
    assert_same(G, O2, "after set_state")
    G.sweep(19)
    O2.sweep(19)
    assert_same(G, O2, "19 sweeps after set_state")
    G.close()


def test_other_keys_give_other_chains(gpu):
    G1, O1 = lattice_pair(gpu, (10, 10, 10), 0.4, seed=5, replica=0)
    G2, O2 = lattice_pair(gpu, (10, 10, 10), 0.4, seed=5, replica=1)
    for G, O in ((G1, O1), (G2, O2)):
        G.sweep(4)
        O.sweep(4)
        assert_same(G, O, "keyed")
    assert not np.array_equal(G1.get_state()[0], G2.get_state()[0])
    G1.close()
    G2.close()


def fcc_state(cells_fcc, eta, offset=0.137):
    """A face-centred cubic crystal (4 spheres per cubic unit cell) at packing
    fraction eta in a periodic box, in cells of the smallest even count per
    axis narrower than 2/sqrt(3), as compact lists with lattice tags."""
    rho = 6.0 * eta / math.pi
    a = (4.0 / rho) ** (1.0 / 3.0)
    L = cells_fcc * a
    limit = 2.0 / math.sqrt(3.0) * (1.0 - 1e-5)
    m = int(math.ceil(L / limit))
    m += m & 1
    while L / m >= limit:
        m += 2
    w = np.float32(L / m)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.array([(i, j, k) for k in range(cells_fcc) for j in range(cells_fcc)
                  for i in range(cells_fcc)], np.float64)
    pts = ((g[:, None, :] + basis[None, :, :]).reshape(-1, 3) + offset) * a
    pts = np.mod(pts, m * np.float64(w))
    cell3 = np.clip(np.ceil(pts / np.float64(w)).astype(np.int64) - 1, 0, m - 1)
    loc = (pts - cell3 * np.float64(w)).astype(np.float32)
    assert (loc > 0).all() and (loc <= w).all()
    cell = (cell3[:, 2] * m + cell3[:, 1]) * m + cell3[:, 0]
    order = np.argsort(cell, kind="stable")
    counts = np.bincount(cell, minlength=m ** 3)
    start = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    return (m, m, m), np.float32([w, w, w]), loc[order], start, order.astype(np.uint32)


def trial_box_counts(m, w, xyz, start, n_moves, delta):
    """Per occupied cell, the spheres of its 26 neighbours whose squared
    distance is below 1.0001 to the box that holds every trial position of
    the cell's update (the own spheres' bounding box grown by
    ceil(n_M / n) (delta + 2e-7) + 1e-5 and cut to the cell): the length of
    the sub-sweep's neighbour list for a lane per cell."""
    w = float(w[0])
    M = m[0]
    counts = np.diff(start.astype(np.int64))
    cell_of = np.repeat(np.arange(M ** 3), counts)
    cz, cy, cx = cell_of // (M * M), (cell_of // M) % M, cell_of % M
    gpos = np.stack([cx * w + xyz[:, 0], cy * w + xyz[:, 1], cz * w + xyz[:, 2]], 1)
    Lb = M * w
    out = np.zeros(M ** 3, np.int64)
    for c in range(M ** 3):
        n = counts[c]
        if n == 0:
            continue
        own = xyz[start[c]:start[c + 1]].astype(np.float64)
        e = -(-n_moves // n) * (delta + 2e-7) + 1e-5
        lo, hi = np.maximum(own.min(0) - e, 0.0), np.minimum(own.max(0) + e, w)
        z, y, x = c // (M * M), (c // M) % M, c % M
        d = gpos - np.array([x * w, y * w, z * w])
        d -= Lb * np.round((d - w / 2) / Lb)          # nearest image around the cell
        gap = np.maximum(0.0, np.maximum(lo - d, d - hi))
        out[c] = (((gap ** 2).sum(1) < 1.0001) & (cell_of != c)).sum()
    return out


@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_dense_crystal_exercises_the_spill_path(gpu, lanes):
    """An FCC crystal at eta = 0.70 with n_M = 16 puts more reachable
    neighbours around many cells than the 32-entry list of a lane per cell
    holds; those lanes also test every neighbour straight from memory.  The
    same dense state runs with two and four lanes per cell (lists of 24 and
    16 over a half and a quarter of the neighbour cells).  The chain must be
    bit-exact in every case."""
    m, w, xyz, start, tags = fcc_state(8, 0.70)
    K = trial_box_counts(m, w, xyz, start, 16, 0.05)
    log("  neighbour list per cell: max %d, cells above 32: %d" % (K.max(), (K > 32).sum()))
    assert (K > 32).sum() > 10
    G, O = grid_pair(gpu, m, w, xyz, start, tags, 0, delta=0.05, n_moves=16, seed=9, lanes=lanes)
    G.sweep(3)
    O.sweep(3)
    assert_same(G, O, "dense crystal, 3 sweeps")
    assert G.counters()[1] > 0
    G.sweep(16)
    O.sweep(16)
    assert_same(G, O, "dense crystal, 19 sweeps")
    G.close()


def region_overflow_cells(m, start):
    """Per brick region of the one-lane form (4^3 active cells of a set and
    their neighbours, 9^3 cells with periodic indices), for every set, the
    number of cells holding more than two spheres."""
    M = m[0]
    cnt = np.diff(start.astype(np.int64)).reshape(M, M, M)   # [z][y][x]
    nb = (M // 2 + 3) // 4
    out = []
    for Q in range(8):
        q = (Q & 1, (Q >> 1) & 1, Q >> 2)
        for bz in range(nb):
            for by in range(nb):
                for bx in range(nb):
                    ix = (np.arange(9) + 8 * bx + q[0] - 1) % M
                    iy = (np.arange(9) + 8 * by + q[1] - 1) % M
                    iz = (np.arange(9) + 8 * bz + q[2] - 1) % M
                    out.append(int((cnt[np.ix_(iz, iy, ix)] > 2).sum()))
    return np.array(out)


def test_dense_crystal_on_the_untagged_brick_form(gpu):
    """The dense crystal on the kernel variant the benchmark runs (one lane
    per cell, no tags): brick regions with more than 64 cells of more than
    two spheres load those cells' slots in several rounds, and regions with
    more than the 128 cells the brick lists send every lane to the
    from-memory path.  Bit-exact either way."""
    m, w, xyz, start, tags = fcc_state(8, 0.70)
    k = region_overflow_cells(m, start)
    log("  cells past two spheres per region: max %d, regions above 64: %d, above 128: %d"
        % (k.max(), (k > 64).sum(), (k > 128).sum()))
    assert ((k > 64) & (k <= 128)).any() and (k > 128).any()
    G, O = grid_pair(gpu, m, w, xyz, start, tags, 0, delta=0.05, n_moves=16, seed=9, lanes=1,
                     tagged=False)
    G.sweep(3)
    O.sweep(3)
    assert_same_untagged(G, O, "dense crystal, untagged, 3 sweeps")
    G.sweep(16)
    O.sweep(16)
    assert_same_untagged(G, O, "dense crystal, untagged, 19 sweeps")
    G.close()


def test_launch_shapes_give_one_chain(gpu):
    """Lanes per cell change only how the work is split: 1, 2 and 4 give the
    same state bit for bit, from the lattice and across launch-shape changes
    in the middle of a run."""
    states = []
    for lanes in (1, 2, 4):
        G, _ = lattice_pair(gpu, (12, 12, 12), 0.45, delta=0.08, n_moves=5, seed=21, lanes=lanes)
        G.sweep(9)
        G.set_launch(1 if lanes == 4 else 4)
        G.sweep(20)
        states.append(G.get_state(with_tags=True) + (G.counters(),))
        G.close()
    for st in states[1:]:
        assert np.array_equal(st[0].view(np.uint32), states[0][0].view(np.uint32))
        assert np.array_equal(st[1], states[0][1]) and np.array_equal(st[3], states[0][3])
        assert st[2] == states[0][2] and st[4] == states[0][4]


@pytest.mark.parametrize("window", [10, 17])
def test_plain_tuner_matches_the_oracle(gpu, window):
    """mpmc_sphere_tune against the oracle stepped window by window with the
    tuner rule (the disks' rule with the smallest of the three widths); a
    17-sweep window runs one captured graph and one direct sweep."""
    from oracle import tuned_delta
    G, O = lattice_pair(gpu, (12, 12, 12), 0.45, delta=0.3, n_moves=4, seed=23)
    G.tune(window, 5)
    deltas = [O.delta]
    for _ in range(5):
        t0, a0 = O.counters()
        O.sweep(window)
        t1, a1 = O.counters()
        O.set_delta(tuned_delta(O.delta, t1 - t0, a1 - a0, min(O.w[0], O.w[1]), O.w[2]))
        deltas.append(O.delta)
    log("  delta by window: %s" % ", ".join("%.5f" % d for d in deltas))
    assert G.delta() == O.delta and O.delta != deltas[0]
    assert_same(G, O, "after tuning")
    G.sweep(7)
    O.sweep(7)
    assert_same(G, O, "7 sweeps after tuning")
    G.close()


@pytest.mark.parametrize("lanes", [1, 4])
def test_accumulators_and_msd_match_the_oracle(gpu, lanes):
    """MPMC_FLAG_ACC: the accumulators bit for bit against the oracle's (S10)
    after sweeps through graphs and shifts, the device MSD against the FP64
    mean of the oracle's accumulators, and reset_acc."""
    n, eta = (12, 10, 14), 0.45
    cfg = gpu.SphereConfig(lattice_nx=n[0], lattice_ny=n[1], lattice_nz=n[2], eta=eta, delta=0.12,
                           n_moves=5, seed=31, flags=gpu.FLAG_TAG | gpu.FLAG_ACC)
    G = gpu.HardSphereSystem(cfg)
    G.set_launch(lanes)
    O = SphereOracle.lattice(*n, eta, delta=0.12, n_moves=5, seed=31)
    assert not G.acc().any()
    G.sweep(37)
    O.sweep(37)
    assert_same(G, O, "with accumulators")
    ga, oa = G.acc(), O.acc()
    assert np.abs(oa).max() > 0.1
    assert np.array_equal(ga.view(np.uint32), oa.view(np.uint32)), "accumulators differ"
    ref = float(np.mean(np.sum(oa.astype(np.float64) ** 2, axis=1)))
    assert abs(G.msd() - ref) <= 1e-12 * ref
    G.reset_acc()
    assert not G.acc().any() and G.msd() == 0.0
    G.close()


def test_pair_histogram_and_pressure(gpu):
    G, O = lattice_pair(gpu, (12, 12, 12), 0.4, delta=0.15, n_moves=4, seed=13)
    hist = np.zeros(200, np.float64)
    for k in range(6):
        G.sweep(10)
        O.sweep(10)
        G.pair_histogram(reset=(k == 0))
        hist += O.pair_histogram()
    p, g0, gh, ns = G.pressure()
    assert ns == 6
    assert np.array_equal(gh, hist.astype(np.uint64))
    rho = G.density
    p_ref, g_ref = E.pressure_from_histogram_3d(hist, 6, G.N, rho)
    log("  P %.6f (oracle %.6f), g %.6f (oracle %.6f)" % (p, p_ref, g0, g_ref))
    assert abs(g0 - g_ref) <= 1e-9 * abs(g_ref)
    assert abs(p - p_ref) <= 1e-9 * abs(p_ref)
    G.close()


def assert_same_untagged(G, O, what=""):
    gx, gs, gsw = G.get_state()
    ox, os_, _, osw = O.get_state()
    assert gsw == osw, (what, gsw, osw)
    assert np.array_equal(gs, os_), "cell lists differ " + what
    bad = np.nonzero(gx.view(np.uint32) != ox.view(np.uint32))[0]
    assert bad.size == 0, "positions differ %s at %s" % (what, bad[:5])
    assert G.counters() == tuple(O.counters()), (what, G.counters(), O.counters())


@pytest.mark.parametrize("lanes,tags", [(1, False), (1, True), (4, True)])
def test_full_size_one_million_spheres(gpu, lanes, tags):
    """The benchmark configuration (100^3 spheres at eta = 0.45, n_M = 4),
    compared in full after three sweeps (the oracle takes about half a second
    per sweep at this size): the brick form without and with tags (the
    first sweeps from the lattice, whose cells of four and eight spheres
    send lanes to the from-memory path), and the four-lane form."""
    G, O = lattice_pair(gpu, (100, 100, 100), 0.45, delta=0.1, n_moves=4, seed=1, lanes=lanes,
                        tags=tags)
    G.sweep(3)
    O.sweep(3)
    (assert_same if tags else assert_same_untagged)(G, O, "1M spheres, 3 sweeps")
    G.close()


@pytest.mark.parametrize("n,eta,delta,n_moves,sweeps", [
    ((4, 4, 4), 0.4, 0.15, 4, 25),        # a 4^3-cell grid: one brick, its region wraps twice
    ((4, 6, 20), 0.35, 0.12, 5, 19),      # one, one and three bricks per axis
    ((12, 8, 16), 0.45, 0.12, 4, 37),     # ragged bricks; two captured graphs + 5 direct sweeps
    ((50, 50, 50), 0.45, 0.1, 4, 4),      # the benchmark's spheres per cell, from the lattice
    ((14, 14, 14), 0.5, 0.05, 9, 20)])
def test_brick_form_without_tags(gpu, n, eta, delta, n_moves, sweeps):
    """The default one-lane form as the benchmark runs it (no tags, no
    accumulators: the kernel variant that carries neither), bit-exact."""
    G, O = lattice_pair(gpu, n, eta, delta=delta, n_moves=n_moves, seed=6, lanes=1, tags=False)
    log("  grid %s" % (G.m,))
    G.sweep(sweeps)
    O.sweep(sweeps)
    assert_same_untagged(G, O, "brick, %d sweeps" % sweeps)
    assert G.count_overlaps() == 0
    G.close()


def test_argument_errors(gpu):
    from paper_1211_1646_amd import _lib as L
    G, _ = lattice_pair(gpu, (10, 10, 10), 0.3)
    for call in (lambda: G.subsweep(8), lambda: G.subsweep(-1), lambda: G.shift(6, 0.1),
                 lambda: G.shift(0, 0.6), lambda: G.set_delta(0.6), lambda: G.set_delta(0.0),
                 lambda: G.set_launch(3), lambda: G.set_launch(8), lambda: G.tune(0, 1),
                 lambda: G.tune(5, -1), lambda: G.acc(), lambda: G.msd(), lambda: G.reset_acc()):
        with pytest.raises(L.MPMCError) as e:
            call()
        assert e.value.status == L.MPMC_EINVAL
    xyz, start, _ = G.get_state()
    # two spheres in x-neighbouring cells of one row, moved 0.01 apart
    counts = np.diff(start.astype(np.int64))
    M = G.m[0]
    pair = next(c for c in range(G.C - 1)
                if c % M != M - 1 and counts[c] >= 1 and counts[c + 1] >= 1)
    a, b = int(start[pair]), int(start[pair + 1])
    bad = xyz.copy()
    bad[a, 0] = G.w[0]
    bad[b] = (np.float32(0.01), bad[a, 1], bad[a, 2])
    with pytest.raises(L.MPMCError) as e:
        G.set_state(bad, start, 0)
    assert e.value.status == L.MPMC_EOVERLAP
    bad = xyz.copy()
    bad[0, 2] = 5.0
    with pytest.raises(L.MPMCError) as e:
        G.set_state(bad, start, 0)
    assert e.value.status == L.MPMC_ESTATE
    G.close()


def test_low_density_equation_of_state_on_the_gpu(gpu):
    """The GPU chain's own pressure, from its device histogram and fit, at
    eta = 0.1 against the hard-sphere virial series 1 + 4 eta + 10 eta^2 +
    18.36 eta^3 + ... (1.5216); 32^3 spheres, 20 blocks of 100 histograms."""
    from oracle import estimator as E
    eta = 0.10
    cfg = gpu.SphereConfig(lattice_nx=32, lattice_ny=32, lattice_nz=32, eta=eta, delta=0.55,
                           n_moves=4, seed=17)
    G = gpu.HardSphereSystem(cfg)
    G.sweep(200)
    rho = G.density
    P = []
    for b in range(20):
        for k in range(100):
            G.sweep(2)
            G.pair_histogram(reset=(k == 0))
        p, _, _, ns = G.pressure()
        assert ns == 100
        P.append(p / rho)
    m, se = E.mean_and_error(P, min_blocks=8)
    log("  beta P / rho = %.5f +- %.5f, virial series %.5f" % (m, se, E.virial_pressure_ratio_3d(eta)))
    assert abs(m - E.virial_pressure_ratio_3d(eta)) < 4 * se + 2e-3, (m, se)
    assert m - 1.4 > 3 * se
    assert G.count_overlaps() == 0
    G.close()


def klm_pressure_ratio(eta):
    """Compressibility factor of the hard-sphere fluid from the equation of
    state of Kolafa, Labik and Malijevsky (2004):
    (1 + eta + eta^2 - 2/3 eta^3 (1 + eta)) / (1 - eta)^3, within about 0.02 %
    of simulation in the stable fluid."""
    return (1 + eta + eta ** 2 - 2.0 / 3.0 * eta ** 3 * (1 + eta)) / (1 - eta) ** 3


def test_dense_fluid_equation_of_state_on_the_gpu(gpu):
    """The GPU chain's own pressure at the benchmark's packing fraction,
    eta = 0.45 (64^3 spheres from the lattice, the plain tuner, 2 x 10^4
    sweeps, then 20 blocks of 100 histograms every 5 sweeps), against the
    dense-fluid equation of state (Z = 9.4029), within four standard errors
    plus 0.05 % (Carnahan-Starling's 9.3847 is 0.2 % lower)."""
    from oracle import estimator as E
    eta = 0.45
    cfg = gpu.SphereConfig(lattice_nx=64, lattice_ny=64, lattice_nz=64, eta=eta, delta=0.09,
                           n_moves=4, seed=1)
    G = gpu.HardSphereSystem(cfg)
    G.tune(10, 20)
    G.sweep(20000)
    rho = G.density
    P = []
    for b in range(20):
        for k in range(100):
            G.sweep(5)
            G.pair_histogram(reset=(k == 0))
        p, _, _, ns = G.pressure()
        assert ns == 100
        P.append(p / rho)
    m, se = E.mean_and_error(P, min_blocks=8)
    ref = klm_pressure_ratio(eta)
    log("  beta P / rho = %.5f +- %.5f, dense-fluid equation of state %.5f" % (m, se, ref))
    assert abs(m - ref) < 4 * se + 5e-4 * ref, (m, se, ref)
    assert G.count_overlaps() == 0
    G.close()

