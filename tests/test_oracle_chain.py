"""Pins for the oracle's checkerboard chain (Alg. 1, 2, 4 of the paper):
invariants, independence of the cell order, the cell shift, the particle
shuffle and closed-form equilibrium results for one and two disks.  CPU only."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import OracleSystem
from oracle import estimator as E


def _global_fp64(S):
    gx, gy = S.global_positions()
    return gx, gy


def _min_pair_distance(S):
    """Smallest minimum-image distance over all pairs, brute force FP64."""
    gx, gy = _global_fp64(S)
    Lx, Ly = S.box
    dx = gx[:, None] - gx[None, :]
    dy = gy[:, None] - gy[None, :]
    dx -= Lx * np.round(dx / Lx)
    dy -= Ly * np.round(dy / Ly)
    r2 = dx * dx + dy * dy
    np.fill_diagonal(r2, np.inf)
    return float(np.sqrt(r2.min()))


# ---------------------------------------------------------------- lattice
def test_lattice_initial_state():
    nx = ny = 16
    phi = 0.70
    S = OracleSystem.lattice(nx, ny, phi, flags=OracleSystem.FLAG_TAG)
    xy, start, sweep = S.get_state()
    assert sweep == 0 and S.N == nx * ny and start[-1] == nx * ny
    assert np.all(xy[:, 0] > 0) and np.all(xy[:, 0] <= S.wx)
    assert np.all(xy[:, 1] > 0) and np.all(xy[:, 1] <= S.wy)
    assert S.count_overlaps() == 0
    # lattice sites, FP64: spacing a with N a^2 sqrt(3)/2 = N pi / (4 phi)
    a = math.sqrt(math.pi / (4 * phi) * 2 / math.sqrt(3))
    _, tag = S.aux()
    gx, gy = _global_fp64(S)
    i, j = tag % nx, tag // nx
    assert np.allclose(gx, (i + 0.25 + 0.5 * (j % 2)) * a, atol=2e-6, rtol=0)
    assert np.allclose(gy, (j + 0.5) * a * math.sqrt(3) / 2, atol=2e-6, rtol=0)
    # within a cell: ascending lattice index
    for c in range(S.C):
        t = tag[start[c]:start[c + 1]]
        assert np.all(np.diff(t.astype(np.int64)) > 0)
    # nearest-neighbour distance of the lattice
    assert abs(_min_pair_distance(S) - a) < 1e-5


# ------------------------------------------------------------- invariants
@pytest.mark.parametrize("phi,w_max", [(0.70, 0.0), (0.70, math.sqrt(2.0)), (0.45, 1.932)])
def test_invariants_every_sweep(phi, w_max):
    S = OracleSystem.lattice(20, 20, phi, w_max=w_max, delta=0.2, n_moves=4, seed=11,
                             flags=OracleSystem.FLAG_TAG | OracleSystem.FLAG_ACC)
    N = S.N
    for k in range(60):
        S.sweep(1)
        xy, start, sweep = S.get_state()
        assert sweep == k + 1
        assert start[-1] == N and np.all(np.diff(start.astype(np.int64)) >= 0)
        assert np.diff(start.astype(np.int64)).max() <= S.cap
        assert np.all(xy[:, 0] > 0) and np.all(xy[:, 0] <= S.wx)
        assert np.all(xy[:, 1] > 0) and np.all(xy[:, 1] <= S.wy)
        _, tag = S.aux()
        assert np.array_equal(np.sort(tag), np.arange(N, dtype=np.uint32))
        assert S.count_overlaps() == 0
    assert _min_pair_distance(S) > 1.0 - 1e-6
    t, a = S.counters()
    assert 0 < a < t


def test_trial_count_is_n_moves_per_nonempty_active_cell():
    S = OracleSystem.lattice(24, 24, 0.5, delta=0.2, n_moves=3, seed=5)
    for Q in range(4):
        _, start, _ = S.get_state()
        cnt = np.diff(start.astype(np.int64)).reshape(S.my, S.mx)
        active = cnt[(Q >> 1)::2, (Q & 1)::2]
        t0, _ = S.counters()
        S.subsweep(Q)
        t1, _ = S.counters()
        assert t1 - t0 == 3 * int((active > 0).sum())


def test_cell_order_does_not_matter():
    """Cells of one set are independent (w >= sigma, Sec. 2.1): visiting them
    in another order gives a bit-identical chain."""
    states = []
    for mode in (0, 1, 2):
        S = OracleSystem.lattice(24, 24, 0.70, delta=0.15, n_moves=4, seed=3,
                                 flags=OracleSystem.FLAG_TAG | OracleSystem.FLAG_ACC)
        S.set_cell_order(mode)
        S.sweep(25)
        xy, start, _ = S.get_state()
        acc, tag = S.aux()
        states.append((xy, start, acc, tag, S.counters()))
    for other in states[1:]:
        for a, b in zip(states[0][:4], other[:4]):
            assert np.array_equal(a, b)
        assert states[0][4] == other[4]


def test_checkpoint_resume_is_exact():
    kw = dict(delta=0.12, n_moves=4, seed=9, flags=OracleSystem.FLAG_TAG)
    A = OracleSystem.lattice(16, 16, 0.68, **kw)
    A.sweep(30)
    B = OracleSystem.lattice(16, 16, 0.68, **kw)
    B.sweep(15)
    xy, start, sweep = B.get_state()
    _, tag = B.aux()
    Cs = OracleSystem.grid(B.mx, B.my, B.wx, B.wy, **kw)
    Cs.set_state(xy, start, sweep, tag)
    Cs.sweep(15)
    for a, b in zip(A.get_state(), Cs.get_state()):
        assert np.array_equal(a, b)
    assert np.array_equal(A.aux()[1], Cs.aux()[1])


def test_set_state_rejects_bad_states():
    S = OracleSystem.grid(4, 4, np.float32(1.2), np.float32(1.2))
    start = np.zeros(17, np.uint32)
    start[1:] = 1
    with pytest.raises(ValueError):   # x outside (0, w]
        S.set_state(np.array([[0.0, 0.5]], np.float32), start)
    with pytest.raises(ValueError):   # above capacity
        start2 = np.zeros(17, np.uint32)
        start2[1:] = 5
        S.set_state(np.full((5, 2), 0.5, np.float32), start2)


# ---------------------------------------------------------------- shift
def _tagged_globals(S):
    gx, gy = _global_fp64(S)
    _, tag = S.aux()
    order = np.argsort(tag)
    return gx[order], gy[order]


@pytest.mark.parametrize("f", [0, 1, 2, 3])
def test_shift_translates_every_particle(f):
    """Alg. 4: moving the grid by +f d is moving every disk by -f d."""
    S = OracleSystem.lattice(20, 20, 0.7, delta=0.2, seed=2, flags=OracleSystem.FLAG_TAG)
    S.sweep(10)
    Lx, Ly = S.box
    rng = np.random.default_rng(f)
    for _ in range(20):
        w = S.wx if f < 2 else S.wy
        d = np.float32(rng.uniform(0, 0.5 * w))
        gx0, gy0 = _tagged_globals(S)
        S.shift(f, d)
        gx1, gy1 = _tagged_globals(S)
        sgn = 1.0 if f in (0, 2) else -1.0
        ex = gx0 - (sgn * float(d) if f < 2 else 0.0)
        ey = gy0 - (sgn * float(d) if f >= 2 else 0.0)
        ddx = (gx1 - ex + Lx / 2) % Lx - Lx / 2
        ddy = (gy1 - ey + Ly / 2) % Ly - Ly / 2
        assert np.abs(ddx).max() < 1e-5 and np.abs(ddy).max() < 1e-5
        assert S.N == 400 and S.count_overlaps() == 0


def test_shift_edge_values():
    """Stay iff the shifted coordinate lies in (0, w]: t = 0 leaves, t = w stays."""
    w = np.float32(1.25)
    S = OracleSystem.grid(4, 4, w, w, flags=OracleSystem.FLAG_TAG)
    start = np.zeros(17, np.uint32)
    start[1:] = 2   # both disks in cell 0
    d = np.float32(0.5)
    xy = np.array([[0.5, 0.1], [1.25, 1.25]], np.float32)  # x - d = 0 exactly; x - d = 0.75
    S.set_state(xy, start)
    S.shift(0, d)                                           # +x
    nxy, nstart, _ = S.get_state()
    cnt = np.diff(nstart.astype(np.int64))
    assert cnt[0] == 1 and cnt[3] == 1                      # the t = 0 disk went to cell cx = -1 = 3
    assert nxy[nstart[0], 0] == np.float32(0.75)
    assert nxy[nstart[3], 0] == w                           # 0 + w
    # -x: x + d = w exactly stays
    S2 = OracleSystem.grid(4, 4, w, w, flags=OracleSystem.FLAG_TAG)
    S2.set_state(np.array([[0.75, 0.1], [0.8, 1.2]], np.float32), start)
    S2.shift(1, d)
    nxy, nstart, _ = S2.get_state()
    cnt = np.diff(nstart.astype(np.int64))
    assert cnt[0] == 1 and cnt[1] == 1
    assert nxy[nstart[0], 0] == w                            # 0.75 + 0.5 = w stays
    assert nxy[nstart[1], 0] == (np.float32(0.8) + d) - w    # t - w, exact (Sterbenz)
    # d = 0 is the identity
    S3 = OracleSystem.lattice(12, 12, 0.7, flags=OracleSystem.FLAG_TAG)
    before = S3.get_state()
    S3.shift(2, np.float32(0.0))
    after = S3.get_state()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])


def test_many_shifts_lose_nothing():
    """Sec. 3.2: with one rounded comparison per disk no disk is ever lost."""
    S = OracleSystem.lattice(24, 24, 0.72, delta=0.1, seed=4, flags=OracleSystem.FLAG_TAG)
    rng = np.random.default_rng(7)
    fs = rng.integers(0, 4, 20000)
    us = rng.uniform(0, 1, 20000).astype(np.float32)
    for f, u in zip(fs, us):
        w = S.wx if f < 2 else S.wy
        S.shift(int(f), u * np.float32(0.5) * w)
    _, tag = S.aux()
    assert np.array_equal(np.sort(tag), np.arange(24 * 24, dtype=np.uint32))
    assert S.count_overlaps() == 0


# ------------------------------------------------------------- shuffling
def test_particle_shuffle_is_uniform():
    """Alg. 1: with n_M = 0 a sub-sweep only permutes each active cell;
    over many cells and sweeps all n! orders of n = 2, 3, 4 particles are
    equally likely (chi-square)."""
    S = OracleSystem.lattice(48, 48, 0.72, w_max=1.932, n_moves=0, seed=21,
                             flags=OracleSystem.FLAG_TAG)
    counts = {n: {} for n in (2, 3, 4)}
    for sweep in range(60):
        for Q in range(4):
            _, start, _ = S.get_state()
            _, tag0 = S.aux()
            S.subsweep(Q)
            _, tag1 = S.aux()
            cnt = np.diff(start.astype(np.int64))
            cells = [c for c in range(S.C) if ((c % S.mx) & 1) + 2 * ((c // S.mx) & 1) == Q
                     and 2 <= cnt[c] <= 4]
            for c in cells:
                a, b = tag0[start[c]:start[c + 1]], tag1[start[c]:start[c + 1]]
                perm = tuple(int(np.where(a == t)[0][0]) for t in b)
                counts[cnt[c]][perm] = counts[cnt[c]].get(perm, 0) + 1
        # advance the sweep counter (new streams) with a real sweep
        S.set_n_moves(4)
        S.sweep(1)
        S.set_n_moves(0)
    from scipy.stats import chi2
    for n, table in counts.items():
        perms = list(itertools.permutations(range(n)))
        obs = np.array([table.get(p, 0) for p in perms], float)
        total = obs.sum()
        assert total > 20 * len(perms), (n, total)
        exp = total / len(perms)
        stat = ((obs - exp) ** 2 / exp).sum()
        assert chi2.sf(stat, len(perms) - 1) > 1e-4, (n, stat, obs)


def test_set_order_is_uniform_and_shift_is_uniform():
    S = OracleSystem.lattice(8, 8, 0.5)
    orders, fs, ds = {}, [], []
    for s in range(24000):
        order, f, d = S.draws(s)
        orders[tuple(order)] = orders.get(tuple(order), 0) + 1
        fs.append(f)
        ds.append(float(d) / (0.5 * float(S.wx if f < 2 else S.wy)))
    from scipy.stats import chi2, kstest
    obs = np.array(list(orders.values()), float)
    assert len(orders) == 24
    assert chi2.sf(((obs - 1000) ** 2 / 1000).sum(), 23) > 1e-4
    fc = np.bincount(fs, minlength=4)
    assert chi2.sf(((fc - 6000) ** 2 / 6000).sum(), 3) > 1e-4
    assert min(ds) >= 0 and max(ds) < 1
    assert kstest(ds, "uniform").pvalue > 1e-4


def test_set_shuffle_ablation_fixes_the_order_only():
    """Without the set shuffle (Table 1's "CB. No") the sets run a, b, c, d
    in every sweep, while the shift direction and distance are the ones the
    shuffled chain draws for the same sweep and key."""
    A = OracleSystem.lattice(8, 8, 0.5)
    B = OracleSystem.lattice(8, 8, 0.5, flags=OracleSystem.FLAG_NO_SET_SHUFFLE)
    orders = set()
    for s in range(500):
        oa, fa, da = A.draws(s)
        ob, fb, db = B.draws(s)
        orders.add(tuple(oa))
        assert ob == [0, 1, 2, 3]
        assert (fa, da) == (fb, db)
    assert len(orders) == 24


def _moved_tags(flags, sweeps=3000):
    """One cell of three well-separated disks, one trial per cell: the tag
    of the disk each accepted trial moved, and whether storage order held."""
    w = np.float32(1.9)
    S = OracleSystem.grid(4, 4, w, w, delta=np.float32(0.05), n_moves=1, seed=41,
                          flags=OracleSystem.FLAG_TAG | flags)
    xy = np.array([[0.3, 0.3], [1.5, 0.3], [0.3, 1.5]], np.float32)
    start = np.zeros(17, np.uint32)
    start[1:] = 3
    tag = np.array([10, 11, 12], np.uint32)
    moved, kept_order = [], True
    for k in range(sweeps):
        S.set_state(xy, start, sweep=k, tag=tag)
        S.subsweep(0)
        xy1, _, _ = S.get_state()
        _, tag1 = S.aux()
        kept_order &= bool(np.array_equal(tag1, tag))
        for j in range(3):
            i = int(np.nonzero(tag == tag1[j])[0][0])
            if not np.array_equal(xy1[j], xy[i]):
                moved.append(int(tag1[j]))
    return moved, kept_order


def test_particle_shuffle_ablation_visits_in_stored_order():
    """Without the particle shuffle (Table 1's "P. No") the one trial of a
    cell always goes to the first disk of the stored list, and the list is
    not reordered; with it, each of the three disks is chosen a third of the
    time (chi-square) and the stored order changes."""
    from scipy.stats import chi2
    moved, kept = _moved_tags(OracleSystem.FLAG_NO_PARTICLE_SHUFFLE)
    assert kept and len(moved) > 2500 and set(moved) == {10}
    moved, kept = _moved_tags(0)
    assert not kept
    cnt = np.bincount(np.array(moved) - 10, minlength=3).astype(float)
    e = cnt.sum() / 3
    assert chi2.sf(((cnt - e) ** 2 / e).sum(), 2) > 1e-4


# ------------------------------------------------- closed-form equilibria
def test_single_disk_acceptance_closed_form():
    """One disk, uniformly placed in its cell, displaced uniformly in the
    square: the move stays in the cell with probability
    (1 - delta / (2 wx)) (1 - delta / (2 wy)), and nothing else can reject it."""
    wx, wy = np.float32(1.2), np.float32(1.5)
    delta = np.float32(0.5)
    S = OracleSystem.grid(4, 6, wx, wy, delta=delta, n_moves=4, seed=17)
    start = np.zeros(25, np.uint32)
    start[1:] = 1
    S.set_state(np.array([[0.6, 0.7]], np.float32), start)
    S.sweep(200)
    t0, a0 = S.counters()
    S.sweep(100000)
    t1, a1 = S.counters()
    n = t1 - t0
    p_hat = (a1 - a0) / n
    p = (1 - float(delta) / (2 * float(wx))) * (1 - float(delta) / (2 * float(wy)))
    # moves of one disk are correlated through its position: allow 5 binomial SE x 2
    se = math.sqrt(p * (1 - p) / n)
    assert abs(p_hat - p) < 10 * se, (p_hat, p, se)
    assert n == 4 * 100000


def test_single_disk_acceptance_closed_form_in_circle():
    """One disk, uniformly placed in its cell, displaced uniformly in the
    disk of radius delta (the paper's proposal): with |dx|, |dy| <= delta <=
    w/2 the move stays in the cell with probability
    E[(1 - |dx|/wx)(1 - |dy|/wy)] = 1 - 4 delta/(3 pi) (1/wx + 1/wy)
    + delta^2 / (2 pi wx wy), since E|dx| = 4 delta / (3 pi) and
    E|dx dy| = delta^2 / (2 pi) for a uniform point of the disk."""
    wx, wy = np.float32(1.2), np.float32(1.5)
    delta = np.float32(0.5)
    S = OracleSystem.grid(4, 6, wx, wy, delta=delta, n_moves=4, seed=17,
                          flags=OracleSystem.FLAG_DISK)
    start = np.zeros(25, np.uint32)
    start[1:] = 1
    S.set_state(np.array([[0.6, 0.7]], np.float32), start)
    S.sweep(200)
    t0, a0 = S.counters()
    S.sweep(100000)
    t1, a1 = S.counters()
    n = t1 - t0
    p_hat = (a1 - a0) / n
    d, x, y = float(delta), float(wx), float(wy)
    p = 1 - 4 * d / (3 * math.pi) * (1 / x + 1 / y) + d * d / (2 * math.pi * x * y)
    se = math.sqrt(p * (1 - p) / n)
    assert abs(p_hat - p) < 10 * se, (p_hat, p, se)
    # the square proposal's rate would be far off: the two are told apart
    p_sq = (1 - d / (2 * x)) * (1 - d / (2 * y))
    assert abs(p_hat - p_sq) > 30 * se


def test_single_disk_in_circle_displacements():
    """Accepted in-circle moves of a lone disk deep inside a wide cell are
    uniform in the disk: mean 0, variance delta^2 / 4 per component, mean
    length 2 delta / 3, never longer than delta, components uncorrelated."""
    w = np.float32(1.9)
    delta = np.float32(0.05)
    S = OracleSystem.grid(4, 4, w, w, delta=delta, n_moves=1, seed=23,
                          flags=OracleSystem.FLAG_ACC | OracleSystem.FLAG_DISK)
    start = np.zeros(17, np.uint32)
    start[1:] = 1
    steps = []
    xy = np.array([[0.95, 0.95]], np.float32)
    for k in range(4000):
        S.set_state(xy, start, sweep=k)
        S.subsweep(0)
        acc, _ = S.aux()
        steps.append(acc[0].astype(np.float64))
    st = np.array(steps)
    r = np.hypot(st[:, 0], st[:, 1])
    assert r.max() < float(delta)
    v = float(delta) ** 2 / 4
    assert abs(st[:, 0].mean()) < 5 * math.sqrt(v / len(st))
    assert abs(st[:, 1].mean()) < 5 * math.sqrt(v / len(st))
    assert abs(st[:, 0].var() / v - 1) < 0.1
    assert abs(st[:, 1].var() / v - 1) < 0.1
    # E r = 2 delta / 3, Var r = delta^2 / 18
    assert abs(r.mean() - 2 * float(delta) / 3) < 5 * float(delta) / math.sqrt(18 * len(st))
    assert abs(np.corrcoef(st[:, 0], st[:, 1])[0, 1]) < 0.1


def test_single_disk_displacements():
    """Accepted displacements of a lone disk are symmetric, with variance
    delta^2 / 3 per component when the disk sits deep inside a wide cell, and
    the two components are uncorrelated."""
    w = np.float32(1.9)
    delta = np.float32(0.05)
    S = OracleSystem.grid(4, 4, w, w, delta=delta, n_moves=1, seed=23,
                          flags=OracleSystem.FLAG_ACC)
    start = np.zeros(17, np.uint32)
    start[1:] = 1
    steps = []
    xy = np.array([[0.95, 0.95]], np.float32)
    for k in range(4000):
        S.set_state(xy, start, sweep=k)      # always restart from the cell centre
        S.subsweep(0)
        acc, _ = S.aux()
        steps.append(acc[0].astype(np.float64))
    st = np.array(steps)
    assert np.all(np.abs(st) < float(delta))
    v = float(delta) ** 2 / 3
    assert abs(st[:, 0].mean()) < 5 * math.sqrt(v / len(st))
    assert abs(st[:, 1].mean()) < 5 * math.sqrt(v / len(st))
    assert abs(st[:, 0].var() / v - 1) < 0.1
    assert abs(st[:, 1].var() / v - 1) < 0.1
    assert abs(np.corrcoef(st[:, 0], st[:, 1])[0, 1]) < 0.1


@pytest.mark.parametrize("flags", [0, OracleSystem.FLAG_DISK])
def test_two_disk_separation_density(flags):
    """Two disks in a periodic box: in equilibrium the minimum-image
    separation has density proportional to r on [1, min(L)/2], with square
    and with in-circle proposals alike (both are symmetric)."""
    w = np.float32(1.25)
    S = OracleSystem.grid(6, 6, w, w, delta=np.float32(0.6), n_moves=4, seed=29, flags=flags)
    start = np.zeros(37, np.uint32)
    start[1:] = 2
    S.set_state(np.array([[0.3, 0.3], [1.2, 1.1]], np.float32), start)
    L = 6 * float(w)
    R = L / 2
    rmid = math.sqrt((1 + R * R) / 2)    # splits [1, R] into two equal-probability halves
    inner, outer, below = [], [], 0
    S.sweep(500)
    for k in range(20000):
        S.sweep(5)
        gx, gy = S.global_positions()
        dx = (gx[0] - gx[1] + L / 2) % L - L / 2
        dy = (gy[0] - gy[1] + L / 2) % L - L / 2
        r = math.hypot(dx, dy)
        below += r < 1.0 - 1e-6
        if r <= R:
            inner.append(1.0 if r < rmid else 0.0)
    assert below == 0
    m, se = E.mean_and_error(inner, min_blocks=32)
    assert abs(m - 0.5) < max(4 * se, 0.01), (m, se)


@pytest.mark.parametrize("n_moves", [1, 3])
def test_accept_log_matches_what_moved(n_moves):
    """The accept bits of a sub-sweep agree with what actually moved, an
    observable the bits are not computed from: with one trial per cell, a
    cell's multiset of positions changes iff its bit 0 is set (a proposal is
    never zero); bits only occupy positions below n_M; empty active cells
    log 0; the bits of the active cells add up to the accepted moves."""
    O = OracleSystem.lattice(24, 24, 0.70, w_max=math.sqrt(2.0), delta=0.18, n_moves=n_moves,
                             seed=3)
    O.sweep(4)
    for Q in (0, 3, 1, 2):
        xy0, st0, _ = O.get_state()
        a0 = O.counters()[1]
        O.subsweep(Q)
        xy1, st1, _ = O.get_state()
        assert np.array_equal(st0, st1)
        log = O.accept_log()
        cnt = np.diff(st0.astype(np.int64))
        active = np.zeros(O.mx * O.my, bool)
        for c in range(O.mx * O.my):
            cy, cx = divmod(c, O.mx)
            active[c] = (cx & 1) + 2 * (cy & 1) == Q
        moved_bits = 0
        for c in np.nonzero(active)[0]:
            bits = int(log[c])
            assert bits >> n_moves == 0
            if cnt[c] == 0:
                assert bits == 0
            moved_bits += bin(bits).count("1")
            if n_moves == 1:
                a = np.sort(xy0[st0[c]:st0[c + 1]].view(np.uint64).ravel())
                b = np.sort(xy1[st1[c]:st1[c + 1]].view(np.uint64).ravel())
                assert (bits & 1) == (0 if np.array_equal(a, b) else 1), c
        assert moved_bits == O.counters()[1] - a0
