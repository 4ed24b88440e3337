"""Pins of the 3D hard-sphere oracle (the method in d = 3, Sec. 2):
lattice start, exact draws, invariants, closed-form equilibria of one and two
spheres, the estimator on exact histograms, and the low-density equation of
state against the virial series."""
import math

import numpy as np
import pytest
from scipy.stats import chi2, kstest

from oracle import estimator as E
from oracle.spheres import SphereOracle, trial_displacement


def _min_image_pairs(S):
    """FP64 minimum-image distances of all pairs (small N only)."""
    x = S.global_positions()
    L = np.array(S.box)
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d ** 2).sum(-1))
    iu = np.triu_indices(len(x), 1)
    return r[iu]


def _check_invariants(S, tags0=None):
    xyz, st, tags, _ = S.get_state()
    cnt = np.diff(st.astype(np.int64))
    assert st[-1] == S.N and cnt.min() >= 0 and cnt.max() <= 8
    for a in range(3):
        assert np.all(xyz[:, a] > 0) and np.all(xyz[:, a] <= S.w[a])
    if tags0 is not None:
        assert np.array_equal(np.sort(tags), np.sort(tags0))
    assert S.count_overlaps() == 0
    return tags


def test_lattice_initial_state():
    """Simple cubic lattice at eta: spacing (pi / (6 eta))^(1/3), every cell
    within capacity, every site in its cell, nearest neighbours exactly one
    spacing apart, cells listing spheres in lattice order."""
    eta = 0.40
    S = SphereOracle.lattice(6, 6, 6, eta, delta=0.1)
    a = (math.pi / (6 * eta)) ** (1 / 3)
    assert np.allclose(S.box, [6 * a] * 3, rtol=1e-6)
    assert all(m % 2 == 0 and m >= 4 for m in S.m)
    assert all(1.0 <= w < 2 / math.sqrt(3) for w in S.w)
    tags = _check_invariants(S)
    r = _min_image_pairs(S)
    assert abs(r.min() - a) < 1e-5
    xyz, st, tags, _ = S.get_state()
    for c in range(S.C):
        seg = tags[st[c]:st[c + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)


def test_trial_displacement_bits():
    """x and y come from the high and low halves of the first word, z from
    the high half of the second; each half maps to the midpoint of one of
    65536 parts of (-1, 1) times delta, symmetric under h -> 65535 - h; the
    low half of the second word is unused."""
    delta = np.float32(0.2)
    h = np.arange(0, 65536, 257, dtype=np.uint32)
    for hv in h:
        d = trial_displacement((int(hv) << 16) | (65535 - int(hv)), (int(hv) << 16) | 0x1234, delta)
        e = np.float32((2.0 * hv + 1 - 65536) / 65536.0)
        assert d[0] == np.float32(e * delta) and d[2] == d[0] and d[1] == -d[0]
        d2 = trial_displacement((int(hv) << 16) | (65535 - int(hv)), (int(hv) << 16) | 0xBEEF, delta)
        assert np.array_equal(d, d2)
    assert np.abs(trial_displacement(0xFFFFFFFF, 0xFFFFFFFF, delta)).max() < delta


def test_invariants_every_sweep():
    """Every sweep: counts within capacity, every identity kept once, every
    coordinate in its cell, no overlap in the chain's metric, and no pair
    closer than 1 in FP64 global coordinates (up to re-expression rounding)."""
    S = SphereOracle.lattice(6, 6, 6, 0.45, delta=0.2, n_moves=4, seed=5)
    tags0 = _check_invariants(S)
    for k in range(40):
        S.sweep(1)
        _check_invariants(S, tags0)
        if k % 10 == 9:
            assert _min_image_pairs(S).min() > 1.0 - 1e-6
    t, a = S.counters()
    assert 0 < a < t


def test_cell_order_does_not_matter():
    """Cells of one set never interact (w >= 1): visiting them in row-major,
    reversed or scrambled order gives bit-identical states."""
    states = []
    for mode in (0, 1, 2):
        S = SphereOracle.lattice(8, 8, 8, 0.45, delta=0.25, n_moves=5, seed=9)
        S.sweep(3)
        for Q in (5, 0, 7, 2, 1, 6, 3, 4):
            S.subsweep(Q, mode)
        states.append(S.get_state())
    for st in states[1:]:
        assert np.array_equal(st[0].view(np.uint32), states[0][0].view(np.uint32))
        assert np.array_equal(st[1], states[0][1]) and np.array_equal(st[2], states[0][2])


def test_particle_shuffle_is_uniform():
    """One cell of three spheres far apart, one trial per cell update: the
    trial goes to list[0] of the shuffled list, so each sphere is the one
    moved a third of the time (chi-square), and the stored order changes."""
    w = np.float32(1.1)
    S = SphereOracle.grid((4, 4, 4), (w, w, w), 3, delta=np.float32(0.02), n_moves=1, seed=41)
    xyz = np.array([[0.05, 0.05, 0.05], [1.05, 1.05, 0.05], [1.05, 0.05, 1.05]], np.float32)
    start = np.zeros(65, np.uint32)
    start[1:] = 3
    tag = np.array([10, 11, 12], np.uint32)
    moved, reordered = [], 0
    for k in range(3000):
        S.set_state(xyz, start, tags=tag, sweep=k)
        S.subsweep(0)
        x1, _, t1, _ = S.get_state()
        reordered += int(not np.array_equal(t1, tag))
        for j in range(3):
            i = int(np.nonzero(tag == t1[j])[0][0])
            if not np.array_equal(x1[j], xyz[i]):
                moved.append(int(t1[j]))
    assert reordered > 0 and len(moved) > 1000
    cnt = np.bincount(np.array(moved) - 10, minlength=3).astype(float)
    e = cnt.sum() / 3
    assert chi2.sf(((cnt - e) ** 2 / e).sum(), 2) > 1e-4


def test_set_order_and_shift_are_uniform():
    """Each of the 8 sets takes each of the 8 positions with probability 1/8
    (chi-square over the 8 x 8 table), the 6 shift directions are equally
    likely, and d / (w_f / 2) is uniform on [0, 1)."""
    S = SphereOracle.lattice(10, 10, 10, 0.3)
    n = 16000
    table = np.zeros((8, 8))
    fs, ds = [], []
    for s in range(n):
        order, f, d = S.draws(s)
        assert sorted(order) == list(range(8))
        for pos, q in enumerate(order):
            table[q, pos] += 1
        fs.append(f)
        ds.append(float(d) / (0.5 * float(S.w[f // 2])))
    e = n / 8
    assert chi2.sf(((table - e) ** 2 / e).sum(), 49) > 1e-4
    fc = np.bincount(fs, minlength=6)
    assert len(fc) == 6 and chi2.sf(((fc - n / 6) ** 2 / (n / 6)).sum(), 5) > 1e-4
    assert min(ds) >= 0 and max(ds) < 1 and kstest(ds, "uniform").pvalue > 1e-4


def test_shift_translates_and_loses_nothing():
    """A shift by d along f translates every sphere by exactly -d along that
    axis in global FP64 coordinates (up to the re-expression of one FP32
    coordinate) and keeps every identity; 3,000 random shifts lose nothing."""
    S = SphereOracle.lattice(6, 6, 6, 0.40, delta=0.1)
    rng = np.random.default_rng(3)
    _, _, tags0, _ = S.get_state()
    L = np.array(S.box)
    for k in range(3000):
        f = int(rng.integers(6))
        d = np.float32(rng.random() * 0.5 * float(S.w[f // 2]))
        if k < 30:
            x0 = S.global_positions()
            _, _, t0, _ = S.get_state()
        S.shift(f, d)
        if k < 30:
            x1 = S.global_positions()
            _, _, t1, _ = S.get_state()
            o0, o1 = np.argsort(t0), np.argsort(t1)
            dx = x1[o1] - x0[o0]
            dx -= L * np.round(dx / L)
            sgn = -1.0 if f % 2 == 0 else 1.0
            want = np.zeros(3)
            want[f // 2] = sgn * float(d)
            assert np.abs(dx - want).max() < 1e-5
    _check_invariants(S, tags0)


def test_single_sphere_acceptance_closed_form():
    """One sphere, uniform in its cell, moved uniformly in the cube
    (-delta, delta)^3: it stays in the cell with probability
    prod_a (1 - delta / (2 w_a)), and nothing else rejects it."""
    w = np.float32(1.1)
    delta = np.float32(0.5)
    S = SphereOracle.grid((4, 4, 4), (w, w, w), 1, delta=delta, n_moves=4, seed=17)
    start = np.zeros(65, np.uint32)
    start[1:] = 1
    S.set_state(np.array([[0.5, 0.6, 0.7]], np.float32), start)
    S.sweep(200)
    t0, a0 = S.counters()
    S.sweep(40000)
    t1, a1 = S.counters()
    n = t1 - t0
    p_hat = (a1 - a0) / n
    p = (1 - float(delta) / (2 * float(w))) ** 3
    se = math.sqrt(p * (1 - p) / n)
    assert abs(p_hat - p) < 10 * se, (p_hat, p, se)


def test_two_sphere_separation_density():
    """Two spheres in a periodic box: in equilibrium the minimum-image
    separation has density proportional to r^2 on [1, L/2], so half of the
    mass of [1, R] lies below r_mid = ((1 + R^3) / 2)^(1/3)."""
    w = np.float32(1.1)
    S = SphereOracle.grid((4, 4, 4), (w, w, w), 2, delta=np.float32(0.5), n_moves=4, seed=29)
    start = np.zeros(65, np.uint32)
    start[1:] = 1
    start[2:] = 2
    S.set_state(np.array([[0.3, 0.3, 0.3], [0.6, 0.7, 0.8]], np.float32), start)
    L = 4 * float(w)
    R = L / 2
    rmid = ((1 + R ** 3) / 2) ** (1 / 3)
    S.sweep(200)
    inner = []
    for k in range(20000):
        S.sweep(2)
        r = _min_image_pairs(S)[0]
        assert r > 1.0 - 1e-6
        if r <= R:
            inner.append(1.0 if r < rmid else 0.0)
    m, se = E.mean_and_error(inner, min_blocks=32)
    assert abs(m - 0.5) < max(4 * se, 0.01), (m, se)


def test_estimator_3d_on_exact_histograms():
    """Histograms computed exactly from an analytic g(r) (a constant plus the
    paper's exponential model shape): the 3D sampling points, shell
    normalisation and fit give back g(sigma+) to 1e-5."""
    N, rho = 4096.0, 0.8
    edges = 1.0 + np.arange(201) * 1e-4
    for g0, amp in ((1.0, 0.0), (2.5, 1.5)):
        def g(r):
            return g0 - amp + amp * np.exp(-30.0 * (r - 1.0))
        # ordered pairs: N rho integral of 4 pi r^2 g(r) over each shell
        hist = np.zeros(200)
        for b in range(200):
            r = np.linspace(edges[b], edges[b + 1], 401)
            y = 4 * np.pi * r ** 2 * g(r)
            hist[b] = N * rho * np.trapezoid(y, r)
        got = E.contact_value_3d(hist, 1, N, rho)
        assert abs(got / g0 - 1) < 1e-5, (got, g0)
        if amp == 0.0:   # a constant g is recovered in every shell, not only at contact
            _, gr = E.pair_correlation_3d(hist, 1, N, rho)
            assert np.abs(gr / g0 - 1).max() < 1e-6
    assert abs(E.pressure_3d(rho, 1.0) / rho - (1 + 2 * math.pi / 3 * rho)) < 1e-12


def test_low_density_equation_of_state():
    """beta P / rho of hard spheres from the contact value at eta = 0.1
    equals the virial series 1 + 4 eta + 10 eta^2 + 18.36 eta^3 + ...
    (1.5216); counting unordered pairs would give about 1.25, the second
    virial term alone 1.4."""
    eta = 0.10
    S = SphereOracle.lattice(16, 16, 16, eta, delta=0.55, n_moves=4, seed=7)
    S.sweep(100)
    L = np.array(S.box)
    rho = S.N / float(np.prod(L))
    P, hb = [], np.zeros(200)
    for k in range(2000):
        S.sweep(1)
        hb += S.pair_histogram()
        if (k + 1) % 50 == 0:
            P.append(E.pressure_from_histogram_3d(hb, 50, S.N, rho)[0] / rho)
            hb[:] = 0
    m, se = E.mean_and_error(P, min_blocks=8)
    assert abs(m - E.virial_pressure_ratio_3d(eta)) < 4 * se + 2e-3, (m, se)
    assert m - 1.4 > 3 * se


def test_accumulators_track_each_sphere_displacement():
    """The accumulators (S10) equal each sphere's displacement since the start,
    found independently from FP64 global positions by identity tag (minimum
    image, less the grid shifts of the sweeps' draws): they add every
    accepted move, follow their sphere through shuffles and shifts, and
    start at zero."""
    S = SphereOracle.lattice(10, 10, 10, 0.3, delta=0.2, n_moves=4, seed=5)
    _, _, tags, _ = S.get_state()
    x0 = np.zeros((S.N, 3))
    x0[tags] = S.global_positions()
    assert not S.acc().any()
    S.sweep(40)
    _, _, tags, _ = S.get_state()
    L = np.array(S.box)
    # global positions are taken on the shifted grid: every sweep's shift
    # (S5, S8) translates all of them by -d (f even) or +d (f odd) along its axis
    grid = np.zeros(3)
    for s in range(40):
        _, f, dd = S.draws(s)
        grid[f // 2] += -float(dd) if f % 2 == 0 else float(dd)
    d = S.global_positions() - x0[tags] - grid
    d -= L * np.round(d / L)
    a = S.acc().astype(np.float64)
    assert np.abs(a).max() > 0.2
    assert np.abs(d - a).max() < 1e-4
