"""Pins of the FP64 single-particle reference (serial_ref.c) and of two
oracle utilities, each against something other than the code itself:
  * two disks in a periodic box: the acceptance of a square trial move and
    the density of the separation follow from geometry alone (the relative
    position is uniform outside the unit disk);
  * the smallest pair r^2 of a hand-built state;
  * the threaded sub-sweep gives the serial chain bit for bit."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import OracleSystem, SerialReference


def lens_area(s):
    """Area of the intersection of two disks of radius 1 at centre distance s <= 2."""
    return 2.0 * math.acos(s / 2.0) - 0.5 * s * math.sqrt(4.0 - s * s)


def two_disk_acceptance(L, delta):
    """Acceptance of a uniform square move [-delta, delta)^2 of one of two
    hard disks (sigma = 1) in an L x L periodic box at equilibrium.  The
    relative position r is uniform over the torus minus the unit disk D, so
    P(reject | move u) = |(D - u) minus D| / (L^2 - pi) = (pi - lens(|u|)) /
    (L^2 - pi); averaged over u in the square."""
    I, _ = integrate.dblquad(lambda v, u: lens_area(math.hypot(u, v)), -delta, delta,
                             lambda u: -delta, lambda u: delta, epsabs=1e-12, epsrel=1e-12)
    mean_lens = I / (4.0 * delta * delta)
    return 1.0 - (math.pi - mean_lens) / (L * L - math.pi)


def test_lens_area_limits():
    assert lens_area(0.0) == pytest.approx(math.pi, abs=1e-15)
    assert lens_area(2.0) == pytest.approx(0.0, abs=1e-15)
    # small s: pi - lens(s) = 2 s + O(s^3)
    assert (math.pi - lens_area(1e-4)) / 1e-4 == pytest.approx(2.0, rel=1e-7)


@pytest.mark.parametrize("delta", [0.3, 0.6])
def test_serial_two_disk_acceptance_closed_form(delta):
    L = 8.0
    S = SerialReference(np.array([1.0, 5.0]), np.array([1.0, 4.5]), L, L, delta, seed=99)
    S.run(20_000)                                  # forget the start
    t0, a0 = S.counters()
    S.run(4_000_000)
    t1, a1 = S.counters()
    n = t1 - t0
    rej = (n - (a1 - a0)) / n
    p = 1.0 - two_disk_acceptance(L, delta)
    se = math.sqrt(p * (1 - p) / n) * 3.0           # moves are correlated: generous SE
    assert abs(rej - p) < 5 * se, (rej, p, se)


def test_serial_two_disk_separation_density():
    """Minimum-image separation r of two disks in an 8 x 8 box: density
    proportional to r on [1, 4] (circles that fit inside the torus cell)."""
    L = 8.0
    S = SerialReference(np.array([1.0, 5.0]), np.array([1.0, 4.5]), L, L, 1.5, seed=7)
    S.run(5_000)
    rs = []
    for _ in range(60_000):
        S.run(6)
        x, y = S.positions()
        dx = (x[0] - x[1] + L / 2) % L - L / 2
        dy = (y[0] - y[1] + L / 2) % L - L / 2
        r = math.hypot(dx, dy)
        if r <= 4.0:
            rs.append(r)
    rs = np.array(rs)
    assert rs.min() >= 1.0
    # CDF on [1, 4] for density ~ r: (r^2 - 1) / 15; Kolmogorov-Smirnov
    xs = np.sort(rs)
    F = (xs * xs - 1.0) / 15.0
    ecdf = np.arange(1, len(xs) + 1) / len(xs)
    D = np.max(np.abs(ecdf - F))
    # samples 6 trials apart are correlated; allow 3x the 0.1 % critical value
    assert D < 3 * 1.95 / math.sqrt(len(xs)), D


def test_min_pair_r2_of_a_built_state():
    """Two disks at distance 1.25 along x (r^2 = 1.5625 exactly in FP32),
    one of them across a cell boundary, and a third one far away."""
    O = OracleSystem.grid(4, 4, 1.5, 1.5)
    xy = np.array([[1.0, 0.75], [0.75, 0.75], [0.75, 0.75]], np.float32)
    start = np.zeros(17, np.uint32)
    # cell 0 holds disk 0 at x = 1.0; cell 1 (x offset 1.5) holds disk 1 at
    # local 0.75, i.e. global 2.25; cell 10 holds a far disk
    start[1:] = 1
    start[2:] = 2
    start[11:] = 3
    O.set_state(xy, start)
    assert O.min_pair_r2() == np.float32(1.5625)
    assert O.count_overlaps() == 0


def test_threaded_subsweeps_give_the_serial_chain():
    a = OracleSystem.lattice(96, 96, 0.70, w_max=math.sqrt(2.0), delta=0.12, n_moves=4, seed=3,
                             flags=3)
    b = OracleSystem.lattice(96, 96, 0.70, w_max=math.sqrt(2.0), delta=0.12, n_moves=4, seed=3,
                             flags=3)
    b.set_threads(4)
    a.sweep(25)
    b.sweep(25)
    xa, sa, wa = a.get_state()
    xb, sb, wb = b.get_state()
    assert wa == wb and np.array_equal(sa, sb)
    assert np.array_equal(xa.view(np.uint32), xb.view(np.uint32))
    assert a.counters() == b.counters()
    assert np.array_equal(a.accept_log(), b.accept_log())
    aa, ta = a.aux()
    ab, tb = b.aux()
    assert np.array_equal(ta, tb) and np.array_equal(aa.view(np.uint32), ab.view(np.uint32))
