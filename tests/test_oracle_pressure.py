"""Pins for the pressure path: the FP64 estimator (Sec. 4, Eqs. P, gR, R), the
oracle's pair histogram, the low-density equation of state and agreement with
the FP64 single-particle reference chain.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import OracleSystem, SerialReference
from oracle import estimator as E


def _exact_counts(antiderivative, N, rho, nbins=200, dr=1e-4):
    """Expected ordered-pair counts per bin for a given g(r): N rho 2 pi times
    the integral of r g(r) over the bin, from an antiderivative of r g(r)."""
    r = 1.0 + np.arange(nbins + 1) * dr
    return N * rho * 2 * np.pi * (antiderivative(r[1:]) - antiderivative(r[:-1]))


def test_estimator_constant_and_linear_g():
    N, rho = 1e6, 0.8
    # g = 1: r g(r) integrates to r^2 / 2
    g0 = E.contact_value(_exact_counts(lambda r: r * r / 2, N, rho), 1, N, rho)
    assert abs(g0 - 1) < 1e-8
    # g = 2 + 3 (r - 1): r g(r) = 3 r^2 - r integrates to r^3 - r^2 / 2
    g0 = E.contact_value(_exact_counts(lambda r: r ** 3 - r * r / 2, N, rho), 1, N, rho)
    assert abs(g0 - 2) < 1e-8
    # the number of samples divides out
    h = _exact_counts(lambda r: r * r / 2, N, rho) * 7
    assert abs(E.contact_value(h, 7, N, rho) - 1) < 1e-8


@pytest.mark.parametrize("kappa", [10.0, 30.0, 50.0])
def test_estimator_bias_on_model_distribution(kappa):
    """Sec. 4: with dr = 1e-4, c = 0.02 and degree 5 the extrapolation of an
    exponential model distribution (the paper's test shape, decay 30) is
    biased by less than 1e-5."""
    N, rho = 1e6, 0.8

    def F(r):   # antiderivative of r exp(-kappa (r - 1))
        return -np.exp(-kappa * (r - 1)) * (r / kappa + 1 / kappa ** 2)
    g0 = E.contact_value(_exact_counts(F, N, rho), 1, N, rho)
    assert abs(g0 - 1) < 1e-5


def test_estimator_noisy_histograms_are_unbiased():
    N, rho = 65536, 0.89
    rng = np.random.default_rng(1)
    lam = _exact_counts(lambda r: -np.exp(-30 * (r - 1)) * (r / 30 + 1 / 900), N, rho) * 5.0
    g = [E.contact_value(rng.poisson(lam), 1, N, rho) for _ in range(400)]
    m, se = np.mean(g), np.std(g) / np.sqrt(len(g))
    assert abs(m - 5.0) < 4 * se


def test_pressure_formula_and_virial_coefficients():
    # Eq. P with g = 1 is the second-virial truncation beta P / rho = 1 + 2 phi
    rho = 0.1
    phi = rho * np.pi / 4
    assert abs(E.pressure(rho, 1.0) / rho - (1 + 2 * phi)) < 1e-14
    # exact hard-disk B3/B2^2 and B4/B2^3
    b3 = 4 / 3 - math.sqrt(3) / math.pi
    b4 = 2 - 9 * math.sqrt(3) / (2 * math.pi) + 10 / math.pi ** 2
    assert abs(b3 - 0.782004) < 1e-6 and abs(b4 - 0.532231) < 1e-6
    assert abs(E.virial_pressure_ratio(0.05) - (1 + 0.1 + 4 * b3 * 0.0025 + 8 * b4 * 0.05 ** 3)) < 1e-15


def test_blocking_on_independent_and_correlated_data():
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1, 4096)
    m, se = E.mean_and_error(x)
    assert abs(se - 1 / 64) < 0.3 / 64
    # AR(1) with rho = 0.9: SE grows by sqrt((1 + rho) / (1 - rho)) ~ 4.36
    y = np.zeros(65536)
    e = rng.normal(0, 1, 65536)
    for i in range(1, len(y)):
        y[i] = 0.9 * y[i - 1] + e[i]
    _, se_y = E.mean_and_error(y)
    naive = y.std() / np.sqrt(len(y))
    assert 3.0 < se_y / naive < 5.5


def test_pair_histogram_matches_brute_force():
    """Ordered pairs binned on r^2 edges vs an all-pairs FP64 count; a pair
    may differ only when its FP64 distance sits within 1e-6 of a bin edge."""
    for phi, w_max in [(0.70, 0.0), (0.70, math.sqrt(2.0)), (0.55, 1.932)]:
        S = OracleSystem.lattice(20, 20, phi, w_max=w_max, delta=0.2, seed=13)
        S.sweep(40)
        h = S.pair_histogram()
        gx, gy = S.global_positions()
        Lx, Ly = S.box
        dx = gx[:, None] - gx[None, :]
        dy = gy[:, None] - gy[None, :]
        dx -= Lx * np.round(dx / Lx)
        dy -= Ly * np.round(dy / Ly)
        r = np.sqrt(dx * dx + dy * dy)
        np.fill_diagonal(r, np.inf)
        r = r[r < 1.0201]
        edges = 1.0 + np.arange(201) * 1e-4
        ref = np.histogram(r, bins=edges)[0]
        near = np.abs(r[:, None] - edges[None, :]).min(axis=1) < 1e-6
        diff = np.abs(h.astype(np.int64) - ref).sum()
        assert diff <= 2 * near.sum(), (phi, diff, near.sum())
        assert h.sum() > 0


def test_histogram_rejects_wrapping_reach():
    w = np.float32(1.01)   # narrower than the histogram range -> reach of two cells
    S = OracleSystem.grid(4, 8, w, w)
    with pytest.raises(ValueError):
        S.pair_histogram()


def _oracle_pressure(S, n_samples, every, block=20):
    Lx, Ly = S.box
    rho = S.N / (Lx * Ly)
    P, hb = [], np.zeros(200)
    for k in range(n_samples):
        S.sweep(every)
        hb += S.pair_histogram()
        if (k + 1) % block == 0:
            P.append(E.pressure_from_histogram(hb, block, S.N, rho)[0])
            hb[:] = 0
    return P, rho


def test_low_density_equation_of_state():
    """beta P / rho -> 1 + 2 phi + 3.128 phi^2 + 4.258 phi^3 + O(phi^4) at low
    density (exact B2, B3, B4 of hard disks); at phi = 0.1 the remainder is
    about 6e-4.  An unordered-pair count would give 1.12, an ideal gas 1.2."""
    phi = 0.10
    S = OracleSystem.lattice(64, 64, phi, delta=0.45, n_moves=4, seed=7)
    S.sweep(200)
    P, rho = _oracle_pressure(S, 3000, 1, block=50)
    m, se = E.mean_and_error(P, min_blocks=8)
    z = m / rho
    assert abs(z - E.virial_pressure_ratio(phi)) < 4 * se / rho + 1e-3, (z, se / rho)
    assert z - 1.2 > 3 * se / rho


@pytest.mark.parametrize("phi,n_moves", [(0.30, 4), (0.60, 4), (0.60, 16)])
def test_equation_of_state_matches_serial_reference(phi, n_moves):
    """The checkerboard chain and the plain single-particle chain share the
    equilibrium: their pressures agree within 3 combined standard errors at
    equal numbers of trial moves.  n_M = 16 (each disk of a cell visited
    many times per update, the visit list wrapping around) samples the same
    equilibrium as n_M = 4 (Sec. 2.3: any n_M keeps detailed balance)."""
    S = OracleSystem.lattice(16, 16, phi, delta=0.15, n_moves=n_moves, seed=3)
    S.sweep(500)
    t0 = S.counters()[0]
    P1, rho = _oracle_pressure(S, 8000, 5)
    trials = S.counters()[0] - t0
    gx, gy = S.global_positions()
    Lx, Ly = S.box
    R = SerialReference(gx, gy, Lx, Ly, 0.15, seed=11)
    R.run(trials // 8)
    per = trials // 8000
    P2, hb = [], np.zeros(200)
    for k in range(8000):
        R.run(per)
        hb += R.pair_histogram()
        if (k + 1) % 20 == 0:
            P2.append(E.pressure_from_histogram(hb, 20, R.N, rho)[0])
            hb[:] = 0
    m1, se1 = E.mean_and_error(P1, 8)
    m2, se2 = E.mean_and_error(P2, 8)
    assert abs(m1 - m2) < 3 * math.hypot(se1, se2), (m1, se1, m2, se2)
    assert se1 < 0.02 * m1
