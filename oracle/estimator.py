"""FP64 pressure from the contact value of g(r) -- TEST INFRASTRUCTURE ONLY.

Follows Sec. 4 of the paper step by step:
  * a histogram n[r_i] of pair distances in bins [r_i, r_i + dr), r_i = 1 + i dr
    (ordered pairs: every unordered pair counts twice, so g -> 1 for an ideal
    gas, which is how Eq. gR normalises);
  * Eq. R: sampling point R_i = 2/3 (r_{i+1}^3 - r_i^3) / (r_{i+1}^2 - r_i^2);
  * Eq. gR: g(R_i) = n[r_i] / (N rho 2 pi R_i dr);
  * a degree-5 least-squares polynomial through g(R_i) on (sigma, sigma + c],
    extrapolated to r = sigma (dr = 1e-4, c = 0.02, degree 5);
  * Eq. P: P* = rho (1 + (pi/2) rho g(sigma+)) with sigma = 1.
The fit is an unweighted least-squares problem in the variable (R - 1) / c,
solved with numpy's lstsq.
"""
from __future__ import annotations

import numpy as np

DR = 1e-4
FIT_RANGE = 0.02
DEGREE = 5
NBINS = 200


def sampling_points(nbins: int = NBINS, dr: float = DR) -> np.ndarray:
    """Eq. R for bins r_i = 1 + i dr."""
    i = np.arange(nbins, dtype=np.float64)
    r0 = 1.0 + i * dr
    r1 = 1.0 + (i + 1.0) * dr
    return (2.0 / 3.0) * (r1 ** 3 - r0 ** 3) / (r1 ** 2 - r0 ** 2)


def pair_correlation(hist, n_samples: float, N: float, rho: float, dr: float = DR):
    """Eq. gR: g(R_i) from the summed histogram of n_samples configurations."""
    hist = np.asarray(hist, dtype=np.float64) / float(n_samples)
    R = sampling_points(len(hist), dr)
    return R, hist / (N * rho * 2.0 * np.pi * R * dr)


def contact_value(hist, n_samples, N, rho, dr=DR, c=FIT_RANGE, degree=DEGREE) -> float:
    """g(sigma+) by the degree-`degree` fit over (sigma, sigma + c]."""
    R, g = pair_correlation(hist, n_samples, N, rho, dr)
    keep = (R > 1.0) & (R <= 1.0 + c)
    x = (R[keep] - 1.0) / c
    X = np.vander(x, degree + 1, increasing=True)
    coef, *_ = np.linalg.lstsq(X, g[keep], rcond=None)
    return float(coef[0])


def pressure(rho: float, g_contact: float) -> float:
    """Eq. P with sigma = 1 (dimensionless P* = beta P sigma^2)."""
    return rho * (1.0 + 0.5 * np.pi * rho * g_contact)


def pressure_from_histogram(hist, n_samples, N, rho, **kw):
    g0 = contact_value(hist, n_samples, N, rho, **kw)
    return pressure(rho, g0), g0


def blocking(samples):
    """Flyvbjerg-Petersen blocking: list of (n_blocks, mean, standard error)
    for successive pairwise block averages."""
    x = np.asarray(samples, dtype=np.float64)
    out = []
    while len(x) >= 2:
        n = len(x)
        out.append((n, float(x.mean()), float(x.std(ddof=1) / np.sqrt(n))))
        if n < 4:
            break
        m = n // 2
        x = 0.5 * (x[0:2 * m:2] + x[1:2 * m:2])
    return out


def mean_and_error(samples, min_blocks: int = 16):
    """Mean and a conservative standard error: the largest blocked estimate
    among levels that still have at least `min_blocks` blocks."""
    levels = blocking(samples)
    if not levels:
        raise ValueError("need at least two samples")
    good = [lv for lv in levels if lv[0] >= min_blocks] or levels[:1]
    return levels[0][1], max(lv[2] for lv in good)


def virial_pressure_ratio(phi: float) -> float:
    """Low-density equation of state of hard disks, beta P / rho to third
    order in phi: 1 + 2 phi + 4 (B3/B2^2) phi^2 + 8 (B4/B2^3) phi^3 with the
    exact coefficients B3/B2^2 = 4/3 - sqrt(3)/pi and
    B4/B2^3 = 2 - 9 sqrt(3) / (2 pi) + 10 / pi^2 (B2 rho = 2 phi)."""
    b3 = 4.0 / 3.0 - np.sqrt(3.0) / np.pi
    b4 = 2.0 - 9.0 * np.sqrt(3.0) / (2.0 * np.pi) + 10.0 / np.pi ** 2
    return 1.0 + 2.0 * phi + 4.0 * b3 * phi ** 2 + 8.0 * b4 * phi ** 3


# ---------------------------------------------------------------- 3D spheres
# The same estimator for hard spheres (the method in d = 3): the sampling
# point is the volume-weighted mean radius of the shell [r_i, r_{i+1}), g is
# the pair count over N rho times the shell's surface 4 pi R^2 dr at that
# radius, the contact value comes from the same degree-5 fit, and the
# pressure from the contact theorem in 3D, beta P / rho = 1 + (2 pi / 3) rho
# g(sigma+) (sigma = 1).


def sampling_points_3d(nbins: int = NBINS, dr: float = DR) -> np.ndarray:
    i = np.arange(nbins, dtype=np.float64)
    r0 = 1.0 + i * dr
    r1 = 1.0 + (i + 1.0) * dr
    return 0.75 * (r1 ** 4 - r0 ** 4) / (r1 ** 3 - r0 ** 3)


def pair_correlation_3d(hist, n_samples: float, N: float, rho: float, dr: float = DR):
    hist = np.asarray(hist, dtype=np.float64) / float(n_samples)
    R = sampling_points_3d(len(hist), dr)
    return R, hist / (N * rho * 4.0 * np.pi * R * R * dr)


def contact_value_3d(hist, n_samples, N, rho, dr=DR, c=FIT_RANGE, degree=DEGREE) -> float:
    R, g = pair_correlation_3d(hist, n_samples, N, rho, dr)
    keep = (R > 1.0) & (R <= 1.0 + c)
    x = (R[keep] - 1.0) / c
    X = np.vander(x, degree + 1, increasing=True)
    coef, *_ = np.linalg.lstsq(X, g[keep], rcond=None)
    return float(coef[0])


def pressure_3d(rho: float, g_contact: float) -> float:
    return rho * (1.0 + (2.0 * np.pi / 3.0) * rho * g_contact)


def pressure_from_histogram_3d(hist, n_samples, N, rho, **kw):
    g0 = contact_value_3d(hist, n_samples, N, rho, **kw)
    return pressure_3d(rho, g0), g0


def virial_pressure_ratio_3d(eta: float) -> float:
    """Low-density equation of state of hard spheres, beta P / rho through
    eta^5, from the textbook virial coefficients: 4 (B2), 10 (B3/B2^2 = 5/8),
    18.3648 (B4/B2^3 = 0.2869495, known in closed form), 28.2245 and 39.8151
    (B5, B6, computed numerically in the literature)."""
    c = (4.0, 10.0, 18.3648, 28.2245, 39.8151)
    return 1.0 + sum(ck * eta ** (k + 1) for k, ck in enumerate(c))
