"""Statistics and fits of the eta extrapolation (host code, no GPU)."""
import math

import numpy as np

from paper_1307_0328_amd import extrapolate as X


def test_binning_recovers_the_error_of_a_correlated_series():
    rng = np.random.default_rng(5)
    rho, n = 0.9, 1 << 17
    x = np.empty(n)
    x[0] = rng.normal() / math.sqrt(1 - rho * rho)
    e = rng.normal(size=n)
    for i in range(1, n):
        x[i] = rho * x[i - 1] + e[i]
    mean, err, ratio = X.binning(x)
    # AR(1): var of the mean = sigma_x^2 / n * (1 + rho) / (1 - rho)
    true = math.sqrt(1.0 / (1 - rho * rho) / n * (1 + rho) / (1 - rho))
    assert abs(err / true - 1.0) < 0.25
    # integrated autocorrelation time (1 + rho) / (2 (1 - rho)) = 9.5
    assert 6.0 < 0.5 * ratio * ratio < 13.0
    assert abs(mean) < 5 * true


def test_binning_of_independent_samples_is_the_naive_error():
    x = np.random.default_rng(1).normal(size=1 << 14)
    mean, err, ratio = X.binning(x)
    assert abs(err / (x.std(ddof=1) / math.sqrt(len(x))) - 1.0) < 0.2


def test_fit_reproduces_exact_polynomials():
    eta = np.array([0.01, 0.02, 0.03, 0.04, 0.05])
    y = -2.3 + 7.0 * eta ** 2
    v, dv, c, cov, chi2 = X.fit(eta, y, np.full(5, 1e-4), X.FITS["quad"])
    assert abs(v + 2.3) < 1e-12 and abs(c[1] - 7.0) < 1e-9 and chi2 < 1e-12
    y = -0.98 + 0.5 * eta
    v, dv, c, cov, chi2 = X.fit(eta, y, np.full(5, 1e-5), X.FITS["lin"])
    assert abs(v + 0.98) < 1e-12


def test_fit_error_of_a_two_point_line():
    # two points, equal errors s: the intercept of the line through them has
    # error s * sqrt(x1^2 + x2^2) / (x2 - x1)
    x = np.array([1.0, 3.0])
    s = 0.1
    v, dv, *_ = X.fit(x, np.array([2.0, 4.0]), np.full(2, s), (0, 1))
    assert abs(v - 1.0) < 1e-12
    assert abs(dv - s * math.sqrt(1 + 9) / 2.0) < 1e-12


def test_checkerboard_start_is_a_valid_configuration():
    from oracle import oracle as O
    st = X.checkerboard_state(6, 4, 2, parity=1)
    assert st["bstate"].reshape(2, 24)[0].sum() == 12
    ch = O.Chain(Lx=6, Ly=4, beta=2.0, V=3.0, mu=4.2, eta=0.05, dom_x=3, dom_y=2, dom_tau=2, seed=3)
    ch.set_state(st)
    assert ch.check() == 0
    ch.sweep(3)
    assert ch.check() == 0
