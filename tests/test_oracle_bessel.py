"""Pins for the oracle's own J_nu evaluator (CPU only).

Each check compares against something other than the oracle itself: an
arbitrary-precision library (mpmath), Bessel's integral, the three-term
recurrence, Neumann's sum of squares, and the closed forms at half-integer
order (where Hankel's expansion of Sec. 3.2 terminates and is exact).
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import direct

mpmath.mp.dps = 40


def envelope(x):
    """Amplitude scale of J_n at x: min(1, sqrt(2/(pi x)))."""
    x = np.asarray(x, dtype=np.float64)
    return np.minimum(1.0, np.sqrt(2.0 / (np.pi * np.maximum(x, 1e-300))))


def test_besselj_against_mpmath():
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(600):
        n = int(rng.integers(0, 110))
        x = float(10.0 ** rng.uniform(-4, 5.2))
        v = direct.besselj(n, x)
        t = float(mpmath.besselj(n, mpmath.mpf(x)))
        worst = max(worst, abs(v - t) / envelope(x))
    assert worst < 3e-14, worst


def test_besselj_branch_edges_against_mpmath():
    # arguments at the switches between series / Miller / Hankel
    for n in (0, 1, 2, 7, 30, 63):
        for x in (1.999999, 2.0, 2.000001, 24.99999, 25.0, 25.00001, 2.0 * n * n + 30.0):
            v = direct.besselj(n, x)
            t = float(mpmath.besselj(n, mpmath.mpf(x)))
            assert abs(v - t) <= 3e-14 * envelope(x), (n, x, v, t)


def test_negative_order_against_mpmath():
    for n in (-1, -2, -5, -64):
        for x in (0.3, 7.5, 120.0, 4.0e4):
            v = direct.besselj(n, x)
            t = float(mpmath.besselj(n, mpmath.mpf(x)))
            assert abs(v - t) <= 3e-14 * envelope(x)


def test_zero_argument():
    assert direct.besselj(0, 0.0) == 1.0
    for n in (1, 2, -3, 40):
        assert direct.besselj(n, 0.0) == 0.0


def test_double_double_argument():
    # J_n(hi + lo) with the low part of an exact product must match mpmath at
    # the exact real argument, not at the rounded one.
    rng = np.random.default_rng(3)
    w = rng.uniform(1e4, 1e5, 50)
    r = rng.uniform(0.5, 1.0, 50)
    hi, lo = direct.two_prod(w, r)
    for n in (0, 1, 10):
        v = direct.besselj(n, hi, lo)
        for i in range(50):
            exact = mpmath.mpf(float(w[i])) * mpmath.mpf(float(r[i]))
            t = float(mpmath.besselj(n, exact))
            assert abs(v[i] - t) <= 3e-16 * 0.1 + 1e-14 * envelope(hi[i])


def test_bessel_integral():
    # J_n(x) = (1/2pi) int_{-pi}^{pi} cos(n tau - x sin tau) dtau; the trapezoid
    # rule on a periodic analytic integrand is exact once N > x + n + 40.
    N = 512
    tau = 2.0 * np.pi * np.arange(N) / N
    for n in (0, 1, 2, 5, 17, 40):
        for x in (0.01, 1.0, 3.3, 12.0, 40.0, 100.0):
            ref = np.mean(np.cos(n * tau - x * np.sin(tau)))
            v = direct.besselj(n, x)
            assert abs(v - ref) < 2e-14, (n, x, v, ref)


def test_paper_integral_for_j0():
    # J_0(x) = (1/pi) int_0^pi cos(x cos theta) dtheta  (Sec. 1)
    N = 400
    theta = (np.arange(N) + 0.5) * np.pi / N          # midpoint rule (exact here)
    for x in (0.5, 5.0, 31.5, 80.0):
        ref = np.mean(np.cos(x * np.cos(theta)))
        assert abs(direct.besselj(0, x) - ref) < 2e-14


def test_three_term_recurrence():
    # J_{n-1}(x) + J_{n+1}(x) = (2n/x) J_n(x), across all evaluation branches
    for x in (0.7, 1.9, 2.1, 9.0, 24.9, 25.1, 80.0, 700.0, 3.0e3, 9.7e4):
        for n in range(1, 100, 7):
            a = direct.besselj(n - 1, x)
            b = direct.besselj(n + 1, x)
            c = direct.besselj(n, x)
            scale = abs(a) + abs(b) + abs(2.0 * n / x * c) + 1e-300
            assert abs(a + b - 2.0 * n / x * c) <= 2e-14 * max(scale, envelope(x)), (n, x)


def test_neumann_sum_of_squares():
    # J_0(x)^2 + 2 sum_{k>=1} J_k(x)^2 = 1
    for x in (0.5, 3.0, 30.0, 300.0):
        kmax = int(x + 80)
        j = np.array([direct.besselj(k, x) for k in range(kmax + 1)])
        s = j[0] ** 2 + 2.0 * np.sum(j[1:] ** 2)
        assert abs(s - 1.0) < 1e-14


def _closed_half_integer(nu2, x):
    """Spherical-Bessel closed forms for J_{nu2/2}."""
    a = np.sqrt(2.0 / (np.pi * x))
    if nu2 == 1:
        return a * np.sin(x)
    if nu2 == -1:
        return a * np.cos(x)
    if nu2 == 3:
        return a * (np.sin(x) / x - np.cos(x))
    if nu2 == 5:
        return a * ((3.0 / x ** 2 - 1.0) * np.sin(x) - 3.0 * np.cos(x) / x)
    raise ValueError(nu2)


@pytest.mark.parametrize("nu2", [1, -1, 3, 5])
def test_hankel_expansion_exact_at_half_integer(nu2):
    # At half-integer order a_k(nu) vanishes for k > |nu| - 1/2, so Hankel's
    # expansion (Sec. 3.2) terminates and equals J_nu.  This pins the
    # coefficient formula (second factor 4nu^2 - 9) and the phase -(2nu+1)pi/4.
    x = np.array([0.3, 1.0, 2.5, 10.0, 77.7, 1234.5])
    v = direct.hankel_series(nu2 / 2.0, x, nterms=8)
    ref = _closed_half_integer(nu2, x)
    assert np.all(np.abs(v - ref) <= 5e-15 * np.maximum(1.0, np.abs(ref)) * (1 + 1 / x))


def test_direct_sum_against_mpmath():
    rng = np.random.default_rng(5)
    r = rng.uniform(0.0, 1.0, 9)
    w = rng.uniform(0.0, 3000.0, 7)
    c = rng.standard_normal(9)
    for nu in (0, 3, -2):
        g = direct.dht(nu, r, c, w)
        for j in range(7):
            ref = mpmath.fsum(mpmath.mpf(float(c[k])) *
                              mpmath.besselj(nu, mpmath.mpf(float(w[j])) * mpmath.mpf(float(r[k])))
                              for k in range(9))
            assert abs(g[j] - float(ref)) < 1e-14 * float(np.sum(np.abs(c)))
