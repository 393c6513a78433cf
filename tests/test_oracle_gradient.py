"""Pins of the oracle's gradient (CPU).

* central differences of the oracle's own direct sum L = gbar . g(c, r, w)
  in every coordinate of small inputs (a sign, a factor 1/2, an exchanged
  operand or a wrong order shift each fails these);
* the derivative identity J_nu' = (J_{nu-1} - J_{nu+1})/2 against mpmath's
  derivative of J_nu, including nu = 0 (J_{-1} = -J_1).
"""
import mpmath
import numpy as np
import pytest

from oracle import direct, gradient


@pytest.mark.parametrize("nu", [0, 1, 3, -2])
def test_gradient_matches_central_differences(nu):
    rng = np.random.default_rng(100 + abs(nu))
    n, m = 23, 19
    r = rng.uniform(0.05, 1.0, n)
    w = rng.uniform(0.0, 60.0, m)
    c = rng.standard_normal(n)
    gbar = rng.standard_normal(m)
    dc, dr, dw = gradient.gradient(nu, r, c, w, gbar)

    def loss(c_, r_, w_):
        return float(np.dot(gbar, direct.dht(nu, r_, c_, w_)))

    h = 1e-5
    for k in range(n):
        e = np.zeros(n); e[k] = h
        fd_c = (loss(c + e, r, w) - loss(c - e, r, w)) / (2 * h)
        fd_r = (loss(c, r + e, w) - loss(c, r - e, w)) / (2 * h)
        assert abs(fd_c - dc[k]) <= 1e-7 * (1 + abs(dc[k]))
        assert abs(fd_r - dr[k]) <= 1e-6 * (1 + abs(dr[k]))
    for j in range(m):
        e = np.zeros(m); e[j] = h
        fd_w = (loss(c, r, w + e) - loss(c, r, w - e)) / (2 * h)
        assert abs(fd_w - dw[j]) <= 1e-6 * (1 + abs(dw[j]))


@pytest.mark.parametrize("nu", [0, 1, 4, 7])
def test_derivative_identity_against_mpmath(nu):
    mpmath.mp.dps = 30
    x = np.array([0.0, 0.3, 1.7, 6.0, 24.0, 31.0, 80.0, 300.0])
    got = gradient.besselj_prime(nu, x)
    ref = np.array([float(mpmath.besselj(nu, xx, derivative=1)) for xx in x])
    assert np.max(np.abs(got - ref)) <= 2e-15


def test_selected_entries_match_full():
    rng = np.random.default_rng(7)
    r = rng.uniform(0, 1, 40); w = rng.uniform(0, 200, 35)
    c = rng.standard_normal(40); gbar = rng.standard_normal(35)
    full = gradient.gradient(2, r, c, w, gbar)
    ic, ir, iw = np.array([0, 5, 39]), np.array([3, 17]), np.array([1, 34])
    part = gradient.gradient_at(2, r, c, w, gbar, ic, ir, iw)
    assert np.array_equal(part[0], full[0][ic])
    assert np.allclose(part[1], full[1][ir], rtol=0, atol=1e-13 * np.abs(full[1]).max())
    assert np.allclose(part[2], full[2][iw], rtol=0, atol=1e-13 * np.abs(full[2]).max())
