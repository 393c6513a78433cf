"""Pins for O2 (the method-exact reference) and for the transform definition.

* O2 - O1 is pure truncation error of the expansions, which the parameter
  choice bounds by eps per matrix entry (Sec. 3.3): |O2_j - O1_j| <= eps ||c||_1.
* The discrete transform of a quadrature rule reproduces closed-form Hankel
  transforms: the unit-disk indicator of Sec. 5.2, int_0^1 J_0(w r) r dr =
  J_1(w)/w, and the Gaussian int_0^inf exp(-a r^2) J_0(w r) r dr = exp(-w^2/4a)/(2a).
"""
import mpmath
import numpy as np
import pytest

import workloads
from oracle import direct
from oracle import method


def test_o2_matches_o1_small_dense_config():
    r, w, c = workloads.small_dense(seed=1)
    eps = 1e-12
    g1 = direct.dht(0, r, c, w)
    g2 = method.nufht_reference(0, eps, r, c, w)
    assert np.max(np.abs(g2 - g1)) <= eps * np.sum(np.abs(c))
    assert np.linalg.norm(g2 - g1) / np.linalg.norm(g1) <= eps


@pytest.mark.parametrize("nu,eps", [(1, 1e-12), (2, 1e-10), (5, 1e-12), (10, 1e-12), (4, 1e-6), (-1, 1e-12)])
def test_o2_matches_o1_orders(nu, eps):
    r, w, c = workloads.uniform(700, 600, 1.0, 800.0, seed=20 + abs(nu))
    g1 = direct.dht(nu, r, c, w)
    g2 = method.nufht_reference(nu, eps, r, c, w, min_size=256)
    assert np.max(np.abs(g2 - g1)) <= eps * np.sum(np.abs(c))


def test_o2_with_points_and_frequencies_at_zero():
    r, w, c = workloads.uniform(300, 250, 1.0, 300.0, seed=4)
    r[:5] = 0.0
    w[:7] = 0.0
    for nu in (0, 3):
        g1 = direct.dht(nu, r, c, w)
        g2 = method.nufht_reference(nu, 1e-12, r, c, w, min_size=64)
        assert np.max(np.abs(g2 - g1)) <= 1e-12 * np.sum(np.abs(c))


def test_disk_indicator_closed_form():
    # Gauss-Legendre on [0, 1]: sum_k w_k r_k J_0(w r_k) = J_1(w)/w
    x, wt = np.polynomial.legendre.leggauss(300)
    r = 0.5 * (x + 1.0)
    wq = 0.5 * wt
    w = np.linspace(0.5, 200.0, 40)
    g1 = direct.dht(0, r, wq * r, w)
    g2 = method.nufht_reference(0, 1e-12, r, wq * r, w, min_size=64)
    ref = np.array([float(mpmath.besselj(1, v) / v) for v in w])
    assert np.max(np.abs(g1 - ref)) < 1e-14
    assert np.max(np.abs(g2 - ref)) < 1e-12


def test_gaussian_weber_integral():
    # int_0^inf exp(-a r^2) J_0(w r) r dr = exp(-w^2/(4a)) / (2a), a = 40,
    # with Gauss-Legendre on [0, 1.5] (the tail is below 1e-38).
    a = 40.0
    x, wt = np.polynomial.legendre.leggauss(200)
    r = 0.75 * (x + 1.0)
    wq = 0.75 * wt
    w = np.linspace(0.0, 60.0, 31)
    g = direct.dht(0, r, wq * r * np.exp(-a * r * r), w)
    ref = np.exp(-w * w / (4 * a)) / (2 * a)
    assert np.max(np.abs(g - ref)) < 1e-15


def test_sparse_input_reference():
    # Sec. 5.1.3: with few nonzeros the reference is a direct sum over them only.
    r, w, _ = workloads.uniform(5000, 300, 1.0, 1000.0, seed=8)
    c = workloads.sparse_c(5000, 40, seed=9)
    nz = np.nonzero(c)[0]
    g_full = direct.dht(0, r, c, w)
    g_nz = direct.dht(0, r[nz], c[nz], w)
    assert np.array_equal(g_full, g_nz)
