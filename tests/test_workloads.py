"""Input generators of the p = O(n) study (CPU): the Bessel zeros that place
the Fourier-Bessel points, and the two workloads' layouts.

Pins independent of the generator: the tabulated first zeros of J_0; the
oracle's J_nu (itself pinned against closed forms, recurrences and
quadrature) vanishing at every generated zero; interlacing
j_{nu,k} < j_{nu+1,k} < j_{nu,k+1}; McMahon's spacing j_{nu,k+1} - j_{nu,k} -> pi.
"""
import numpy as np
import pytest

import workloads
from oracle import direct


def test_first_zeros_of_j0():
    z = workloads.bessel_zeros(0, 3)
    ref = np.array([2.404825557695773, 5.520078110286311, 8.653727912911013])   # tabulated
    assert np.max(np.abs(z - ref) / ref) <= 1e-14


@pytest.mark.parametrize("nu", [0, 1, 5, 20, 63])
def test_zeros_are_zeros(nu):
    z = workloads.bessel_zeros(nu, 400)
    assert np.all(np.diff(z) > 0) and z[0] > nu
    j = direct.besselj(nu, z)
    env = np.sqrt(2.0 / (np.pi * z))
    # |J(z_k)| ~ |J'(z_k)| |dz| ~ env |dz|: each zero is right to two ulps
    # (the largest seen is 0.81 ulp)
    assert np.all(np.abs(j) / env <= 2.0 * np.spacing(z))


@pytest.mark.parametrize("nu", [0, 3, 10])
def test_interlacing_and_spacing(nu):
    a = workloads.bessel_zeros(nu, 2000)
    b = workloads.bessel_zeros(nu + 1, 2000)
    assert np.all(a < b) and np.all(b[:-1] < a[1:])
    gaps = np.diff(a)
    assert abs(gaps[-1] - np.pi) < 1e-5          # McMahon: the gap is pi - O(1/k^2)


def test_fourier_bessel_layout():
    r, w, c = workloads.fourier_bessel(500, 2, seed=1)
    z = workloads.bessel_zeros(2, 501)
    assert r.size == w.size == c.size == 500
    assert np.array_equal(w, z[:500]) and np.allclose(r * z[500], z[:500], rtol=1e-15, atol=0)
    assert 0.0 < r[0] and r[-1] < 1.0


def test_exponential_layout():
    r, w, c = workloads.exponential(1001, seed=2)
    assert np.array_equal(r, w)
    assert abs(r[0] - 1001 ** -0.5) <= 1e-15 * r[0] and abs(r[-1] - 1001 ** 0.5) <= 1e-13 * r[-1]
    ratios = r[1:] / r[:-1]
    assert np.max(np.abs(ratios - ratios[0])) <= 1e-13
