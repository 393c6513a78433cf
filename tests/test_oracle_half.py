"""Pins of the oracle's half-integer orders nu = n + 1/2 (CPU).

Each pin checks the oracle against something other than itself:
* J_{n+1/2}: the closed forms of DLMF 10.49 (J_{1/2} = sqrt(2/(pi x)) sin x,
  J_{3/2}, J_{5/2}) and mpmath's besselj, both at 40 digits; the three-term
  recurrence; a double-double argument against mpmath at the exact sum;
* the parameters: a_k(n + 1/2) vanish beyond k = n (the expansion is exact),
  the crossover's defining equations, minimality of L, and the bound B(L)
  against the actual truncation error measured with mpmath's J;
* the Chebyshev coefficients beta_k(x) of j_n(x y): SciPy's spherical Bessel
  function reconstructed from them, and the integral
  beta_k = eps_k (-1)^((k-n)/2) int_0^1 P_n(s) J_k(x s) ds by SciPy's quad;
* O2 at half-integer orders: within eps |c|_1 of O1 entry by entry, and the
  Gaussian Hankel transform int_0^inf e^{-a r^2} r^{nu+1} J_nu(w r) dr =
  w^nu e^{-w^2/(4a)} / (2a)^{nu+1} (DLMF 10.22.51) by quadrature through both.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate, special

from oracle import direct, method
from oracle import params as prm

mp.mp.dps = 40


def test_closed_forms():
    x = np.concatenate([np.logspace(-6, 4, 200), np.linspace(0.1, 60, 300)])
    forms = {
        0: lambda t: mp.sqrt(2 / (mp.pi * t)) * mp.sin(t),
        1: lambda t: mp.sqrt(2 / (mp.pi * t)) * (mp.sin(t) / t - mp.cos(t)),
        2: lambda t: mp.sqrt(2 / (mp.pi * t)) * ((3 / t ** 2 - 1) * mp.sin(t) - 3 * mp.cos(t) / t),
    }
    for n, f in forms.items():
        got = direct.besselj(n + 0.5, x)
        for xi, g in zip(x, got):
            ref = float(f(mp.mpf(xi)))
            env = min(1.0, math.sqrt(2.0 / (math.pi * xi)))
            assert abs(g - ref) <= 2e-15 * max(abs(ref), env), (n, xi, g, ref)


@pytest.mark.parametrize("n", [0, 3, 10, 31, 64, 99])
def test_against_mpmath(n):
    rng = np.random.default_rng(500 + n)
    x = np.concatenate([np.logspace(-5, 5, 40), rng.uniform(0.0, 2.0 * n + 40.0, 60),
                        np.linspace(max(n - 3.0, 0.1), n + 3.0, 13)])
    got = direct.besselj(n + 0.5, x)
    for xi, g in zip(x, got):
        ref = float(mp.besselj(n + mp.mpf(1) / 2, mp.mpf(xi)))
        env = min(1.0, math.sqrt(2.0 / (math.pi * xi)))
        assert abs(g - ref) <= 1e-15 * max(abs(ref), env), (n, xi, g, ref)


def test_recurrence_and_double_double_argument():
    x = np.linspace(0.3, 400.0, 997)
    for n in (1, 4, 17, 60):
        nu = n + 0.5
        jm, j0, jp = (direct.besselj(v, x) for v in (nu - 1, nu, nu + 1))
        scale = np.maximum.reduce([np.abs(jm), np.abs(jp), np.abs(2 * nu / x * j0)])
        assert np.all(np.abs(jm + jp - 2 * nu / x * j0) <= 4e-15 * np.maximum(scale, 1e-300) + 1e-300)
    # a product omega r formed exactly: the low part must move the value
    w, r = 98765.4321, 0.7654321987
    hi, lo = direct.two_prod(np.array([w]), np.array([r]))
    for n in (0, 5):
        g = direct.besselj(n + 0.5, hi, lo)[0]
        ref = float(mp.besselj(n + mp.mpf(1) / 2, mp.mpf(w) * mp.mpf(r)))
        assert abs(g - ref) <= 2e-17, (n, g, ref)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5, 3.5, 5.5, 10.5, 21.5, 63.5, 99.5])
@pytest.mark.parametrize("eps", [1e-12, 1e-6])
def test_parameters(nu, eps):
    n = int(nu - 0.5)
    M, z, L = prm.half_parameters(nu, eps)
    assert M == min(prm.num_asy_terms(nu, eps), (n + 2) // 2)
    # the expansion ends at a_n
    for k in range(n + 1, n + 6):
        assert prm.hankel_coef(nu, k) == 0.0
    assert prm.hankel_coef(nu, n) != 0.0
    assert z >= 1.0
    if 2 * M >= n + 1:
        S = sum(abs(prm.hankel_coef(nu, k)) * z ** -k for k in range(n + 1))
        assert S <= 10.0 * (1 + 1e-12)
        if z > 1.0:
            assert abs(S / 10.0 - 1.0) < 1e-10
    else:
        assert abs(prm.asy_bound(nu, M, z) / eps - 1.0) < 1e-10
    assert prm.half_local_bound(nu, L, z) < eps
    if L > 0:
        assert prm.half_local_bound(nu, L - 1, z) >= eps


@pytest.mark.parametrize("nu", [0.5, 2.5, 7.5, 12.5])
def test_local_truncation_within_bound(nu):
    # the truncated expansion against mpmath's J at random points of the local
    # region: error <= B(L) (the bound) and <= eps
    eps = 1e-10
    n = int(nu - 0.5)
    M, z, L = prm.half_parameters(nu, eps)
    rng = np.random.default_rng(int(2 * nu))
    x = rng.uniform(0.0, z, 40)
    x[0] = z
    y = rng.uniform(0.0, 1.0, 40)
    e = n % 2
    beta = method.half_coefficients(n, L, x)                     # (L+1, 40)
    T = np.array([method.chebyshev_t(2 * L + e, np.array([yi]))[e::2, 0] for yi in y])   # (40, L+1)
    approx = np.sqrt(y) * np.sqrt(2 * x / np.pi) * np.einsum("ij,ji->i", T, beta)
    ref = np.array([float(mp.besselj(nu, mp.mpf(a) * mp.mpf(b))) for a, b in zip(x, y)])
    err = np.max(np.abs(approx - ref))
    assert err <= prm.half_local_bound(nu, L, z) and err <= eps, (err, L)


@pytest.mark.parametrize("n,x", [(0, 0.8), (1, 3.0), (2, 9.5), (5, 20.0), (12, 31.0)])
def test_half_coefficients_pinned(n, x):
    L = 40
    beta = method.half_coefficients(n, L, np.array([x]))[:, 0]
    e = n % 2
    # reconstruction of SciPy's j_n on [-1, 1]
    ys = np.linspace(-1.0, 1.0, 41)
    T = method.chebyshev_t(2 * L + e, ys)[e::2]
    # 41 coefficients, each rounded at ~1e-16
    assert np.max(np.abs(beta @ T - special.spherical_jn(n, x * ys))) <= 1e-14
    # the integral form for a few k
    for l in (0, 1, 3, 7):
        k = e + 2 * l
        v, _ = integrate.quad(lambda s: special.eval_legendre(n, s) * special.jv(k, x * s), 0.0, 1.0,
                              epsabs=1e-16, epsrel=1e-13, limit=200)
        ref = (1.0 if k == 0 else 2.0) * (-1.0) ** ((k - n) // 2) * v
        assert abs(beta[l] - ref) <= 1e-14, (k, beta[l], ref)


@pytest.mark.parametrize("nu", [0.5, 1.5, 4.5, 9.5, 20.5])
def test_method_exact_against_direct(nu):
    rng = np.random.default_rng(int(10 * nu))
    r = rng.uniform(0.0, 1.0, 1200)
    w = rng.uniform(0.0, 900.0, 1000)
    c = rng.standard_normal(1200)
    eps = 1e-12
    g1 = direct.dht(nu, r, c, w)
    g2 = method.nufht_reference(nu, eps, r, c, w)
    assert np.max(np.abs(g2 - g1)) <= eps * np.sum(np.abs(c))
    assert np.linalg.norm(g2 - g1) <= eps * np.linalg.norm(g1)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_gaussian_hankel_transform(nu):
    # int_0^inf exp(-a r^2) r^(nu+1) J_nu(w r) dr = w^nu exp(-w^2/(4a)) / (2a)^(nu+1)
    a = 3.0
    x, wx = np.polynomial.legendre.leggauss(400)
    R = 12.0 / math.sqrt(a)
    r = 0.5 * R * (x + 1.0)
    c = 0.5 * R * wx * np.exp(-a * r * r) * r ** (nu + 1.0)
    w = np.linspace(0.0, 25.0, 60)
    exact = w ** nu * np.exp(-w * w / (4 * a)) / (2 * a) ** (nu + 1.0)
    g1 = direct.dht(nu, r, c, w)
    g2 = method.nufht_reference(nu, 1e-12, r, c, w, min_size=64)
    assert np.max(np.abs(g1 - exact)) <= 1e-14
    assert np.max(np.abs(g2 - exact)) <= 1e-13
