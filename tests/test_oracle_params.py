"""Pins for the oracle's expansion parameters and expansions (CPU only).

* (M, L) = (4, 31) at nu = 0, eps = 1e-12 is the pair the paper prints for its
  Fig. 1 ("31-term local and 4-term asymptotic" expansions of J_0).
* The asymptotic bound of eq. asy-error really bounds the M-term expansion's
  error against the true J_nu, and it is tight at the crossover z.
* The Wimp expansion with the local rank L is eps-accurate on the whole local
  region [0, z]; the argument x/2 of its coefficients is pinned by Neumann's
  addition theorem (the expansion at y = 1), evaluated with mpmath.
"""
import mpmath
import numpy as np
import pytest

from oracle import direct
from oracle import method
from oracle import params as prm

mpmath.mp.dps = 40


def test_printed_fig1_parameters():
    M, z, L = prm.parameters(0, 1e-12)
    assert (M, L) == (4, 31)


def test_num_asy_terms_cap_and_growth():
    assert prm.num_asy_terms(0, 1e-12) == 4
    assert prm.num_asy_terms(100, 1e-15) == 20          # the cap of 20
    assert prm.num_asy_terms(-10, 1e-12) == prm.num_asy_terms(10, 1e-12)
    ms = [prm.num_asy_terms(0, 10.0 ** -e) for e in range(4, 16)]
    assert ms == sorted(ms)


@pytest.mark.parametrize("nu,eps", [(0, 1e-12), (1, 1e-12), (5, 1e-12), (10, 1e-12),
                                    (0, 1e-6), (63, 1e-12), (3, 1e-9)])
def test_crossover_is_root_of_bound(nu, eps):
    M, z, L = prm.parameters(nu, eps)
    assert abs(prm.asy_bound(nu, M, z) - eps) <= 1e-12 * eps
    # B^asy decreases through the root
    assert prm.asy_bound(nu, M, 0.999 * z) > eps > prm.asy_bound(nu, M, 1.001 * z)


@pytest.mark.parametrize("nu", [0, 1, 2, 5, 10])
def test_asymptotic_error_within_bound_and_tight(nu):
    eps = 1e-12
    M, z, L = prm.parameters(nu, eps)
    xs = np.concatenate([np.linspace(z, 1.3 * z, 150), np.geomspace(1.3 * z, 200 * z, 150)])
    h = np.array([direct.asy_block_apply(nu, M, [x], [1.0], [1.0])[0] for x in xs])
    jt = np.array([float(mpmath.besselj(nu, mpmath.mpf(float(x)))) for x in xs])
    err = np.abs(h - jt)
    bound = np.array([prm.asy_bound(nu, M, x) for x in xs])
    assert np.all(err <= bound * (1 + 1e-6) + 2e-16)
    assert err[:150].max() > 0.1 * eps                  # crossover is not loose


@pytest.mark.parametrize("nu", [0, 1, 2, 4, 5, 6, 10])
def test_wimp_expansion_accurate_on_local_region(nu):
    # max over w r <= z of |J_nu(w r) - sum_{l<=L} C_l(w R) T(r/R)| <= eps,
    # with R = 1 and w in [0, z] (the bound depends only on the product z).
    eps = 1e-12
    M, z, L = prm.parameters(nu, eps)
    w = np.linspace(0.0, z, 61)
    y = np.linspace(0.0, 1.0, 41)
    C = method.wimp_coefficients(nu, L, w)              # (L+1, 61)
    odd = nu % 2
    T = method.chebyshev_t(2 * L + odd, y)[odd::2]      # (L+1, 41)
    approx = C.T @ T                                    # (61, 41)
    worst = 0.0
    for i in range(w.size):
        exact = np.array([float(mpmath.besselj(nu, mpmath.mpf(float(w[i])) * mpmath.mpf(float(t))))
                          for t in y])
        worst = max(worst, float(np.max(np.abs(approx[i] - exact))))
    assert worst <= eps, worst


@pytest.mark.parametrize("nu", [0, 2, 6, 1, 3])
def test_wimp_coefficients_neumann_addition(nu):
    # At y = 1 every T(1) = 1, so sum_l C_l(x) = J_nu(x).  Written with
    # C_l(x) = delta_l J_{nu/2+l}(x/2) J_{nu/2-l}(x/2) this is Neumann's addition
    # theorem J_n(2s) = sum_k J_k(s) J_{n-k}(s); all in mpmath.
    L = 60
    for x in (0.7, 9.0, 31.0, 50.0):
        s = mpmath.mpf(x) / 2
        if nu % 2 == 0:
            a = nu // 2
            tot = sum((1 if l == 0 else 2) * mpmath.besselj(a + l, s) * mpmath.besselj(a - l, s)
                      for l in range(L + 1))
        else:
            a = (nu - 1) // 2
            tot = sum(2 * mpmath.besselj(a + 1 + l, s) * mpmath.besselj(a - l, s) for l in range(L + 1))
        assert abs(float(tot) - float(mpmath.besselj(nu, mpmath.mpf(x)))) < 1e-15
        # and the oracle's coefficients agree with these
        C = method.wimp_coefficients(nu, L, np.array([x]))
        assert abs(C[:, 0].sum() - float(mpmath.besselj(nu, mpmath.mpf(x)))) < 1e-14


def test_wimp_printed_argument_is_a_garble():
    # With the printed argument (x instead of x/2) the expansion is far from J_0.
    L = 31
    x = 20.0
    a = sum((1 if l == 0 else 2) * direct.besselj(l, x) * direct.besselj(-l, x) for l in range(L + 1))
    assert abs(a - direct.besselj(0, x)) > 1e-2


def test_local_rank_is_minimal():
    for nu, eps in [(0, 1e-12), (5, 1e-12), (10, 1e-6), (63, 1e-12)]:
        M, z, L = prm.parameters(nu, eps)
        assert prm.local_bound(nu, L, z) < eps
        assert L == 0 or prm.local_bound(nu, L - 1, z) >= eps


def test_half_integer_order_hankel_coefficients_vanish():
    # a_k(1/2) = 0 for k >= 1 and a_k(3/2) = 0 for k >= 2 (terminating series)
    assert direct.hankel_coef(0.5, 1) == 0.0
    assert direct.hankel_coef(1.5, 1) != 0.0 and direct.hankel_coef(1.5, 2) == 0.0
    assert abs(prm.hankel_coef(7, 3) - direct.hankel_coef(7, 3)) <= 1e-15 * abs(prm.hankel_coef(7, 3))


@pytest.mark.parametrize("nu,eps", [(0, 1e-12), (1, 1e-10), (10, 1e-8), (37, 1e-8), (100, 1e-8)])
def test_tail_local_rank_keeps_the_local_expansion_within_eps(nu, eps):
    """With the tail rank L, the Wimp expansion sum_{l <= L} C_l(x) T_{2l(+1)}(y)
    reproduces J_nu(x y) to eps at random x in (0, z], y in [0, 1] -- J from
    mpmath, T from numpy's Chebyshev module, independent of the rank rule --
    and L never exceeds Lemma 3.1's."""
    import mpmath
    from numpy.polynomial import chebyshev
    M, z, L_lemma = prm.parameters(nu, eps)
    L, _ = prm.tail_local_rank(nu, eps, z, L_lemma)
    assert L <= L_lemma
    rng = np.random.default_rng(nu)
    a = nu // 2
    worst = 0.0
    for _ in range(25):
        x = z * rng.uniform(0.05, 1.0)
        y = rng.uniform(0.0, 1.0)
        s = mpmath.mpf(0)
        for l in range(L + 1):
            if nu % 2 == 0:
                C = (1 if l == 0 else 2) * mpmath.besselj(a + l, x / 2) * mpmath.besselj(a - l, x / 2)
                T = chebyshev.chebval(y, [0] * (2 * l) + [1])
            else:
                C = 2 * mpmath.besselj(a + 1 + l, x / 2) * mpmath.besselj(a - l, x / 2)
                T = chebyshev.chebval(y, [0] * (2 * l + 1) + [1])
            s += C * T
        worst = max(worst, abs(float(s - mpmath.besselj(nu, x * y))))
    print("nu", nu, "eps", eps, "L lemma", L_lemma, "L tail", L, "worst", worst)
    assert worst <= eps
