"""Pins of the disk solver's oracle (Sec. 5.3) against closed forms.

A field made of a few Dirichlet eigenfunctions psi_jl = J_l(j_{l,j} r) e^{i l theta}
(the planted modes beta_jl, real-valued: beta_{j,-l} = (-1)^l conj(beta_jl)),
sampled with SciPy's J_l, is a closed-form test of every step:

* its forcing f = (Delta + kappa^2) u = sum (kappa^2 - j_{l,j}^2) beta_jl psi_jl
  must come back from the analysis as alpha_jl = (kappa^2 - j_{l,j}^2) beta_jl
  in the planted entries and 0 elsewhere (orthogonality of the J_l(j_{l,j} r)
  under r dr, their norm J_{l+1}(j_{l,j})^2 / 2, and of e^{i l theta} on the
  trapezoid grid);
* the Helmholtz solve of that f must return u itself on the grid;
* the synthesis of the planted coefficients must return u.
A sign error in the angular exponent, a dropped factor r, a wrong
normalisation or a wrong eigenvalue moves or rescales the recovered entries.
"""
import numpy as np
import pytest
from scipy import special

import workloads
from oracle import fb

KAPPA = 25.0          # the paper's example


def planted(m=48, t=32, L=8, J=10, seed=3):
    r, wr, zeros, _ = workloads.disk(m, t, L, J, seed=seed)
    rng = np.random.default_rng(seed)
    beta = np.zeros((2 * L + 1, J), dtype=np.complex128)
    for l in range(0, 4):
        for j in range(4):
            v = rng.standard_normal() + (1j * rng.standard_normal() if l else 0.0)
            beta[l + L, j] = v
            beta[-l + L, j] = (-1) ** l * np.conj(v)
    theta = 2.0 * np.pi * np.arange(t) / t
    u = np.zeros((m, t))
    f = np.zeros((m, t))
    for l in range(-L, L + 1):
        for j in range(J):
            b = beta[l + L, j]
            if b == 0:
                continue
            z = zeros[abs(l), j]
            psi = np.outer(special.jv(l, z * r), np.exp(1j * l * theta))
            u += np.real(b * psi)
            f += np.real((KAPPA ** 2 - z ** 2) * b * psi)
    return r, wr, zeros, beta, u, f


def test_analysis_recovers_planted_coefficients():
    r, wr, zeros, beta, u, f = planted()
    L = beta.shape[0] // 2
    alpha = fb.analysis(L, r, wr, f, zeros)
    expect = np.array([(KAPPA ** 2 - zeros[abs(l)] ** 2) * beta[l + L] for l in range(-L, L + 1)])
    scale = np.abs(expect).max()
    assert np.abs(alpha - expect).max() <= 1e-11 * scale


def test_helmholtz_returns_planted_field():
    r, wr, zeros, beta, u, f = planted()
    L = beta.shape[0] // 2
    got, alpha, b = fb.helmholtz(KAPPA, L, r, wr, f, zeros)
    assert np.abs(b - beta).max() <= 1e-11 * np.abs(beta).max()
    assert np.abs(got - u).max() <= 1e-11 * np.abs(u).max()


def test_synthesis_of_planted_coefficients():
    r, wr, zeros, beta, u, f = planted()
    L = beta.shape[0] // 2
    got = fb.synthesis(L, r, f.shape[1], beta, zeros)
    assert np.abs(got - u).max() <= 1e-13 * np.abs(u).max() * 10


@pytest.mark.parametrize("l", [0, 1, 5])
def test_single_radial_mode_normalisation(l):
    """f = J_l(z r) cos(l theta) for one zero z: alpha_{j,+-l} = 1/2 (1 for
    l = 0) at that zero and 0 at the other zeros of the same order."""
    m, t, L, J = 40, 16, 6, 6
    r, wr, zeros, _ = workloads.disk(m, t, L, J, seed=0)
    theta = 2.0 * np.pi * np.arange(t) / t
    z = zeros[l, 2]
    f = np.outer(special.jv(l, z * r), np.cos(l * theta))
    alpha = fb.analysis(L, r, wr, f, zeros)
    want = np.zeros_like(alpha)
    if l == 0:
        want[L, 2] = 1.0
    else:
        want[L + l, 2] = 0.5
        want[L - l, 2] = 0.5 * (-1) ** l        # J_{-l} = (-1)^l J_l
    assert np.abs(alpha - want).max() <= 1e-12
