"""O3: Fourier-Bessel expansions and the Helmholtz solver on the unit disk
(Sec. 5.3), by their definitions.

TEST INFRASTRUCTURE ONLY (see :mod:`oracle`).

Grid: radii r_k with radial weights wr_k (a rule for int_0^1 g(r) dr) and the
angles theta_s = 2 pi s / t.  For orders l = -L .. L and the first J positive
zeros z_jl = j_{l,j} of J_l (j_{-l,j} = j_{l,j}):

* analysis, eq. FB-coef with the trapezoid rule in theta and the given rule
  in r, the angular integral taken as a mean (1 / 2 pi) int d theta: the
  eigenfunctions have int int |psi_jl|^2 r dr d theta = pi J_{l+1}(z_jl)^2, so
  the printed factor 2 / J_{l+1}^2 goes with the angular mean, not the plain
  integral (the pins in the tests decide this):
      F_l(r_k)  = (1 / t) sum_s f(r_k, theta_s) e^{-i l theta_s}
      alpha_jl  = 2 / J_{l+1}(z_jl)^2  sum_k wr_k r_k F_l(r_k) J_l(z_jl r_k)
* synthesis, the truncated expansion on the grid:
      u(r_k, theta_s) = Re sum_l e^{i l theta_s} sum_j beta_jl J_l(z_jl r_k)
* Helmholtz, (Delta + kappa^2) u = f with u = 0 on the circle: the Dirichlet
  eigenfunctions J_l(z_jl r) e^{i l theta} have eigenvalues lambda_jl = -z_jl^2,
  so beta_jl = alpha_jl / (lambda_jl + kappa^2).

Every radial sum is the direct sum of :mod:`oracle.direct` (O1) at the order
l itself, negative orders included; J_{l+1}(z_jl) is the oracle's own J; the
angular sums are written out as a matrix-vector product (no FFT).
"""
import numpy as np

from oracle import direct


def _angles(t):
    return 2.0 * np.pi * np.arange(t) / t


def analysis(L: int, r, wr, f, zeros):
    """alpha[l + L, j - 1] for l = -L .. L, j = 1 .. J (complex).

    r, wr: m radii and radial weights; f: m x t real samples
    f(r_k, 2 pi s / t); zeros: (L + 1) x J, row l the zeros of J_l."""
    r = np.asarray(r, dtype=np.float64)
    wr = np.asarray(wr, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    zeros = np.asarray(zeros, dtype=np.float64)
    t = f.shape[1]
    theta = _angles(t)
    J = zeros.shape[1]
    alpha = np.zeros((2 * L + 1, J), dtype=np.complex128)
    for l in range(-L, L + 1):
        F = (f @ np.exp(-1j * l * theta)) / t
        c = wr * r * F
        z = zeros[abs(l)]
        a = direct.dht(l, r, c.real, z) + 1j * direct.dht(l, r, c.imag, z)
        alpha[l + L] = 2.0 * a / direct.besselj(l + 1, z) ** 2
    return alpha


def synthesis(L: int, r, t: int, beta, zeros):
    """u[k, s] = Re sum_l e^{i l theta_s} sum_j beta[l + L, j - 1] J_l(z_jl r_k)."""
    r = np.asarray(r, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.complex128)
    zeros = np.asarray(zeros, dtype=np.float64)
    theta = _angles(t)
    u = np.zeros((r.size, t), dtype=np.float64)
    for l in range(-L, L + 1):
        z = zeros[abs(l)]
        b = beta[l + L]
        U = direct.dht(l, z, b.real, r) + 1j * direct.dht(l, z, b.imag, r)
        u += np.real(np.outer(U, np.exp(1j * l * theta)))
    return u


def divide(L: int, alpha, zeros, kappa: float):
    """beta_jl = alpha_jl / (lambda_jl + kappa^2), lambda_jl = -z_jl^2."""
    zeros = np.asarray(zeros, dtype=np.float64)
    beta = np.empty_like(np.asarray(alpha, dtype=np.complex128))
    for l in range(-L, L + 1):
        beta[l + L] = alpha[l + L] / (kappa ** 2 - zeros[abs(l)] ** 2)
    return beta


def helmholtz(kappa: float, L: int, r, wr, f, zeros):
    """(u, alpha, beta): the solution on the grid and its coefficients."""
    alpha = analysis(L, r, wr, f, zeros)
    beta = divide(L, alpha, zeros, kappa)
    return synthesis(L, r, np.asarray(f).shape[1], beta, zeros), alpha, beta
