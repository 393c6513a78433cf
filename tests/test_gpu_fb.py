"""The disk solver (Sec. 5.3) on the GPU against the oracle and closed forms,
for both ways of taking the radial sums (the library's transforms, and the
direct sums with J_l evaluated in place):

* analysis of a random smooth forcing (m = 64 Gauss-Legendre radii, t = 64
  angles, L = 20, J = 24) against the oracle's direct sums: every alpha_jl
  within nrm_jl sum_k wr_k r_k (4 eps |F_l(r_k)| + 10 log2(t) u mean_s
  |f(r_k, .)|) -- the transform's per-entry bound eps |c|_1 on the real and
  imaginary parts, plus the rounding of the angular sums (FFT on one side,
  the explicit sum on the other, absolute in F_l, |J_l| <= 1), times the
  normalisation nrm_jl = 2 / J_{l+1}^2 -- and relative l2 <= 10 eps;
* synthesis of random decaying coefficients: every u within
  4 eps sum_jl |beta_jl|;
* the Helmholtz solve (kappa = 25, the paper's example) of the planted-mode
  forcing returns the planted field and coefficients, and agrees with the
  oracle's solve of a random forcing;
* the largest orders (L = 100, t = 256, m = 256 and the benchmarked m = 512,
  J = 128, eps = 1e-8) on sampled orders against the oracle;
* edge cases: L = 0 with t = 2, J = 1, t = 4096, and m, J not multiples of
  the direct kernels' 64-wide tiles (ragged tails).
"""
import numpy as np
import pytest
import torch
from scipy import special

import workloads
from oracle import direct, fb

pytestmark = pytest.mark.gpu

KAPPA = 25.0


@pytest.fixture(scope="module")
def nuht():
    import paper_2411_09583_amd as lib
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib.load_library()
    return lib


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def alpha_bar(L, r, wr, f, zeros, eps):
    """nrm_jl sum_k wr_k r_k (4 eps |F_l(r_k)| + 10 log2(t) u mean_s |f(r_k, .)|)."""
    t = f.shape[1]
    theta = 2.0 * np.pi * np.arange(t) / t
    u = np.finfo(np.float64).eps / 2
    fft_err = 10.0 * max(np.log2(t), 1.0) * u * np.mean(np.abs(f), axis=1)
    bar = np.zeros((2 * L + 1, zeros.shape[1]))
    for l in range(-L, L + 1):
        F = (f @ np.exp(-1j * l * theta)) / t
        s = np.sum(wr * r * (4.0 * eps * (np.abs(F.real) + np.abs(F.imag)) + fft_err))
        nrm = 2.0 / direct.besselj(l + 1, zeros[abs(l)]) ** 2
        bar[l + L] = nrm * s
    return bar


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


METHODS = ["transform", "direct"]


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("eps", [1e-12, 1e-8])
def test_analysis_against_oracle(nuht, eps, method):
    m, t, L, J = 64, 64, 20, 24
    r, wr, zeros, f = workloads.disk(m, t, L, J, seed=11)
    s = nuht.DiskSolver(dev(r), dev(wr), t, dev(zeros), eps, method=method)
    a = host(s.analysis(dev(f)))
    s.close()
    a1 = fb.analysis(L, r, wr, f, zeros)
    err = np.abs(a - a1)
    print("eps", eps, "rel_l2", rel_l2(a, a1), "max err / bar", (err / alpha_bar(L, r, wr, f, zeros, eps)).max())
    assert rel_l2(a, a1) <= 10 * eps
    assert np.all(err <= alpha_bar(L, r, wr, f, zeros, eps))


@pytest.mark.parametrize("method", METHODS)
def test_synthesis_against_oracle(nuht, method):
    m, t, L, J, eps = 64, 64, 20, 24, 1e-12
    r, wr, zeros, _ = workloads.disk(m, t, L, J, seed=12)
    rng = np.random.default_rng(13)
    decay = np.exp(-0.1 * np.abs(np.arange(-L, L + 1)))[:, None] * np.exp(-0.1 * np.arange(J))[None, :]
    beta = (rng.standard_normal((2 * L + 1, J)) + 1j * rng.standard_normal((2 * L + 1, J))) * decay
    s = nuht.DiskSolver(dev(r), dev(wr), t, dev(zeros), eps, method=method)
    u = host(s.synthesis(dev(beta)))
    s.close()
    u1 = fb.synthesis(L, r, t, beta, zeros)
    bar = 4 * eps * np.sum(np.abs(beta.real) + np.abs(beta.imag))
    print("max err", np.abs(u - u1).max(), "bar", bar)
    assert np.abs(u - u1).max() <= bar


def planted(m, t, L, J, seed):
    r, wr, zeros, _ = workloads.disk(m, t, L, J, seed=seed)
    rng = np.random.default_rng(seed)
    beta = np.zeros((2 * L + 1, J), dtype=np.complex128)
    for l in range(0, 5):
        for j in range(5):
            v = rng.standard_normal() + (1j * rng.standard_normal() if l else 0.0)
            beta[l + L, j] = v
            beta[-l + L, j] = (-1) ** l * np.conj(v)
    theta = 2.0 * np.pi * np.arange(t) / t
    u = np.zeros((m, t))
    f = np.zeros((m, t))
    for l in range(-4, 5):
        for j in range(5):
            z = zeros[abs(l), j]
            psi = np.outer(special.jv(l, z * r), np.exp(1j * l * theta))
            u += np.real(beta[l + L, j] * psi)
            f += np.real((KAPPA ** 2 - z ** 2) * beta[l + L, j] * psi)
    return r, wr, zeros, beta, u, f


@pytest.mark.parametrize("method", METHODS)
def test_helmholtz_planted_modes(nuht, method):
    m, t, L, J, eps = 64, 32, 10, 16, 1e-12
    r, wr, zeros, beta, u, f = planted(m, t, L, J, seed=14)
    s = nuht.DiskSolver(dev(r), dev(wr), t, dev(zeros), eps, method=method)
    ug, ag, bg = s.helmholtz(KAPPA, dev(f), return_coefficients=True)
    ug, bg = host(ug), host(bg)
    s.close()
    print("beta err", np.abs(bg - beta).max(), "u err", np.abs(ug - u).max())
    assert np.abs(bg - beta).max() <= 1e-9 * np.abs(beta).max()
    assert np.abs(ug - u).max() <= 1e-9 * np.abs(u).max()


@pytest.mark.parametrize("method", METHODS)
def test_helmholtz_against_oracle(nuht, method):
    m, t, L, J, eps = 48, 32, 12, 20, 1e-12
    r, wr, zeros, f = workloads.disk(m, t, L, J, seed=15)
    s = nuht.DiskSolver(dev(r), dev(wr), t, dev(zeros), eps, method=method)
    ug, ag, bg = s.helmholtz(KAPPA, dev(f), return_coefficients=True)
    ug, ag, bg = host(ug), host(ag), host(bg)
    s.close()
    u1, a1, b1 = fb.helmholtz(KAPPA, L, r, wr, f, zeros)
    print("alpha rel", rel_l2(ag, a1), "beta rel", rel_l2(bg, b1), "u rel", rel_l2(ug, u1))
    assert rel_l2(ag, a1) <= 1e-11
    assert rel_l2(bg, b1) <= 1e-11
    assert rel_l2(ug, u1) <= 1e-11


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("m,seed", [(256, 16), (512, 190)])   # the second is the benchmarked solve
def test_largest_orders_sampled(nuht, method, m, seed):
    t, L, J, eps = 256, 100, 128, 1e-8
    r, wr, zeros, f = workloads.disk(m, t, L, J, seed=seed)
    s = nuht.DiskSolver(dev(r), dev(wr), t, dev(zeros), eps, method=method)
    a = host(s.analysis(dev(f)))
    s.close()
    theta = 2.0 * np.pi * np.arange(t) / t
    for l in (0, 1, 37, -50, 99, -100, 100):
        F = (f @ np.exp(-1j * l * theta)) / t
        c = wr * r * F
        z = zeros[abs(l)]
        a1 = 2.0 * (direct.dht(l, r, c.real, z) + 1j * direct.dht(l, r, c.imag, z)) / direct.besselj(l + 1, z) ** 2
        fft_err = 10.0 * np.log2(t) * np.finfo(np.float64).eps / 2 * np.mean(np.abs(f), axis=1)
        bar = (2.0 / direct.besselj(l + 1, z) ** 2) * np.sum(
            wr * r * (4 * eps * (np.abs(F.real) + np.abs(F.imag)) + fft_err))
        err = np.abs(a[l + L] - a1)
        print("l", l, "max err / bar", (err / bar).max())
        assert np.all(err <= bar)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("m,t,L,J", [(16, 2, 0, 1), (24, 4, 1, 3), (32, 4096, 30, 8), (100, 128, 40, 70)])
def test_edge_sizes(nuht, m, t, L, J, method):
    eps = 1e-12
    r, wr, zeros, f = workloads.disk(m, t, L, J, seed=17)
    s = nuht.DiskSolver(dev(r), dev(wr), t, dev(zeros), eps, method=method)
    a = host(s.analysis(dev(f)))
    u = host(s.helmholtz(3.0, dev(f)))
    s.close()
    a1 = fb.analysis(L, r, wr, f, zeros)
    u1, _, _ = fb.helmholtz(3.0, L, r, wr, f, zeros)
    assert np.all(np.abs(a - a1) <= alpha_bar(L, r, wr, f, zeros, eps) + 1e-300)
    assert np.abs(u - u1).max() <= 1e-10 * max(np.abs(u1).max(), 1e-300)
