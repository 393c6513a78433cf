"""The p = O(n) study (Sec. 5.1): Fourier-Bessel and exponentially distributed
points and frequencies, against the oracle's direct sum.

* Fourier-Bessel (w_j = j_{nu,j}, r_k = j_{nu,k}/j_{nu,n+1}) for nu = 0, 1, 7
  and exponential (log-spaced w = r over [n^(-1/2), n^(1/2)]) for nu = 0, 3, at
  n = m = 3000 and eps = 1e-8, 1e-12: relative l2 <= 2 max(eps, 2e-14) and every
  entry within 2 eps |c|_1 (the exponential case gives the deepest partition);
* both at n = m = 1e6, nu = 0, eps = 1e-8 (the configuration of the paper's
  runtime figure) on 64 sampled outputs, each a direct sum over all points;
* Fourier-Bessel at n = m = 1e6 at the ends of the runtime study's order sweep
  (nu = 10, 100 at eps = 1e-8) and tolerance sweep (eps = 1e-4, 1e-15 at
  nu = 0), sampled the same way;
* the accuracy study: Fourier-Bessel, n = m = 1e5, c with 1000 N(0, 1)
  nonzeros, reference = the direct sum over the nonzeros only, for eps from
  1e-4 to 1e-14: relative l2 <= max(eps, 1.5e-14).  Seen: 1.4e-5, 4.6e-7,
  3.9e-9, 5.6e-11, 4.8e-13, 9.0e-15 -- the error follows eps down to 1e-14
  without the saturation near n times machine precision that FP64 phases
  would bring, since every phase is formed exactly.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import direct

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nuht():
    import paper_2411_09583_amd as lib
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib.load_library()
    return lib


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def run(nuht, nu, eps, r, c, w):
    p = nuht.Plan(dev(r), dev(w), nu, eps)
    g = host(p.execute(dev(c)))
    info = p.info()
    p.close()
    return g, info


CASES = [("fourier_bessel", 0), ("fourier_bessel", 1), ("fourier_bessel", 7), ("exponential", 0), ("exponential", 3)]


@pytest.mark.parametrize("kind,nu", CASES)
@pytest.mark.parametrize("eps", [1e-8, 1e-12])
def test_p_equals_n_small(nuht, kind, nu, eps):
    if kind == "fourier_bessel":
        r, w, c = workloads.fourier_bessel(3000, nu, seed=140 + nu)
    else:
        r, w, c = workloads.exponential(3000, seed=150 + nu)
    g, info = run(nuht, nu, eps, r, c, w)
    g1 = direct.dht(nu, r, c, w)
    err = np.abs(g - g1)
    print(kind, nu, eps, "levels", info["levels"], "blocks", info["n_local"], info["n_asy"], info["n_direct"],
          "rel_l2", rel_l2(g, g1), "max/|c|_1", err.max() / np.sum(np.abs(c)))
    assert rel_l2(g, g1) <= 2.0 * max(eps, 2e-14)
    assert np.all(err <= 2.0 * eps * np.sum(np.abs(c)))


@pytest.mark.parametrize("kind", ["fourier_bessel", "exponential"])
def test_p_equals_n_full_size_sampled(nuht, kind):
    n, nu, eps = 1_000_000, 0, 1e-8
    if kind == "fourier_bessel":
        r, w, c = workloads.fourier_bessel(n, nu, seed=160)
    else:
        r, w, c = workloads.exponential(n, seed=161)
    g, info = run(nuht, nu, eps, r, c, w)
    idx = np.random.default_rng(162).choice(n, 64, replace=False)
    g1 = direct.dht(nu, r, c, w[idx])
    print(kind, "levels", info["levels"], "blocks", info["n_local"], info["n_asy"], info["n_direct"],
          "rel_l2", rel_l2(g[idx], g1))
    assert rel_l2(g[idx], g1) <= 2.0 * eps
    assert np.all(np.abs(g[idx] - g1) <= 2.0 * eps * np.sum(np.abs(c)))


def test_accuracy_study(nuht):
    n, nu = 100_000, 0
    r, w, _ = workloads.fourier_bessel(n, nu, seed=0)
    c = workloads.sparse_c(n, 1000, seed=170)
    nz = np.nonzero(c)[0]
    g1 = direct.dht(nu, r[nz], c[nz], w)          # the direct sum over the nonzeros
    rd, wd, cd = dev(r), dev(w), dev(c)
    errs = {}
    for eps in (1e-4, 1e-6, 1e-8, 1e-10, 1e-12, 1e-14):
        p = nuht.Plan(rd, wd, nu, eps)
        g = host(p.execute(cd))
        p.close()
        errs[eps] = rel_l2(g, g1)
        print("eps", eps, "rel_l2", errs[eps])
    for eps, e in errs.items():
        assert e <= max(eps, 1.5e-14), (eps, e)


# The order and tolerance sweeps of the runtime study (Sec. 5.1, Fourier-Bessel
# only): the two ends of each sweep at full size, on sampled outputs.
SWEEP = [(10, 1e-8), (100, 1e-8), (0, 1e-4), (0, 1e-15)]


@pytest.mark.parametrize("nu,eps", SWEEP)
def test_fourier_bessel_sweep_full_size_sampled(nuht, nu, eps):
    n = 1_000_000
    r, w, c = workloads.fourier_bessel(n, nu, seed=180 + nu)
    g, info = run(nuht, nu, eps, r, c, w)
    idx = np.random.default_rng(181).choice(n, 64, replace=False)
    g1 = direct.dht(nu, r, c, w[idx])
    bar = max(eps, 2e-14)
    print("nu", nu, "eps", eps, "M", info["M"], "L", info["L"], "levels", info["levels"],
          "blocks", info["n_local"], info["n_asy"], info["n_direct"], "rel_l2", rel_l2(g[idx], g1),
          "max/|c|_1", np.abs(g[idx] - g1).max() / np.sum(np.abs(c)))
    assert rel_l2(g[idx], g1) <= 2.0 * bar
    assert np.all(np.abs(g[idx] - g1) <= 2.0 * bar * np.sum(np.abs(c)))
