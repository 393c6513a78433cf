"""Half-integer orders nu = n + 1/2 on the GPU (nuht_plan_half) against the oracle.

Bars as for integer orders: relative l2 and normwise max error against the
direct sum (O1) at most eps = 1e-12 in FP64, the GPU against the
method-exact reference (O2, same parameters and partition) well below eps,
and at eps = 1e-6 with FP32 spreading rel-l2 <= eps and every entry within
eps |c|_1.  Cases span the exact (terminating) asymptotic expansions of low
orders, Newton crossovers of higher ones, direct-heavy partitions, the edge
cases of the method, the adjoint, the gradient (orders nu -+ 1 are
half-integers too) and the radial 3-D workload at n = m = 1e6.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import direct, gradient as ograd, method
from oracle import params as oparams

pytestmark = pytest.mark.gpu

TOL = 1e-12


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
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def rel_max(a, b):
    mb = np.max(np.abs(b)) if b.size else 0.0
    return np.max(np.abs(a - b)) / mb if mb > 0 else (np.max(np.abs(a - b)) if a.size else 0.0)


def run(nuht, nu, eps, r, c, w, **opts):
    p = nuht.Plan(dev(r), dev(w), nu, eps, **opts)
    g = host(p.execute(dev(c)))
    info = p.info()
    p.close()
    return g, info


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5, 3.5, 5.5, 10.5, 21.5, 40.5])
def test_half_orders(nuht, nu):
    r, w, c = workloads.uniform(2500, 2200, 1.0, 2000.0, seed=400 + int(2 * nu))
    g, info = run(nuht, nu, 1e-12, r, c, w)
    M, z, L = oparams.half_parameters(nu, 1e-12)
    print(nu, "(M, z, L)", (info["M"], info["z"], info["L"]), "blocks", info["n_local"], info["n_asy"],
          info["n_direct"], flush=True)
    assert info["half_order"] == 1 and info["nu"] == int(nu)
    assert (info["M"], info["L"]) == (M, L) and abs(info["z"] - z) <= 1e-13 * z
    g1 = direct.dht(nu, r, c, w)
    print("  vs direct sum: rel l2 %.2e rel max %.2e" % (rel_l2(g, g1), rel_max(g, g1)))
    assert rel_l2(g, g1) <= TOL and rel_max(g, g1) <= TOL
    g2 = method.nufht_reference(nu, 1e-12, r, c, w, min_size=info["min_size"])
    assert rel_l2(g, g2) <= 2e-13 and rel_max(g, g2) <= 2e-13


@pytest.mark.parametrize("nu,min_size", [(1.5, 16), (4.5, 5000), (12.5, 300)])
def test_half_direct_heavy(nuht, nu, min_size):
    r, w, c = workloads.uniform(1800, 1600, 1.0, 900.0, seed=420 + int(2 * nu))
    g, info = run(nuht, nu, 1e-12, r, c, w, min_size=min_size)
    assert info["n_direct"] > 0
    g1 = direct.dht(nu, r, c, w)
    assert rel_l2(g, g1) <= TOL and rel_max(g, g1) <= TOL


def test_half_edge_cases(nuht):
    rng = np.random.default_rng(430)
    r = rng.uniform(0, 1, 700); r[:20] = 0.0; r[20:60] = r[60]
    w = rng.uniform(0, 800, 600); w[:15] = 0.0; w[15:40] = w[40]
    c = rng.standard_normal(700)
    for nu in (0.5, 1.5, 6.5):
        g, _ = run(nuht, nu, 1e-12, r, c, w, min_size=64)
        g1 = direct.dht(nu, r, c, w)
        assert rel_l2(g, g1) <= TOL and rel_max(g, g1) <= TOL, nu
        assert np.all(g[w == 0.0] == 0.0)                 # J_nu(0) = 0 for nu > 0
    g, _ = run(nuht, 2.5, 1e-12, r[:1] + 0.3, c[:1], w)
    assert rel_l2(g, direct.dht(2.5, r[:1] + 0.3, c[:1], w)) <= TOL
    # wholly local and wholly asymptotic matrices
    g, info = run(nuht, 3.5, 1e-12, r * 0.001, c, w * 0.001)
    assert info["n_asy"] == 0 and rel_l2(g, direct.dht(3.5, r * 0.001, c, w * 0.001)) <= TOL
    g, info = run(nuht, 0.5, 1e-12, r + 1.0, c, w + 10.0)
    assert info["n_local"] == 0 and rel_l2(g, direct.dht(0.5, r + 1.0, c, w + 10.0)) <= TOL
    # empty inputs
    g, _ = run(nuht, 1.5, 1e-12, np.zeros(0), np.zeros(0), w[:7])
    assert np.array_equal(g, np.zeros(7))
    # invalid orders
    with pytest.raises(nuht.NuhtError):
        nuht.Plan(dev(r), dev(w), -0.5, 1e-12)
    with pytest.raises(nuht.NuhtError):
        nuht.Plan(dev(r), dev(w), 100.5, 1e-12)
    with pytest.raises(ValueError):
        nuht.Plan(dev(r), dev(w), 0.25, 1e-12)


@pytest.mark.parametrize("nu", [0.5, 2.5])
def test_half_fp32_and_tolerances(nuht, nu):
    r, w, c = workloads.uniform(3000, 2500, 1.0, 2500.0, seed=440 + int(2 * nu))
    g1 = direct.dht(nu, r, c, w)
    g32, _ = run(nuht, nu, 1e-6, r, c, w, precision=nuht.NUHT_FP32_SPREAD)
    assert rel_l2(g32, g1) <= 1e-6 and np.max(np.abs(g32 - g1)) <= 1e-6 * np.sum(np.abs(c))
    for eps in (1e-4, 1e-8, 1e-14):
        g, _ = run(nuht, nu, eps, r, c, w)
        assert rel_l2(g, g1) <= max(eps, 2e-14), (eps, rel_l2(g, g1))


def test_half_adjoint(nuht):
    r, w, _ = workloads.uniform(2500, 2200, 1.0, 1500.0, seed=450)
    y = np.random.default_rng(451).standard_normal(w.size)
    for nu in (0.5, 3.5):
        p = nuht.Plan(dev(r), dev(w), nu, 1e-12)
        cb = host(p.adjoint(dev(y)))
        p.close()
        ref = direct.dht(nu, w, y, r)
        assert rel_l2(cb, ref) <= TOL and rel_max(cb, ref) <= TOL


def test_half_gradient(nuht):
    r, w, c = workloads.uniform(1500, 1300, 1.0, 800.0, seed=460)
    gbar = np.random.default_rng(461).standard_normal(w.size)
    nu = 2.5
    p = nuht.Plan(dev(r), dev(w), nu, 1e-12)
    dc, dr, dw = (host(t) for t in p.gradient(dev(c), dev(gbar)))
    p.close()
    rc, rr, rw = ograd.gradient(nu, r, c, w, gbar)
    for got, ref in ((dc, rc), (dr, rr), (dw, rw)):
        assert rel_l2(got, ref) <= TOL, rel_l2(got, ref)
    # order 1/2 has no order -1/2 neighbour: dr and domega are refused, dc works
    q = nuht.Plan(dev(r), dev(w), 0.5, 1e-12)
    with pytest.raises(nuht.NuhtError):
        q.gradient(dev(c), dev(gbar))
    dc, _, _ = q.gradient(dev(c), dev(gbar), want_r=False, want_omega=False)
    assert rel_l2(host(dc), direct.dht(0.5, w, gbar, r)) <= TOL
    q.close()


def test_radial_3d_full_size(nuht):
    r, w, c = workloads.radial_3d()
    p = nuht.Plan(dev(r), dev(w), 0.5, 1e-12)
    g = host(p.execute(dev(c)))
    info = p.info()
    p.close()
    idx = np.random.default_rng(470).choice(w.size, 512, replace=False)
    g1 = direct.dht(0.5, r, c, w[idx])
    print("radial 3-D 1e6: rel l2 %.2e rel max %.2e" % (rel_l2(g[idx], g1), rel_max(g[idx], g1)),
          "(M, z, L)", (info["M"], info["z"], info["L"]), "blocks", info["n_local"], info["n_asy"], info["n_direct"])
    assert rel_l2(g[idx], g1) <= TOL and rel_max(g[idx], g1) <= TOL
