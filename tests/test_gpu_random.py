"""Random transforms against the oracle's direct sum (broad parity sweep).

Forty seeded cases (workloads.random_case): sizes 1 .. 4000, orders -8 .. 20,
tolerances 1e-4 .. 1e-12, uniform / clustered / log-spaced / duplicated /
zero-containing points and frequencies.  Bars: relative l2 <= 2 max(eps,
2e-14) and every entry within 2 eps |c|_1 of the direct sum (the method's
entrywise bound is eps |c|_1; the factor 2 covers the rounding of the
direct sum's own terms at loose tolerances and of the FP64 floor at tight
ones).  Where the plan spreads items on the matrix cores, the vector-unit
spreading of the same plan must agree to 5e-15.
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


@pytest.mark.parametrize("seed", range(40))
def test_random_case(nuht, seed):
    nu, eps, r, w, c, kind = workloads.random_case(seed)
    p = nuht.Plan(dev(r), dev(w), nu, eps)
    g = host(p.execute(dev(c)))
    info = p.info()
    p.close()
    g1 = direct.dht(nu, r, c, w)
    nrm = np.linalg.norm(g1)
    err = np.abs(g - g1)
    rel = np.linalg.norm(g - g1) / nrm if nrm > 0 else np.linalg.norm(g - g1)
    print(seed, kind, "n", r.size, "m", w.size, "nu", nu, "eps", eps, "rel_l2", rel,
          "max/|c|_1", err.max() / np.sum(np.abs(c)), "dense", info["dense_items"], "/", info["spread_items"])
    assert rel <= 2.0 * max(eps, 2e-14)
    assert np.all(err <= 2.0 * eps * np.sum(np.abs(c)))
    if info["dense_items"] > 0:
        q = nuht.Plan(dev(r), dev(w), nu, eps, vector_spread=True)
        gv = host(q.execute(dev(c)))
        q.close()
        scale = max(np.max(np.abs(gv)), 1e-300)
        assert np.max(np.abs(g - gv)) <= 5e-15 * scale
