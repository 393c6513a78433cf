"""Spreading on the matrix cores (dense items) against the vector-unit
spreading of the same plan, and both against the oracle's direct sum.

Workload: n = 30000 points r ~ U[0, 1), m = 2000 frequencies omega ~ U[0, 2000)
(seeded).  Its asymptotic blocks hold about a thousand points each on grids of
the minimum size, so most spreading items are dense (their points reach the
grid from a few first cells).  Cases cover the kernel instances: 4, 6, 8, 12,
14 and 16 channels (one and two column tiles; orders 0, 10, 16, 20 and
tolerances 1e-6 .. 1e-12), 20, 24, 28 and 32 (three and four tiles; orders
30 .. 60), ES width 16 (eps = 1e-13, every tile row a tap), and two
ineligible plans (width 17 at eps = 1e-14, 36 channels at order 70) that must
report no dense items.

Per case:
* the plan reports dense items (none with vector_spread, none when ineligible);
* the two spreadings give the same transform up to summation order: relative
  l2 and max differences below 5e-15 up to 16 channels (each cell sums about a
  thousand terms in a different order; rounding moves a sum by ~1e-16 of its
  terms' magnitude, and the differences seen are up to 6e-16).  From 20
  channels (orders 30 and up) the channel sums of the Hankel terms grow well
  above the result near the crossover before they decay, and the rounding of
  the two orders grows with them (1.0e-14 rel-l2, 2.4e-14 max at order 60):
  there the bar is a twentieth of the vector path's own error against the
  direct sum (8.4e-13 at order 60), i.e. the paths agree far below the
  method's truncation;
* the transform meets the oracle's bars: relative l2 <= max(eps, 2e-14) against
  the direct sum, and for eps = 1e-12 every entry within eps |c|_1.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import direct

pytestmark = pytest.mark.gpu

CASES = [  # nu, eps, expected channels (2M padded), dense expected
    (0, 1e-12, 8, True),
    (0, 1e-9, 6, True),
    (0, 1e-6, 4, True),
    (10, 1e-12, 12, True),
    (16, 1e-12, 14, True),
    (20, 1e-12, 16, True),
    (30, 1e-12, 20, True),
    (40, 1e-12, 24, True),
    (50, 1e-12, 28, True),
    (60, 1e-12, 32, True),
    (0, 1e-13, 8, True),     # ES width 16
    (0, 1e-14, 8, False),    # ES width 17: vector units only
    (70, 1e-12, 36, False),  # 36 channels: vector units only
]


@pytest.fixture(scope="module")
def nuht():
    import paper_2411_09583_amd as lib
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib.load_library()
    return lib


@pytest.fixture(scope="module")
def data():
    r, w, c = workloads.uniform(30000, 2000, 1.0, 2000.0, seed=120)
    return r, w, c, {}


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def rel_max(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("nu,eps,nch,dense", CASES)
def test_dense_spreading(nuht, data, nu, eps, nch, dense):
    r, w, c, cache = data
    rd, wd, cd = dev(r), dev(w), dev(c)
    p = nuht.Plan(rd, wd, nu, eps)
    g = host(p.execute(cd))
    info = p.info()
    p.close()
    q = nuht.Plan(rd, wd, nu, eps, vector_spread=True)
    gv = host(q.execute(cd))
    info_v = q.info()
    q.close()
    print(nu, eps, "M", info["M"], "w", info["es_width"], "items", info["spread_items"], "dense", info["dense_items"])
    assert 2 * info["M"] <= nch and info["spread_items"] > 0
    assert info_v["dense_items"] == 0
    if dense:
        assert info["dense_items"] > info["spread_items"] // 2
    else:
        assert info["dense_items"] == 0
    d_l2, d_max = rel_l2(g, gv), rel_max(g, gv)
    if nu not in cache:
        cache[nu] = direct.dht(nu, r, c, w)
    g1 = cache[nu]
    print("  matrix vs vector spreading", d_l2, d_max, "vector vs direct sum", rel_l2(gv, g1), rel_max(gv, g1),
          "matrix vs direct sum", rel_l2(g, g1), rel_max(g, g1))
    if nch <= 16:
        assert d_l2 <= 5e-15 and d_max <= 5e-15
    else:
        assert d_l2 <= max(5e-15, rel_l2(gv, g1) / 20) and d_max <= max(5e-15, rel_max(gv, g1) / 20)
    assert rel_l2(g, g1) <= max(eps, 2e-14)
    if eps == 1e-12:
        assert np.max(np.abs(g - g1)) <= eps * np.sum(np.abs(c))
