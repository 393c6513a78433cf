"""Batched transforms (one graph) and the autotuner, on the GPU.

* a batch of uneven transforms (orders 0..63, negative and zero sizes
  included) gives exactly the outputs of the same plans executed one by one;
* each transform agrees with the method-exact reference on sampled outputs
  (rel-l2 <= 2e-13: the GPU path's own error) and with the direct sum within
  the entrywise bound eps |c|_1, and, for |nu| <= 10, within 1e-12 in rel-l2
  (at higher orders the paper's parameters leave the method's own truncation
  at ~1e-12 against the direct sum);
* the captured graph is replayed several times with other GPU work and
  synchronisations in between, with fresh input/output buffers, and every
  replay matches the eager result;
* tuned batches and tuned plans stay correct.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import direct, method

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


def small_batch():
    # uneven sizes and orders; sizes kept small so the oracle checks are quick
    tr = workloads.batch(count=14, seed=5, lo=2.0, hi=4.0, nu_max=63)
    tr.append(dict(nu=-3, r=np.random.default_rng(1).uniform(0, 1, 700),
                   w=np.random.default_rng(2).uniform(0, 700, 650), c=np.random.default_rng(3).standard_normal(700)))
    tr.append(dict(nu=2, r=np.zeros(0), w=np.random.default_rng(4).uniform(0, 10, 50), c=np.zeros(0)))   # n = 0
    tr.append(dict(nu=1, r=np.random.default_rng(5).uniform(0, 1, 40), w=np.zeros(0),
                   c=np.random.default_rng(6).standard_normal(40)))                                     # m = 0
    return tr


def test_batch_equals_individual_and_oracle(nuht):
    tr = small_batch()
    b = nuht.Batch([dev(t["r"]) for t in tr], [dev(t["w"]) for t in tr], [t["nu"] for t in tr], 1e-12)
    gs = [host(g) for g in b.execute([dev(t["c"]) for t in tr])]
    b.close()
    rng = np.random.default_rng(11)
    for t, g in zip(tr, gs):
        p = nuht.Plan(dev(t["r"]), dev(t["w"]), t["nu"], 1e-12)
        g1 = host(p.execute(dev(t["c"])))
        p.close()
        assert np.array_equal(g, g1), t["nu"]
        if t["w"].size == 0:
            continue
        if t["r"].size == 0:
            assert np.all(g == 0.0)
            continue
        idx = rng.choice(t["w"].size, min(64, t["w"].size), replace=False)
        ref = direct.dht(t["nu"], t["r"], t["c"], t["w"][idx])
        ref2 = method.nufht_reference_rows(t["nu"], 1e-12, t["r"], t["c"], t["w"], idx)
        err2 = np.linalg.norm(g[idx] - ref2) / np.linalg.norm(ref2)
        assert err2 <= 2e-13, (t["nu"], t["r"].size, err2)
        err = np.linalg.norm(g[idx] - ref) / np.linalg.norm(ref)
        if abs(t["nu"]) <= 10:
            assert err <= TOL, (t["nu"], t["r"].size, err)
        assert np.max(np.abs(g[idx] - ref)) <= 1e-12 * np.sum(np.abs(t["c"]))


def test_graph_replays_with_work_in_between(nuht):
    tr = small_batch()[:10]
    b = nuht.Batch([dev(t["r"]) for t in tr], [dev(t["w"]) for t in tr], [t["nu"] for t in tr], 1e-12)
    eager = []
    for t in tr:
        p = nuht.Plan(dev(t["r"]), dev(t["w"]), t["nu"], 1e-12)
        eager.append(host(p.execute(dev(t["c"]))))
        p.close()
    x = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(4):
        cs = [dev(t["c"]) for t in tr]                  # fresh input buffers each time
        gs = b.execute(cs)
        y = torch.sum(x * x)                            # other work between replays
        if rep % 2:
            torch.cuda.synchronize()
        for g, e in zip(gs, eager):
            assert np.array_equal(host(g), e), rep
        assert float(y) > 0
    b.close()


def test_empty_batch(nuht):
    b = nuht.Batch([], [], [], 1e-12)
    assert b.execute([]) == []
    b.close()


def test_tuned_batch_and_plan(nuht):
    tr = workloads.batch(count=6, seed=12, lo=3.0, hi=4.3, nu_max=20)
    b = nuht.Batch([dev(t["r"]) for t in tr], [dev(t["w"]) for t in tr], [t["nu"] for t in tr], 1e-12, tune=True)
    gs = [host(g) for g in b.execute([dev(t["c"]) for t in tr])]
    infos = [b.info(i) for i in range(len(tr))]
    b.close()
    rng = np.random.default_rng(13)
    for t, g, inf in zip(tr, gs, infos):
        assert inf["spread_chunk"] in (512, 1024, 2048, 4096)
        idx = rng.choice(t["w"].size, min(48, t["w"].size), replace=False)
        ref = direct.dht(t["nu"], t["r"], t["c"], t["w"][idx])
        # the method-exact reference with the options the tuner chose
        ref2 = method.nufht_reference_rows(t["nu"], 1e-12, t["r"], t["c"], t["w"], idx, min_size=inf["min_size"])
        assert np.linalg.norm(g[idx] - ref2) / np.linalg.norm(ref2) <= 2e-13
        if abs(t["nu"]) <= 10:
            assert np.linalg.norm(g[idx] - ref) / np.linalg.norm(ref) <= TOL
        assert np.max(np.abs(g[idx] - ref)) <= 1e-12 * np.sum(np.abs(t["c"]))
    r, w, c = workloads.uniform(20000, 20000, 1.0, 2e4, seed=14)
    p = nuht.Plan(dev(r), dev(w), 4, 1e-12)
    best = p.tune(dev(c))
    assert best["spread_chunk"] in (512, 1024, 2048, 4096) and best["ms"] > 0
    assert p.info()["min_size"] == best["min_size"]
    g = host(p.execute(dev(c)))
    p.close()
    idx = rng.choice(w.size, 64, replace=False)
    ref = direct.dht(4, r, c, w[idx])
    assert np.linalg.norm(g[idx] - ref) / np.linalg.norm(ref) <= TOL
