"""nuht_gradient_noalloc against nuht_gradient, through the C ABI.

The entry point allocates nothing: its temporaries live in the library's
per-device array and it only runs partitions the plan already holds.  Bar:
the same kernels run in the same order on the same inputs, so its outputs
must equal nuht_gradient's bit for bit, on two calls in a row (the second on
a smaller transform, reusing the array), and it must refuse, without
enqueueing anything, a plan whose partitions are not built yet and a
transform too large for the array.
"""
import numpy as np
import pytest
import torch

import workloads

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
    return None if t is None else t.detach().cpu().numpy()


def prepared(nuht, n, m, nu, seed):
    r, w, c = workloads.uniform(n, m, 1.0, 1500.0, seed=seed)
    gbar = np.random.default_rng(seed + 1).standard_normal(m)
    p = nuht.Plan(dev(r), dev(w), nu, 1e-12)
    ref = [host(t) for t in p.gradient(dev(c), dev(gbar))]     # builds the partitions of nu, nu -+ 1
    return p, dev(c), dev(gbar), ref


def test_noalloc_equals_gradient_two_calls(nuht):
    pa, ca, ga, ref_a = prepared(nuht, 3000, 2500, 5, seed=700)
    pb, cb, gb, ref_b = prepared(nuht, 1200, 900, -2, seed=710)   # smaller, and a negative order
    print("calls: noalloc on n=3000 m=2500 nu=5, then n=1200 m=900 nu=-2", flush=True)
    out_a = [host(t) for t in pa.gradient_noalloc(ca, ga)]
    out_b = [host(t) for t in pb.gradient_noalloc(cb, gb)]
    for got, ref in ((out_a, ref_a), (out_b, ref_b)):
        for g, e, name in zip(got, ref, ("dc", "dr", "domega")):
            assert g.shape == e.shape, name
            assert np.array_equal(g, e), (name, np.max(np.abs(g - e)))
    # the larger call once more after the smaller one: nothing left over counts
    again = [host(t) for t in pa.gradient_noalloc(ca, ga)]
    for g, e in zip(again, ref_a):
        assert np.array_equal(g, e)
    # only some outputs
    dc, dr, dw = pb.gradient_noalloc(cb, gb, want_c=False, want_r=False)
    assert dc is None and dr is None and np.array_equal(host(dw), ref_b[2])
    pa.close()
    pb.close()


def test_noalloc_refuses_unbuilt_partitions(nuht):
    r, w, c = workloads.uniform(800, 700, 1.0, 900.0, seed=720)
    y = np.random.default_rng(721).standard_normal(700)
    p = nuht.Plan(dev(r), dev(w), 3, 1e-12)
    with pytest.raises(nuht.NuhtError) as e:
        p.gradient_noalloc(dev(c), dev(y))
    assert e.value.code == -7
    p.adjoint(dev(y))                                   # builds the transposed partition of order 3 only
    dc, _, _ = p.gradient_noalloc(dev(c), dev(y), want_r=False, want_omega=False)
    ref, _, _ = p.gradient(dev(c), dev(y), want_r=False, want_omega=False)
    assert np.array_equal(host(dc), host(ref))
    with pytest.raises(nuht.NuhtError) as e:            # orders 2 and 4 are still missing
        p.gradient_noalloc(dev(c), dev(y), want_c=False)
    assert e.value.code == -7
    p.close()


def test_noalloc_refuses_transforms_above_the_array(nuht):
    # 2 (n + m) doubles must fit the 8 388 608 of the array
    n = m = 2_200_000
    r, w, c = workloads.uniform(n, m, 1.0, 50.0, seed=730)
    p = nuht.Plan(dev(r), dev(w), 0, 1e-6)
    y = dev(np.ones(m))
    with pytest.raises(nuht.NuhtError) as e:
        p.gradient_noalloc(dev(c), y, want_c=False)
    assert e.value.code == -6
    p.close()
