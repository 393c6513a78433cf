"""GPU: an execution forked over two streams equals the same execution on one.

nuht_execute runs the local moments and direct blocks on the library's side
stream, beside the spreading, grid assembly and FFT, and rejoins the caller's
stream before the local rows.  Profiling the local-moment stage keeps every
stage on the caller's stream.  Both orders run the same kernels on the same
data, and each kernel's sums have a fixed order, so the outputs must agree
bit for bit; repeated forked executions (the second reusing the plan's fork
events while the first may still run) must too, and so must the gradient,
whose transforms fork the same way.  Sizes span many blocks of every kind
(local, asymptotic, direct) at three orders.
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


@pytest.mark.parametrize("nu", [0, 1, 10])
def test_forked_equals_serial(nuht, nu):
    print("fork", nu, flush=True)
    r, w, c = workloads.large_uniform(seed=70 + nu, n=200_000, m=150_000)
    r, w, c = (torch.as_tensor(a, device="cuda") for a in (r, w, c))
    p = nuht.Plan(r, w, nu, 1e-12)
    info = p.info()
    assert info["n_local"] > 0 and info["n_asy"] > 0 and info["n_direct"] > 0
    g_fork = p.execute(c)
    g_again = torch.empty_like(g_fork)
    for _ in range(3):
        p.execute(c, out=g_again)
    p.profile(True, stages=["local_moments"])
    g_serial = p.execute(c)
    p.profile(False)
    torch.cuda.synchronize()
    p.close()
    assert torch.equal(g_fork, g_serial)
    assert torch.equal(g_again, g_serial)


def test_forked_streams_keep_order(nuht):
    # two plans executed back to back on one stream share the side stream; a
    # second stream running another plan meanwhile must not disturb either
    print("fork order", flush=True)
    r, w, c = workloads.large_uniform(seed=81, n=120_000, m=120_000)
    r, w, c = (torch.as_tensor(a, device="cuda") for a in (r, w, c))
    pa = nuht.Plan(r, w, 0, 1e-12)
    pb = nuht.Plan(r, w, 3, 1e-10)
    ref_a, ref_b = pa.execute(c), pb.execute(c)
    torch.cuda.synchronize()
    other = torch.cuda.Stream()
    outs_a, outs_b = [], []
    for k in range(4):
        ck = c * (k + 1)
        outs_a.append(pa.execute(ck))
        with torch.cuda.stream(other):
            outs_b.append(pb.execute(ck))
    torch.cuda.synchronize()
    for k in range(4):
        scale = float(k + 1)
        assert torch.allclose(outs_a[k], ref_a * scale, rtol=1e-14, atol=1e-300 + 1e-14 * float(ref_a.abs().max()))
        assert torch.allclose(outs_b[k], ref_b * scale, rtol=1e-14, atol=1e-300 + 1e-14 * float(ref_b.abs().max()))
    pa.close()
    pb.close()
