"""GPU: the plan's sort of the points and frequencies (nuht_plan_order).

Bar: bit-exact.  The sorted values equal numpy's sort (with -0.0 read as
+0.0) and the permutations equal numpy's stable argsort, on all three sort
paths (one workgroup per segment when both hold at most 4096 keys, the
splitter sort up to 2^18 -- 64 bucket slots up to 65536 keys, 1024 above --
and the LSD radix sort beyond), at ragged sizes around
the tile and bucket sizes, with duplicates, signed zeros, presorted and
reversed inputs, clustered inputs, values spread over hundreds of binades,
and inputs built against the sampler so that one bucket overflows the LDS
and takes the global-memory path.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

SMALL_MAX = 4096
SS64_MAX = 1 << 16
SS_MAX = 1 << 18


@pytest.fixture(scope="module")
def nuht():
    import paper_2411_09583_amd as lib
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib.load_library()
    return lib


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


def check_order(nuht, r, w, label):
    print(label, r.size, w.size, flush=True)
    p = nuht.Plan(dev(r), dev(w), 0, 1e-8)
    rs, pr, ws, pw = (t.cpu().numpy() for t in p.order())
    p.close()
    for x, xs, px, name in ((r, rs, pr, "r"), (w, ws, pw, "omega")):
        xp = np.where(x == 0.0, 0.0, x)           # -0.0 sorts (and is stored) as +0.0
        ref = np.argsort(xp, kind="stable")
        assert np.array_equal(px, ref), f"{label}: permutation of {name}"
        assert np.array_equal(xs.view(np.uint64), xp[ref].view(np.uint64)), f"{label}: sorted {name}"


def check_each_side(nuht, x, label):
    # x as the points and as the frequencies, against a few zeros on the other
    # side (every product is 0, so any spread of values plans as local blocks)
    zeros = np.zeros(5)
    check_order(nuht, x, zeros, label + " (points)")
    check_order(nuht, zeros, x, label + " (frequencies)")


@pytest.mark.parametrize("n,m", [(1, 1), (5, 3), (0, 300), (2047, 2048), (SMALL_MAX, SMALL_MAX), (SMALL_MAX + 1, 9),
                                 (8191, 8193), (30000, 60001), (SS64_MAX, SS64_MAX), (SS64_MAX + 1, 3000),
                                 (5000, SS64_MAX + 7), (250_000, 170_001), (SS_MAX, 1000), (1_000_000, 1_000_000),
                                 (SS_MAX + 1, 3000), (5000, SS_MAX + 7)])
def test_sort_uniform(nuht, n, m):
    rng = np.random.default_rng(n + 7 * m)
    check_order(nuht, rng.uniform(0.0, 1.0, n), rng.uniform(0.0, 1e5, m), "uniform")


@pytest.mark.parametrize("n", [3000, 50_000, 200_000, 300_000])
def test_sort_duplicates_and_zeros(nuht, n):
    rng = np.random.default_rng(3 + n)
    r = rng.choice(np.array([0.0, -0.0, 0.25, 0.5, 0.75, 1.0]), n)
    r[rng.choice(n, n // 3, replace=False)] = rng.uniform(0.0, 1.0, n // 3)
    w = np.repeat(rng.uniform(0.0, 100.0, max(1, n // 250)), 250)
    rng.shuffle(w)
    check_order(nuht, r, w, "duplicates")
    check_order(nuht, np.zeros(n), np.full(n // 7, 3.0), "all equal")


@pytest.mark.parametrize("n", [4000, 60_000, 200_000, 1_100_000])
def test_sort_presorted_reversed_clustered(nuht, n):
    k = np.arange(n)
    cheb = 0.5 * (1.0 - np.cos(np.pi * (k + 0.5) / n))          # clustered at both ends
    check_order(nuht, np.sort(cheb), np.sort(cheb)[::-1] * 1e4, "presorted / reversed")
    rng = np.random.default_rng(5 + n)
    check_each_side(nuht, rng.permutation(cheb), "clustered")
    check_each_side(nuht, 10.0 ** rng.uniform(-300, 300, n), "binades")


def sampler_positions(n):
    # the splitter sort's sample of an n-key segment (one hashed point per stratum)
    B = -(-n // 2048)
    ns = min(n, 32 * B)
    s = np.arange(ns, dtype=np.uint64)
    h = (s * np.uint64(0x9E3779B9)) & np.uint64(0xFFFFFFFF)
    for sh, mul in ((16, 0x85EBCA6B), (13, 0xC2B2AE35)):
        h ^= h >> np.uint64(sh)
        h = (h * np.uint64(mul)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    lo = (s.astype(np.int64) * n) // ns
    hi = ((s.astype(np.int64) + 1) * n) // ns
    return lo + ((h * (hi - lo).astype(np.uint64)) >> np.uint64(32)).astype(np.int64)


def test_sort_bucket_overflow(nuht):
    # The sampled points take only the values 0.25 and 0.75 (so the splitters
    # are those two, with equality buckets), every other point is crowded into
    # a narrow interval at 0.5: the range bucket between the splitters then
    # holds all of them, beyond the LDS.  A crowd of width 1e-9 differs in 24
    # low bits of the key (3 passes), one of width 1e-12 in 14 (2 passes, so
    # the result is copied back).
    rng = np.random.default_rng(11)
    for n, width, label in ((60_000, 1e-9, "odd pass count"), (50_000, 1e-12, "even pass count"),
                            (200_000, 1e-9, "1024 bucket slots")):
        x = 0.5 + width * rng.uniform(0.0, 1.0, n)
        pos = sampler_positions(n)
        assert np.unique(pos).size == pos.size and pos.max() < n
        x[pos] = rng.choice(np.array([0.25, 0.75]), pos.size)
        check_each_side(nuht, x, "overflow, " + label)
