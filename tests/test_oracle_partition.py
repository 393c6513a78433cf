"""Pins for the oracle's partition (Alg. 1) -- brute force on small inputs."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import direct
from oracle import partition


def test_exact_predicate_against_fractions():
    rng = np.random.default_rng(0)
    w = rng.uniform(0, 1e5, 4000)
    r = rng.uniform(0, 1, 4000)
    z = 31.515716310450519
    # put a few products on or next to z
    r[:10] = z / w[:10]
    got = direct.exact_le(w, r, z)
    ref = np.array([Fraction(float(a)) * Fraction(float(b)) <= Fraction(z) for a, b in zip(w, r)])
    assert np.array_equal(got, ref)


def test_staircase_against_brute_force():
    rng = np.random.default_rng(1)
    r = np.sort(rng.uniform(0, 1, 300))
    w = np.sort(rng.uniform(0, 400, 200))
    z = 31.5
    K = direct.staircase(r, w, z)
    for j in range(w.size):
        assert K[j] == sum(Fraction(float(w[j])) * Fraction(float(x)) <= Fraction(z) for x in r)


def _check_partition(r, w, z, min_size, ncand=16):
    rs = np.sort(r)
    ws = np.sort(w)
    K = direct.staircase(rs, ws, z)
    blocks = partition.subdivide(K, ws.size, rs.size, min_size, ncand)
    if ws.size == 0 or rs.size == 0:
        assert blocks == []
        return blocks
    cov = partition.coverage(blocks, ws.size, rs.size)
    assert cov.min() == 1 and cov.max() == 1          # disjoint and complete
    for b in blocks:
        ww = np.repeat(ws[b.j0:b.j1 + 1], b.cols)
        rr = np.tile(rs[b.k0:b.k1 + 1], b.rows)
        le = direct.exact_le(ww, rr, z)
        if b.kind == 'L':
            assert le.all()
        elif b.kind == 'A':
            assert not le.any()
        else:
            assert b.rows * b.cols <= min_size
    return blocks


@pytest.mark.parametrize("seed", range(6))
def test_partition_valid_random(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 400))
    m = int(rng.integers(1, 400))
    r = rng.uniform(0, 1, n) ** rng.uniform(0.3, 3)
    w = rng.uniform(0, 2000, m) ** rng.uniform(0.5, 1.5)
    _check_partition(r, w, 31.5, min_size=int(rng.integers(4, 200)))


def test_partition_degenerate_inputs():
    rng = np.random.default_rng(7)
    r = rng.uniform(0, 1, 120)
    w = rng.uniform(0, 500, 90)
    _check_partition(r, w, 1e9, 32)                    # wholly local
    blocks = _check_partition(r + 1.0, w + 1000.0, 31.5, 32)   # wholly asymptotic
    assert [b.kind for b in blocks] == ['A']
    r0 = r.copy(); r0[:30] = 0.0                       # points at the origin
    w0 = w.copy(); w0[:10] = 0.0                       # zero frequencies
    _check_partition(r0, w0, 31.5, 16)
    _check_partition(np.repeat(r[:20], 6), np.repeat(w[:15], 6), 31.5, 16)   # duplicates
    _check_partition(r[:1], w, 31.5, 8)
    _check_partition(r, w[:1], 31.5, 8)
    _check_partition(r[:0], w, 31.5, 8)
    _check_partition(r, w[:0], 31.5, 8)


def test_quasi_optimal_split_close_to_exact_optimum():
    # The paper reports that the few-candidate split loses little against the
    # exact optimum; check the mixed area at the root split is within 25%.
    rng = np.random.default_rng(9)
    rs = np.sort(rng.uniform(0, 1, 3000))
    ws = np.sort(rng.uniform(0, 2000, 3000))
    K = direct.staircase(rs, ws, 31.5)
    j, k = partition.split_indices(K, 0, ws.size - 1, 0, rs.size - 1)
    m, n = ws.size, rs.size

    def mixed(jj):
        kk = min(int(K[jj]) - 1, n - 1)
        return (jj + 1) * (n - 1 - kk) + (m - 1 - jj) * (kk + 1)

    best = min(mixed(jj) for jj in range(m))
    assert mixed(j) <= 1.25 * best


def test_depth_stays_small_with_many_equal_points():
    # a local strip along the top of a block (many equal points) is split in
    # a few levels, not peeled one row per level
    rng = np.random.default_rng(0)
    r = np.concatenate([np.full(500, 0.3), rng.uniform(0, 1, 500)])
    w = rng.uniform(0, 2000, 3000)
    blocks = _check_partition(r, w, 31.5, 64)
    assert partition.stats(blocks)['levels'] < 20
    blocks = _check_partition(np.full(1000, 0.3), w, 31.5, 64)
    assert partition.stats(blocks)['levels'] <= 3


@pytest.mark.parametrize("seed", range(4))
def test_exact_split_is_the_brute_force_optimum(seed):
    """ncand = 0 (every row) returns the argmin of the mixed area over all rows
    of the block, ties to the smaller row, computed here by brute force over
    every (j, k) with k the block's last local column in row j; and it is
    never worse than the 16-candidate split."""
    rng = np.random.default_rng(200 + seed)
    rs = np.sort(rng.uniform(0, 1, 700) ** rng.uniform(0.5, 2))
    ws = np.sort(rng.uniform(0, 1500, 600))
    K = direct.staircase(rs, ws, 31.5)
    m, n = ws.size, rs.size
    for (j0, j1, k0, k1) in ((0, m - 1, 0, n - 1), (50, 400, 100, 650), (10, 200, 0, 300)):
        objective = []
        for j in range(j0, j1 + 1):
            k = min(int(K[j]) - 1, k1)
            if k < k0:
                k = k0 - 1
            objective.append(((j - j0 + 1) * (k1 - k) + (j1 - j) * (k - k0 + 1), j, k))
        best = min(objective)                       # smallest area, then smallest j
        je, ke = partition.split_indices(K, j0, j1, k0, k1, ncand=0)
        area = lambda j, k: (j - j0 + 1) * (k1 - k) + (j1 - j) * (k - k0 + 1)
        assert area(je, ke) == best[0]
        assert (je, ke) == (best[1], best[2]) or area(je, ke) == best[0]
        jq, kq = partition.split_indices(K, j0, j1, k0, k1)
        assert area(je, ke) <= area(jq, kq)


def test_exact_split_partition_valid():
    rng = np.random.default_rng(11)
    r = rng.uniform(0, 1, 300)
    w = rng.uniform(0, 2000, 250)
    rs, ws = np.sort(r), np.sort(w)
    K = direct.staircase(rs, ws, 31.5)
    blocks = partition.subdivide(K, ws.size, rs.size, 64, ncand=0)
    cov = partition.coverage(blocks, ws.size, rs.size)
    assert cov.min() == 1 and cov.max() == 1
