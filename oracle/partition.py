"""Matrix subdivision into local, asymptotic and direct blocks (Sec. 4.1).

TEST INFRASTRUCTURE ONLY (see :mod:`oracle`).

With r and w sorted ascending, entry (j, k) of A(j,k) = J_nu(w_j r_k) is *local*
when w_j r_k <= z and *asymptotic* otherwise.  Alg. 1 (Subdivide) keeps a set
of mixed blocks, splits each at an index pair (j, k) on the curve w r = z
into four, sends the upper-left part to the local set, the lower-right part to
the asymptotic set and the two off-diagonal parts back to the mixed set, or to
the direct set when their area is at most min_size.

Readings of the paper taken here (each listed in the design doc):
* SplitIndices takes rows j as the candidates that index w, columns k the ones
  that index r (Alg. 1 prints the two lists swapped).
* The split minimises the mixed area (j-j0+1)(k1-k) + (j1-j)(k-k0+1) -- the text
  says the objective is minimised and that the fast area is to be maximised;
  the argmax in the display is read as that.  Ties go to the smaller j.
* The quasi-optimal solve uses 16 equispaced candidate rows including both
  ends (floor of linspace(j0, jl, 16)), jl being the block's last row with a
  local entry; for each, k is the largest column in the block with
  w_j r_k <= z, or k0-1 when there is none.  Restricting the candidates to
  rows that can hold a split point keeps the depth logarithmic when the local
  region is a thin strip along the block's top (many equal points).
* The lower-left child (j+1:j1, k0:k) is tested by its own area (j1-j)(k-k0+1);
  the printed (j1-j)(k1-k+1) is read as a typo.  Both off-diagonal children go
  to the direct set when their area is <= min_size.
* A mixed block that is wholly local (w_{j1} r_{k1} <= z) or wholly asymptotic
  (w_{j0} r_{k0} > z) is sent whole to that set before any split; empty
  children are dropped.
* Products w_j r_k are compared with z exactly (not after rounding).
"""
from dataclasses import dataclass
from typing import List

import numpy as np


@dataclass(frozen=True)
class Block:
    """Index rectangle rows j0..j1 (frequencies), columns k0..k1 (points),
    inclusive, in sorted order; level 1 is the whole matrix."""
    kind: str   # 'L', 'A' or 'D'
    j0: int
    j1: int
    k0: int
    k1: int
    level: int

    @property
    def rows(self) -> int:
        return self.j1 - self.j0 + 1

    @property
    def cols(self) -> int:
        return self.k1 - self.k0 + 1


def split_indices(K, j0: int, j1: int, k0: int, k1: int, ncand: int = 16):
    """Quasi-optimal SplitIndices (Sec. 4.1).  K[j] = #{k : w_j r_k <= z}.

    The candidate rows are equispaced over j0 .. jl, jl being the last row of
    the block that holds a local entry (K is nonincreasing in j, so jl is found
    by bisection); rows below jl cannot hold the split point.  ncand = 0 takes
    every row j0 .. jl: the exact optimum of the objective (Sec. 4.1 notes an
    O(j1 - j0 + k1 - k0) exact solve)."""
    lo, hi = j0, j1
    while lo < hi:
        mid = lo + (hi - lo + 1) // 2
        if K[mid] > k0:
            lo = mid
        else:
            hi = mid - 1
    jl = lo
    best = None
    if jl > j0 and ncand == 0:
        cands = range(j0, jl + 1)
    elif jl > j0:
        cands = [j0 + (c * (jl - j0)) // (ncand - 1) for c in range(ncand)]
    else:
        cands = [j0]
    for j in cands:
        k = min(int(K[j]) - 1, k1)
        if k < k0:
            k = k0 - 1
        mixed_area = (j - j0 + 1) * (k1 - k) + (j1 - j) * (k - k0 + 1)
        if best is None or mixed_area < best[0]:
            best = (mixed_area, j, k)
    return best[1], best[2]


def subdivide(K, m: int, n: int, min_size: int = 1024, ncand: int = 16) -> List[Block]:
    """Alg. 1 over the staircase K (length m, sorted frequencies)."""
    out: List[Block] = []
    if m == 0 or n == 0:
        return out
    mixed = [(0, m - 1, 0, n - 1, 1)]
    while mixed:
        j0, j1, k0, k1, lev = mixed.pop()
        if K[j1] >= k1 + 1:                 # w_{j1} r_{k1} <= z: wholly local
            out.append(Block('L', j0, j1, k0, k1, lev))
            continue
        if K[j0] <= k0:                     # w_{j0} r_{k0} > z: wholly asymptotic
            out.append(Block('A', j0, j1, k0, k1, lev))
            continue
        j, k = split_indices(K, j0, j1, k0, k1, ncand)
        if k >= k0:
            out.append(Block('L', j0, j, k0, k, lev))
        if j < j1 and k < k1:
            out.append(Block('A', j + 1, j1, k + 1, k1, lev))
        if k < k1:                          # upper right (j0:j, k+1:k1)
            if (j - j0 + 1) * (k1 - k) > min_size:
                mixed.append((j0, j, k + 1, k1, lev + 1))
            else:
                out.append(Block('D', j0, j, k + 1, k1, lev))
        if j < j1 and k >= k0:              # lower left (j+1:j1, k0:k)
            if (j1 - j) * (k - k0 + 1) > min_size:
                mixed.append((j + 1, j1, k0, k, lev + 1))
            else:
                out.append(Block('D', j + 1, j1, k0, k, lev))
    return out


def stats(blocks: List[Block]) -> dict:
    """Counts and memberships per block class."""
    d = {}
    for kind in 'LAD':
        bs = [b for b in blocks if b.kind == kind]
        d[kind] = dict(count=len(bs),
                       area=int(sum(b.rows * b.cols for b in bs)),
                       row_members=int(sum(b.rows for b in bs)),
                       col_members=int(sum(b.cols for b in bs)))
    d['levels'] = max((b.level for b in blocks), default=0)
    return d


def coverage(blocks: List[Block], m: int, n: int) -> np.ndarray:
    """How many blocks cover each entry (brute force, small sizes only)."""
    cov = np.zeros((m, n), dtype=np.int32)
    for b in blocks:
        cov[b.j0:b.j1 + 1, b.k0:b.k1 + 1] += 1
    return cov
