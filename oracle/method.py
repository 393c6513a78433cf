"""O2: the method-exact reference (Alg. 2 with expansions summed directly).

TEST INFRASTRUCTURE ONLY (see :mod:`oracle`).

Alg. 2 chooses (M, z, L), subdivides the matrix (Alg. 1) and applies each block
by its expansion.  Here every block is applied by *summing its expansion
directly*, entry by entry, with no NUFFT:

* local block (rows j0..j1, columns k0..k1), R = r_{k1}: the Wimp expansion
  (Sec. 3.1) as the rank-(L+1) product C T^T of Sec. 3.1,
      g_j += sum_{l=0}^{L} C_l(w_j R) sum_k c_k T_{2l}(r_k / R)          (nu even)
      C_l(x) = delta_l J_{nu/2+l}(x/2) J_{nu/2-l}(x/2),  delta_0 = 1, else 2,
  and for odd nu the odd-order form
      g_j += sum_{l=0}^{L} C_l(w_j R) sum_k c_k T_{2l+1}(r_k / R),
      C_l(x) = 2 J_{(nu+1)/2+l}(x/2) J_{(nu-1)/2-l}(x/2);
* asymptotic block: the M-term Hankel formula of eq. asy-error summed entry by
  entry (``direct.asy_block_apply``);
* direct block: J_nu itself (``direct.dht``).

Half-integer orders nu = n + 1/2 take their parameters from
``params.half_parameters`` and local blocks from ``half_local_block_apply``
(J_{n+1/2}(x y) = sqrt(y) sqrt(2x/pi) j_n(x y), j_n's Chebyshev series in y).

The difference O2 - O1 is therefore pure truncation error of the expansions,
bounded entrywise by eps, so |O2_j - O1_j| <= eps * sum_k |c_k|.

Readings taken here (each listed in the design doc): the Wimp coefficient's argument
is x/2 (the printed C_l(x) has argument x, but the proof of Lemma 3.1 and
Neumann's addition theorem at y = 1 fix x/2); the odd-order expansion is the
one above; when a local block's largest point is r = 0 the block uses
R = z / w_{j1} (or R = 1 if that frequency is also 0), which keeps every
argument w R within [0, z] where Lemma 3.1 applies.
"""
import numpy as np

from oracle import direct
from oracle import params as prm
from oracle import partition


def chebyshev_t(nmax: int, y: np.ndarray) -> np.ndarray:
    """T_0 .. T_nmax at y by the three-term recurrence T_{k+1} = 2y T_k - T_{k-1}."""
    T = np.empty((nmax + 1, y.size))
    T[0] = 1.0
    if nmax >= 1:
        T[1] = y
    for k in range(1, nmax):
        T[k + 1] = 2.0 * y * T[k] - T[k - 1]
    return T


def wimp_coefficients(nu: int, L: int, x: np.ndarray, x_lo: np.ndarray = None) -> np.ndarray:
    """C_l(x) for l = 0..L at the arguments x (+ x_lo), shape (L+1, len(x));
    nu >= 0.  Even nu: delta_l J_{nu/2+l}(x/2) J_{nu/2-l}(x/2); odd nu:
    2 J_{(nu+1)/2+l}(x/2) J_{(nu-1)/2-l}(x/2)."""
    x = np.asarray(x, dtype=np.float64)
    xl = np.zeros_like(x) if x_lo is None else np.asarray(x_lo, dtype=np.float64)
    half, half_lo = 0.5 * x, 0.5 * xl          # exact halving
    C = np.empty((L + 1, x.size))
    if nu % 2 == 0:
        a = nu // 2
        for l in range(L + 1):
            d = 1.0 if l == 0 else 2.0
            C[l] = d * direct.besselj(a + l, half, half_lo) * direct.besselj(a - l, half, half_lo)
    else:
        a = (nu - 1) // 2
        for l in range(L + 1):
            C[l] = 2.0 * direct.besselj(a + 1 + l, half, half_lo) * direct.besselj(a - l, half, half_lo)
    return C


def spherical_jn(n: int, t: np.ndarray) -> np.ndarray:
    """j_n(t) = sqrt(pi / (2 t)) J_{n+1/2}(t) (DLMF 10.47.3) for real t, with
    the oracle's J, j_n(-t) = (-1)^n j_n(t) and j_n(0) = [n == 0]."""
    t = np.asarray(t, dtype=np.float64)
    a = np.abs(t)
    out = np.where(a > 0, 0.0, 1.0 if n == 0 else 0.0)
    pos = a > 0
    if np.any(pos):
        out[pos] = np.sqrt(np.pi / (2.0 * a[pos])) * direct.besselj(n + 0.5, a[pos])
    return np.where(t < 0, (-1.0) ** n * out, out)


def half_coefficients(n: int, L: int, x: np.ndarray) -> np.ndarray:
    """beta_{e+2l}(x), l = 0..L (e = n mod 2): the Chebyshev coefficients of
    y -> j_n(x y) on [-1, 1], by the discrete Chebyshev transform at Q
    Chebyshev points (Q well above the degrees involved, so the aliased
    coefficients are below the rounding level).  Shape (L+1, len(x))."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    e = n % 2
    kmax = 2 * L + e
    Q = int(kmax + 2 * np.max(x, initial=0.0) + 64)
    odd = 2 * np.arange(Q) + 1                            # theta_q = pi (2q + 1) / (2Q)
    ks = np.arange(e, kmax + 1, 2)
    F = spherical_jn(n, np.outer(x, np.cos(np.pi * odd / (2 * Q))))          # (len(x), Q)
    # cos(k theta_q) with the integer k (2q + 1) reduced modulo 4Q first, so
    # large k do not magnify the rounding of theta_q
    C = np.cos(np.pi * (np.outer(odd, ks) % (4 * Q)) / (2 * Q))             # (Q, L+1)
    beta = (F @ C) * (2.0 / Q)
    beta[:, ks == 0] *= 0.5
    return beta.T


def half_local_block_apply(nu: float, L: int, z: float, w_rows, r_cols, c_cols) -> np.ndarray:
    """One local block at the half-integer order nu = n + 1/2:
        g_j += sqrt(2 x_j / pi) sum_l beta_{e+2l}(x_j) sum_k c_k sqrt(y_k) T_{e+2l}(y_k),
    x_j = w_j R, y_k = r_k / R, from J_{n+1/2}(x y) = sqrt(y) sqrt(2x/pi) j_n(x y)."""
    n = int(round(nu - 0.5))
    w_rows = np.asarray(w_rows, dtype=np.float64)
    r_cols = np.asarray(r_cols, dtype=np.float64)
    c_cols = np.asarray(c_cols, dtype=np.float64)
    R = float(r_cols[-1])
    if R == 0.0:
        wmax = float(w_rows[-1])
        R = z / wmax if wmax > 0.0 else 1.0
    y = r_cols / R
    e = n % 2
    T = chebyshev_t(2 * L + e, y)
    t = T[e::2] @ (c_cols * np.sqrt(y))                   # moments, length L+1
    x = w_rows * R
    B = half_coefficients(n, L, x)                        # (L+1, rows)
    return np.sqrt(2.0 * x / np.pi) * (t @ B)


def local_block_apply(nu: int, L: int, z: float, w_rows, r_cols, c_cols) -> np.ndarray:
    """Rank-(L+1) Wimp product for one local block: C (T^T c)  (Sec. 3.1)."""
    w_rows = np.asarray(w_rows, dtype=np.float64)
    r_cols = np.asarray(r_cols, dtype=np.float64)
    c_cols = np.asarray(c_cols, dtype=np.float64)
    R = float(r_cols[-1])
    if R == 0.0:
        wmax = float(w_rows[-1])
        R = z / wmax if wmax > 0.0 else 1.0
    y = r_cols / R
    odd = nu % 2
    T = chebyshev_t(2 * L + odd, y)
    t = T[odd::2] @ c_cols                         # moments, length L+1
    xh, xl = direct.two_prod(w_rows, np.full_like(w_rows, R))
    C = wimp_coefficients(nu, L, xh, xl)            # (L+1, rows)
    return t @ C


def _order(nu):
    """(sign, order used, local-block routine): negative integer orders through
    J_{-nu} = (-1)^nu J_nu; half-integer orders with their own local form."""
    if prm.is_half(nu):
        return 1.0, float(nu), half_local_block_apply
    nu = int(nu)
    return (-1.0 if (nu < 0 and (-nu) % 2 == 1) else 1.0), abs(nu), local_block_apply


def nufht_reference(nu, eps: float, r, c, w, min_size: int = 1024,
                    ncand: int = 16, M: int = None, return_blocks: bool = False):
    """Alg. 2 with every block's expansion summed directly.  Output follows the
    order of w."""
    r = np.asarray(r, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    sign, anu, local = _order(nu)
    M, z, L = prm.any_parameters(anu, eps, M)
    pr = np.argsort(r, kind='stable')
    pw = np.argsort(w, kind='stable')
    rs, cs, ws = r[pr], c[pr], w[pw]
    K = direct.staircase(rs, ws, z)
    blocks = partition.subdivide(K, ws.size, rs.size, min_size, ncand)
    gs = np.zeros(ws.size)
    for b in blocks:
        rows = slice(b.j0, b.j1 + 1)
        cols = slice(b.k0, b.k1 + 1)
        if b.kind == 'L':
            gs[rows] += local(anu, L, z, ws[rows], rs[cols], cs[cols])
        elif b.kind == 'A':
            gs[rows] += direct.asy_block_apply(anu, M, ws[rows], rs[cols], cs[cols])
        else:
            gs[rows] += direct.dht(anu, rs[cols], cs[cols], ws[rows])
    g = np.empty_like(gs)
    g[pw] = sign * gs
    if return_blocks:
        return g, dict(M=M, z=z, L=L, blocks=blocks)
    return g


def nufht_reference_rows(nu, eps: float, r, c, w, rows, min_size: int = 1024,
                         ncand: int = 16, M: int = None):
    """O2 at selected outputs only: the same partition and expansions as
    :func:`nufht_reference`, summed for the outputs w[rows] (caller order).
    Cost O(len(rows) * n) plus the local moments of the blocks involved."""
    r = np.asarray(r, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    sign, anu, local = _order(nu)
    M, z, L = prm.any_parameters(anu, eps, M)
    pr = np.argsort(r, kind='stable')
    pw = np.argsort(w, kind='stable')
    rs, cs, ws = r[pr], c[pr], w[pw]
    inv = np.empty_like(pw)
    inv[pw] = np.arange(pw.size)
    sel = np.sort(inv[rows])                  # sorted positions of the wanted outputs
    K = direct.staircase(rs, ws, z)
    blocks = partition.subdivide(K, ws.size, rs.size, min_size, ncand)
    acc = {int(j): 0.0 for j in sel}
    for b in blocks:
        lo = np.searchsorted(sel, b.j0)
        hi = np.searchsorted(sel, b.j1, side='right')
        if lo == hi:
            continue
        js = sel[lo:hi]
        cols = slice(b.k0, b.k1 + 1)
        if b.kind == 'L':
            v = local(anu, L, z, ws[js], rs[cols], cs[cols])
        elif b.kind == 'A':
            v = direct.asy_block_apply(anu, M, ws[js], rs[cols], cs[cols])
        else:
            v = direct.dht(anu, rs[cols], cs[cols], ws[js])
        for j, x in zip(js, v):
            acc[int(j)] += x
    return sign * np.array([acc[int(inv[q])] for q in rows])
