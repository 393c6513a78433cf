"""O1: the direct discrete Hankel transform and the oracle's own J_nu.

TEST INFRASTRUCTURE ONLY (see :mod:`oracle`).

g_j = sum_k c_k J_nu(w_j r_k)   (Sec. 1, eq. DHT; Sec. 2 writes it as g = A c
with A(j,k) = J_nu(w_j r_k)).  The sum is evaluated entry by entry in C
(``bessel.c``) with exact double-double arguments and compensated summation.
Orders are integers or positive half-integers (nu = n + 1/2, the radial
Fourier transform in odd dimensions).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from oracle.build_oracle import build
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_besselj.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int64, _dp]
    lib.orc_besselj_twice.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int64, _dp]
    lib.orc_dht_twice.argtypes = [ctypes.c_int, ctypes.c_int64, _dp, _dp, ctypes.c_int64, _dp, _dp, ctypes.c_int]
    lib.orc_hankel_series.argtypes = [ctypes.c_double, _dp, ctypes.c_int64, ctypes.c_int, _dp]
    lib.orc_hankel_coef.argtypes = [ctypes.c_double, ctypes.c_int]
    lib.orc_hankel_coef.restype = ctypes.c_double
    lib.orc_dht.argtypes = [ctypes.c_int, ctypes.c_int64, _dp, _dp, ctypes.c_int64, _dp, _dp, ctypes.c_int]
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_staircase.argtypes = [ctypes.c_int64, _dp, ctypes.c_int64, _dp, ctypes.c_double, _i64p]
    lib.orc_exact_le.argtypes = [_dp, _dp, ctypes.c_int64, ctypes.c_double, _i32p]
    lib.orc_asy_block.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int64, _dp,
                                  ctypes.c_int64, _dp, _dp, _dp]
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def two_prod(a, b):
    """Exact product a*b = hi + lo (Veltkamp/Dekker splitting, no fma needed)."""
    a = _f64(a)
    b = _f64(b)
    hi = a * b
    split = 134217729.0  # 2^27 + 1
    ca = split * a
    ah = ca - (ca - a)
    al = a - ah
    cb = split * b
    bh = cb - (cb - b)
    bl = b - bh
    lo = ((ah * bh - hi) + ah * bl + al * bh) + al * bl
    return hi, lo


def twice_order(nu) -> int:
    """2 nu for an integer order (any sign) or a positive half-integer order."""
    t = 2.0 * float(nu)
    if t != round(t):
        raise ValueError(f"order {nu} is neither an integer nor a half-integer")
    t = int(round(t))
    if t % 2 == 1 and t < 1:
        raise ValueError("negative half-integer orders are not supported")
    return t


def besselj(nu, x, x_lo=None):
    """J_nu(x + x_lo) for integer nu (any sign) or half-integer nu > 0, x >= 0,
    elementwise."""
    lib = _load()
    xh = _f64(np.atleast_1d(x))
    xl = _f64(np.zeros_like(xh) if x_lo is None else np.broadcast_to(x_lo, xh.shape))
    out = np.empty_like(xh)
    lib.orc_besselj_twice(twice_order(nu), _ptr(xh), _ptr(xl), xh.size, _ptr(out))
    return out.reshape(np.shape(x)) if np.ndim(x) else out[0]


def hankel_series(nu: float, x, nterms: int):
    """Hankel's large-argument expansion (Sec. 3.2) at real order nu, keeping
    the terms a_k/x^k for k = 0 .. nterms-1."""
    lib = _load()
    xs = _f64(np.atleast_1d(x))
    out = np.empty_like(xs)
    lib.orc_hankel_series(float(nu), _ptr(xs), xs.size, int(nterms), _ptr(out))
    return out.reshape(np.shape(x)) if np.ndim(x) else out[0]


def hankel_coef(nu: float, k: int) -> float:
    """a_k(nu) = prod_{s=1}^{k} (4 nu^2 - (2s-1)^2) / (k! 8^k)  (Sec. 3.2)."""
    return _load().orc_hankel_coef(float(nu), int(k))


def dht(nu, r, c, w, nthreads: int = 0):
    """O1: g_j = sum_k c_k J_nu(w_j r_k) by direct summation (Sec. 1, eq. DHT).

    r, c: the n points and their weights; w: the m frequencies.  Any order of
    the inputs; the output follows the order of w.  Zero weights are skipped,
    which makes the sparse-input reference of Sec. 5.1.3 (a vector with few
    nonzeros) cost O(nnz * m).
    """
    lib = _load()
    r = _f64(r)
    c = _f64(c)
    w = _f64(w)
    g = np.zeros(w.shape[0], dtype=np.float64)
    if r.size and w.size:
        lib.orc_dht_twice(twice_order(nu), r.size, _ptr(r), _ptr(c), w.size, _ptr(w), _ptr(g), int(nthreads))
    return g


def max_threads() -> int:
    return int(_load().orc_max_threads())


def staircase(r_sorted, w, z: float):
    """K[j] = #{k : w_j r_k <= z} for ascending r, deciding each product exactly."""
    lib = _load()
    r_sorted = _f64(r_sorted)
    w = _f64(w)
    K = np.zeros(w.size, dtype=np.int64)
    if w.size:
        lib.orc_staircase(r_sorted.size, _ptr(r_sorted), w.size, _ptr(w), float(z), _ptr(K, _i64p))
    return K


def exact_le(w, r, z: float):
    """Elementwise [w*r <= z] with the product decided exactly."""
    lib = _load()
    w = _f64(w)
    r = _f64(r)
    out = np.zeros(w.size, dtype=np.int32)
    lib.orc_exact_le(_ptr(w), _ptr(r), w.size, float(z), _ptr(out, _i32p))
    return out.astype(bool)


def asy_block_apply(nu, M: int, w_rows, r_cols, c_cols):
    """sum_k c_k H_M(w_i r_k) for each row i, with H_M the M-term Hankel
    approximation of J_nu (Sec. 3.2, eq. asy-error), summed directly."""
    lib = _load()
    w_rows = _f64(w_rows)
    r_cols = _f64(r_cols)
    c_cols = _f64(c_cols)
    g = np.zeros(w_rows.size, dtype=np.float64)
    if w_rows.size and r_cols.size:
        lib.orc_asy_block(float(nu), int(M), w_rows.size, _ptr(w_rows), r_cols.size,
                          _ptr(r_cols), _ptr(c_cols), _ptr(g))
    return g
