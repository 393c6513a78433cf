"""Seeded synthetic inputs for the nonuniform discrete Hankel transform.

This module only draws inputs; it holds none of the transform's arithmetic.
The tests, the benchmark and the smoke check use it on both sides of every
comparison (GPU library and CPU oracle).

All arrays are float64.  Draw order within one workload: r, then w, then c,
then y (the cotangent of the gradient workload).  The workloads follow the
shapes and distributions of the paper's experiments (Sec. 5) and of the
benchmark configurations:

* ``uniform``       r ~ U[0, rmax), w ~ U[0, wmax), c ~ N(0, 1)
* ``radial_2d``     the radial 2-D Fourier transform of a smooth profile:
                    Chebyshev-clustered r on [0, 1], trapezoid weights w_k,
                    c_k = r_k w_k exp(-40 r_k^2) cos(30 r_k), log-spaced w on
                    [1e-2, 1e5] (stands in for the radial-FT study of Sec. 5.2)
* ``radial_3d``     the radial Fourier transform in three dimensions (order
                    1/2): the same points and frequencies, c_k = r_k^(3/2) w_k
                    exp(-40 r_k^2) cos(30 r_k)  (F(omega) = (2 pi)^(3/2)
                    omega^(-1/2) sum_k c_k J_{1/2}(omega r_k))
* ``sparse_c``      c with a fixed number of N(0, 1) nonzeros at random indices
                    (the accuracy study of Sec. 5.1.3)
* ``batch``         many independent transforms with uneven n, m and order
* ``fourier_bessel`` the Fourier-Bessel case of the p = O(n) study (Sec. 5.1):
                    w_j = j_{nu,j}, r_k = j_{nu,k} / j_{nu,n+1} (the scaled
                    zeros of J_nu, from ``bessel_zeros``), n = m
* ``exponential``   the exponentially distributed case of the same study:
                    w_j = r_j log-spaced over [n^(-1/2), n^(1/2)], n = m
* ``disk``          the Helmholtz solver on the unit disk (Sec. 5.3): m
                    Gauss-Legendre radii on [0, 1] with their weights, t
                    equispaced angles, the first J zeros of J_0 .. J_L, and a
                    random smooth forcing that vanishes with its derivatives
                    at r = 1 (Gaussian bumps times (1 - r^2)^6)
"""
import numpy as np


def uniform(n: int, m: int, rmax: float, wmax: float, seed: int):
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.0, rmax, n)
    w = rng.uniform(0.0, wmax, m)
    c = rng.standard_normal(n)
    return r, w, c


def small_dense(seed: int = 1):
    """n = m = 2000, r ~ U[0,1), w ~ U[0,500), c ~ N(0,1)."""
    return uniform(2000, 2000, 1.0, 500.0, seed)


def large_uniform(seed: int = 2, n: int = 1_000_000, m: int = 1_000_000):
    """n = m = 1e6, r ~ U[0,1) unsorted, w ~ U[0,1e5), c ~ N(0,1)."""
    return uniform(n, m, 1.0, 1e5, seed)


def radial_2d(n: int = 1_000_000, m: int = 1_000_000):
    """Deterministic radial 2-D Fourier-transform workload (no randomness)."""
    i = np.arange(n, dtype=np.float64)
    r = 0.5 * (1.0 - np.cos(np.pi * i / (n - 1)))
    wt = np.empty(n)
    wt[0] = 0.5 * (r[1] - r[0])
    wt[-1] = 0.5 * (r[-1] - r[-2])
    wt[1:-1] = 0.5 * (r[2:] - r[:-2])
    c = r * wt * np.exp(-40.0 * r * r) * np.cos(30.0 * r)
    k = np.arange(m, dtype=np.float64)
    w = 10.0 ** (-2.0 + 7.0 * k / (m - 1))
    return r, w, c


def radial_3d(n: int = 1_000_000, m: int = 1_000_000):
    """Deterministic radial 3-D Fourier-transform workload (order 1/2)."""
    i = np.arange(n, dtype=np.float64)
    r = 0.5 * (1.0 - np.cos(np.pi * i / (n - 1)))
    wt = np.empty(n)
    wt[0] = 0.5 * (r[1] - r[0])
    wt[-1] = 0.5 * (r[-1] - r[-2])
    wt[1:-1] = 0.5 * (r[2:] - r[:-2])
    c = r ** 1.5 * wt * np.exp(-40.0 * r * r) * np.cos(30.0 * r)
    k = np.arange(m, dtype=np.float64)
    w = 10.0 ** (-2.0 + 7.0 * k / (m - 1))
    return r, w, c


def sparse_c(n: int, nnz: int, seed: int):
    """A length-n vector with nnz N(0,1) entries at distinct random indices."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(n, size=nnz, replace=False)
    c = np.zeros(n)
    c[idx] = rng.standard_normal(nnz)
    return c


def cotangent(m: int, seed: int):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(m)


def batch(count: int = 256, seed: int = 5, lo: float = 3.0, hi: float = 6.0, nu_max: int = 63):
    """count independent transforms: nu ~ U{0..nu_max}, n and m log-uniform in
    [10^lo, 10^hi], r ~ U[0,1), w ~ U[0, n_i), c ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nu = int(rng.integers(0, nu_max + 1))
        n = int(round(10.0 ** rng.uniform(lo, hi)))
        m = int(round(10.0 ** rng.uniform(lo, hi)))
        r = rng.uniform(0.0, 1.0, n)
        w = rng.uniform(0.0, float(n), m)
        c = rng.standard_normal(n)
        out.append(dict(nu=nu, r=r, w=w, c=c))
    return out


def differentiation(seed: int = 6, n: int = 1_000_000, m: int = 1_000_000):
    """The differentiation case: r, w, c as the large uniform case, then the
    target y ~ N(0,1) of the loss 0.5 |g - y|^2 (drawn in that order)."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.0, 1.0, n)
    w = rng.uniform(0.0, 1e5, m)
    c = rng.standard_normal(n)
    y = rng.standard_normal(m)
    return r, w, c, y


def random_case(seed: int):
    """A seeded random transform for broad parity checks.

    Returns (nu, eps, r, w, c, kind): n, m log-uniform in [1, 4000]; order
    nu in [-8, 20]; eps in {1e-4, 1e-6, 1e-8, 1e-10, 1e-12}; the product range
    rmax * wmax log-uniform in [10, 2e4]; kind picks the distributions:
    'uniform' (r ~ U[0, rmax), w ~ U[0, wmax)), 'clustered' (r ~ |N(rmax/2,
    rmax/20)|, w ~ U[wmax/2, wmax)), 'log' (log-uniform r and w over three
    decades below their maxima), 'dups' (r drawn from 10 distinct values),
    'zeros' (uniform with a tenth of r and of w set to 0).  c ~ N(0, 1).
    """
    rng = np.random.default_rng(1000 + seed)
    n = int(round(10 ** rng.uniform(0.0, np.log10(4000.0))))
    m = int(round(10 ** rng.uniform(0.0, np.log10(4000.0))))
    nu = int(rng.integers(-8, 21))
    eps = float(rng.choice([1e-4, 1e-6, 1e-8, 1e-10, 1e-12]))
    prod = 10 ** rng.uniform(1.0, np.log10(2e4))
    rmax = 10 ** rng.uniform(-1.0, 1.0)
    wmax = prod / rmax
    kind = str(rng.choice(["uniform", "clustered", "log", "dups", "zeros"]))
    if kind == "clustered":
        r = np.abs(rng.normal(0.5 * rmax, 0.05 * rmax, n))
        w = rng.uniform(0.5 * wmax, wmax, m)
    elif kind == "log":
        r = rmax * 10 ** rng.uniform(-3.0, 0.0, n)
        w = wmax * 10 ** rng.uniform(-3.0, 0.0, m)
    elif kind == "dups":
        r = rng.choice(rng.uniform(0.0, rmax, 10), n)
        w = rng.uniform(0.0, wmax, m)
    else:
        r = rng.uniform(0.0, rmax, n)
        w = rng.uniform(0.0, wmax, m)
        if kind == "zeros":
            r[rng.random(n) < 0.1] = 0.0
            w[rng.random(m) < 0.1] = 0.0
    c = rng.standard_normal(n)
    return nu, eps, r, w, c, kind


def bessel_zeros(nu: int, count: int) -> np.ndarray:
    """The first ``count`` positive zeros j_{|nu|,1} < j_{|nu|,2} < ... of J_nu
    (J_{-nu} = (-1)^nu J_nu has the same zeros), computed by SciPy's
    ``special.jn_zeros``.  Used only to place points and frequencies."""
    from scipy import special
    if count <= 0:
        return np.zeros(0)
    return np.asarray(special.jn_zeros(abs(int(nu)), int(count)), dtype=np.float64)


def fourier_bessel(n: int, nu: int, seed: int):
    """w_j = j_{nu,j} (j = 1..n), r_k = j_{nu,k} / j_{nu,n+1} (k = 1..n), c ~ N(0, 1)."""
    z = bessel_zeros(nu, n + 1)
    r = z[:n] / z[n]
    w = z[:n].copy()
    c = np.random.default_rng(seed).standard_normal(n)
    return r, w, c


def exponential(n: int, seed: int):
    """w_j = r_j = 10^(log10(n) (j-1)/(n-1) - log10(n)/2), j = 1..n: log-spaced
    over [n^(-1/2), n^(1/2)], so the products w r span [1/n, n]; c ~ N(0, 1)."""
    if n == 1:
        x = np.ones(1)
    else:
        lg = np.log10(n)
        x = 10.0 ** (lg * np.arange(n) / (n - 1) - 0.5 * lg)
    c = np.random.default_rng(seed).standard_normal(n)
    return x.copy(), x.copy(), c


def disk(m: int, t: int, L: int, J: int, seed: int, bumps: int = 8):
    """Polar grid, zeros and forcing of the disk solver.

    Returns (r, wr, zeros, f): r, wr the m Gauss-Legendre nodes and weights
    mapped to [0, 1] (ascending r); zeros an (L + 1) x J array, row l the
    first J positive zeros of J_l; f an m x t array of samples
    f(r_k, 2 pi s / t) of (1 - r^2)^6 sum_i a_i exp(-|x - x_i|^2 / (2 s_i^2)),
    a_i ~ N(0, 1), centres x_i uniform in the disk of radius 0.7, widths
    s_i ~ U[0.08, 0.2]."""
    x, wx = np.polynomial.legendre.leggauss(m)
    r = 0.5 * (x + 1.0)
    wr = 0.5 * wx
    zeros = np.stack([bessel_zeros(l, J) for l in range(L + 1)]) if J > 0 else np.zeros((L + 1, 0))
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(bumps)
    rad = 0.7 * np.sqrt(rng.uniform(0.0, 1.0, bumps))
    ang = rng.uniform(0.0, 2.0 * np.pi, bumps)
    sw = rng.uniform(0.08, 0.2, bumps)
    theta = 2.0 * np.pi * np.arange(t) / t
    X = r[:, None] * np.cos(theta)[None, :]
    Y = r[:, None] * np.sin(theta)[None, :]
    f = np.zeros((m, t))
    for i in range(bumps):
        d2 = (X - rad[i] * np.cos(ang[i])) ** 2 + (Y - rad[i] * np.sin(ang[i])) ** 2
        f += a[i] * np.exp(-d2 / (2.0 * sw[i] ** 2))
    f *= ((1.0 - r * r) ** 6)[:, None]
    return r, wr, zeros, f
