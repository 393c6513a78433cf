"""Expansion orders and crossover point (Sec. 3).

TEST INFRASTRUCTURE ONLY (see :mod:`oracle`).

For order nu and tolerance eps the method uses
* M   asymptotic terms, from the heuristic eq. num-asy-terms (Sec. 3.3);
* z   the crossover: the root of xi(z) = B^asy(z) - eps found by Newton's method,
      B^asy being the first-neglected-terms bound of eq. asy-error (Sec. 3.2);
* L   the smallest integer with B^loc(z) < eps, B^loc being the Wimp truncation
      bound of Lemma 3.1 (Sec. 3.1); the local sum keeps l = 0 .. L.

Readings of the paper taken here (each listed in the design doc):
* a_l(nu) is the product prod_{s=1}^{l} (4 nu^2 - (2s-1)^2) / (l! 8^l): the printed
  second factor "(4nu^2 - 3)" is read as "(4nu^2 - 9)", the pattern its last
  factor fixes.
* Lemma 3.1 sums l = 0 .. L, so an "L-term" local expansion keeps L + 1 terms.
* Odd nu: the paper only says a similar expansion and bound exist.  The bound
  used here follows the even-order proof step by step for the odd-order Wimp
  expansion sum_l 2 J_{(nu+1)/2+l}(x/2) J_{(nu-1)/2-l}(x/2) T_{2l+1}(y).
* Outside the Lemma's hypotheses (a Siegel argument >= 1, or a non-convergent
  geometric tail) the bound is taken as +inf, so that L grows until they hold.
* Negative orders use |nu| (J_{-nu} = (-1)^nu J_nu).

Half-integer orders nu = n + 1/2 (n >= 0; the paper treats integer orders only):
* Hankel's expansion terminates after a_n (a_l(nu) = 0 for l > n), so with
  2M >= n + 1 terms it is exact: M is the eq. num-asy-terms value capped at
  ceil((n + 1) / 2).  With an exact expansion B^asy = 0 and the crossover is
  set by conditioning instead: z is the smallest z >= 1 at which the retained
  terms' magnitudes sum_{k < min(2M, n+1)} |a_k| z^-k are at most 10 (an
  asymptotic entry, omega r > z, then amplifies the type-3 transforms' error,
  about eps / 10, by at most 10).
  When 2M < n + 1 the crossover is Newton's root as for integer orders (at
  least 1).
* Local blocks use J_{n+1/2}(x y) = sqrt(y) sqrt(2x/pi) j_n(x y) with the
  Chebyshev series of the entire function y -> j_n(x y) (parity (-1)^n):
  beta_k(x), k = n mod 2, n mod 2 + 2, ...  L is the smallest integer with
  B(L) = 2 sqrt(2z/pi) sum_{k > 2L + e, k = e mod 2} exp(k psi(z/k)) < eps,
  from |beta_k(x)| <= 2 max_{t <= x} |J_k(t)| and the Siegel bound
  |J_k(k p)| <= exp(k psi(p)) that Lemma 3.1 also uses (DLMF 10.14.5); +inf
  while some k <= z.
"""
import math

SQRT_2_OVER_PI = math.sqrt(2.0 / math.pi)


def num_asy_terms(nu: int, eps: float) -> int:
    """M = min(floor(1 + nu/5 - log10(eps)/4), 20)  (eq. num-asy-terms)."""
    return min(math.floor(1.0 + abs(nu) / 5.0 - math.log10(eps) / 4.0), 20)


def hankel_coef(nu: float, l: int) -> float:
    """a_l(nu) = prod_{s=1}^{l} (4 nu^2 - (2s-1)^2) / (l! 8^l)  (Sec. 3.2)."""
    a = 1.0
    for s in range(1, l + 1):
        a *= (4.0 * nu * nu - (2 * s - 1) ** 2) / (8.0 * s)
    return a


def asy_bound(nu: int, M: int, z: float) -> float:
    """B^asy(z): the first two neglected terms of the M-term expansion at
    argument z, times sqrt(2/pi)  (eq. asy-error)."""
    a0 = abs(hankel_coef(nu, 2 * M))
    a1 = abs(hankel_coef(nu, 2 * M + 1))
    return SQRT_2_OVER_PI * (a0 / z ** (2 * M + 0.5) + a1 / z ** (2 * M + 1.5))


def crossover(nu: int, eps: float, M: int) -> float:
    """z: root of xi(z) = B^asy(z) - eps by Newton's method (Sec. 3.3).

    xi is convex and decreasing on z > 0, so Newton's iteration started left of
    the root increases monotonically to it.  The start is the root of the first
    term alone, which lies left of the root of the full bound.
    """
    a0 = SQRT_2_OVER_PI * abs(hankel_coef(nu, 2 * M))
    a1 = SQRT_2_OVER_PI * abs(hankel_coef(nu, 2 * M + 1))
    p0 = 2 * M + 0.5
    p1 = 2 * M + 1.5
    z = (a0 / eps) ** (1.0 / p0)
    for _ in range(200):
        xi = a0 * z ** -p0 + a1 * z ** -p1 - eps
        dxi = -p0 * a0 * z ** (-p0 - 1.0) - p1 * a1 * z ** (-p1 - 1.0)
        step = xi / dxi
        z_new = z - step
        if abs(z_new - z) <= 1e-15 * z:
            return z_new
        z = z_new
    return z


def psi(p: float) -> float:
    """psi(p) = log p + sqrt(1-p^2) - log(1 + sqrt(1-p^2)), 0 < p <= 1 (Lemma 3.1)."""
    s = math.sqrt(1.0 - p * p)
    return math.log(p) + s - math.log(1.0 + s)


def local_bound(nu: int, L: int, z: float) -> float:
    """B^loc(z) for the local expansion with terms l = 0 .. L (Lemma 3.1)."""
    nu = abs(nu)
    if z <= 0.0:
        return 0.0
    if nu % 2 == 0:
        d_beta = 2 * L + 2 + nu
        d_gamma = 2 * L + 2 - nu
        gamma_applies = (L + 1) >= nu / 2.0
        lead_b, lead_g = nu / 2.0, nu / 2.0
    else:
        d_beta = 2 * L + 3 + nu
        d_gamma = 2 * L + 3 - nu
        gamma_applies = d_gamma > 0
        lead_b, lead_g = (nu + 1) / 2.0, (nu - 1) / 2.0
    pb = z / d_beta
    if pb >= 1.0:
        return math.inf
    beta = psi(pb)
    if gamma_applies:
        if d_gamma <= 0:
            return math.inf
        pg = z / d_gamma
        if pg >= 1.0:
            return math.inf
        gamma = psi(pg)
    else:
        gamma = 0.0
    if beta + gamma >= 0.0:
        return math.inf
    return (2.0 * math.exp(lead_b * beta - lead_g * gamma + (L + 1) * (beta + gamma))
            / (1.0 - math.exp(beta + gamma)))


def local_rank(nu: int, eps: float, z: float, L_max: int = 100000) -> int:
    """L: the smallest integer with B^loc(z) < eps (Sec. 3.3)."""
    for L in range(0, L_max):
        if local_bound(nu, L, z) < eps:
            return L
    raise ValueError("no local rank below L_max")


def parameters(nu: int, eps: float, M: int = None):
    """(M, z, L) for order nu and tolerance eps (Alg. 2, first three lines)."""
    if M is None:
        M = num_asy_terms(nu, eps)
    z = crossover(nu, eps, M)
    L = local_rank(nu, eps, z)
    return M, z, L


def tail_local_rank(nu: int, eps: float, z: float, L_lemma: int, grid: int = 512):
    """A tighter local rank: the smallest L <= L_lemma whose dropped Wimp terms
    sum_{l > L} |C_l(x)| stay at or below eps / 2 at the grid points
    x = z g / grid, g = 1 .. grid (every entry of a local block is off by at
    most that sum, the Chebyshev factors being bounded by 1).  C_l(x) =
    delta_l J_{a+l}(x/2) J_{a-l}(x/2) (even nu), 2 J_{a+1+l}(x/2) J_{a-l}(x/2)
    (odd nu), a = floor(|nu| / 2), with SciPy's J.  Returns (L, tail maxima
    per L)."""
    import numpy as np
    from scipy import special
    nu = abs(int(nu))
    a = nu // 2
    lmax = L_lemma + 40
    l = np.arange(lmax + 1)
    tailmax = np.zeros(lmax + 1)
    for g in range(1, grid + 1):
        y = 0.5 * z * g / grid
        hi = special.jv(a + 1 + l, y) if nu % 2 else special.jv(a + l, y)
        lo = special.jv(np.abs(a - l), y)
        f = np.where((l > 0) | (nu % 2 == 1), 2.0, 1.0)
        C = f * np.abs(hi * lo)
        after = np.concatenate((np.cumsum(C[::-1])[::-1][1:], [0.0]))   # sum over l' > l
        tailmax = np.maximum(tailmax, after)
    for L in range(L_lemma):
        if tailmax[L] <= 0.5 * eps:
            return L, tailmax
    return L_lemma, tailmax


# ---------------------------------------------------------------------------
# Half-integer orders.
# ---------------------------------------------------------------------------
def is_half(nu) -> bool:
    """nu = n + 1/2 with n >= 0."""
    t = 2.0 * float(nu)
    return t == round(t) and int(round(t)) % 2 == 1 and t > 0


def half_num_asy_terms(nu: float, eps: float) -> int:
    """M for nu = n + 1/2: eq. num-asy-terms, capped where the expansion ends."""
    n = int(round(nu - 0.5))
    return min(num_asy_terms(nu, eps), (n + 2) // 2)


def half_crossover(nu: float, eps: float, M: int) -> float:
    """z for nu = n + 1/2 (see the module notes): conditioning when the M-term
    expansion is exact, else Newton's root; at least 1."""
    n = int(round(nu - 0.5))
    if 2 * M < n + 1:
        return max(crossover(nu, eps, M), 1.0)
    a = [abs(hankel_coef(nu, k)) for k in range(n + 1)]
    S = lambda z: sum(ak * z ** -k for k, ak in enumerate(a))
    if S(1.0) <= 10.0:
        return 1.0
    lo, hi = 1.0, 2.0
    while S(hi) > 10.0:
        hi *= 2.0
    for _ in range(200):                 # bisection: S decreases on z > 0
        mid = 0.5 * (lo + hi)
        if S(mid) > 10.0:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-15 * hi:
            break
    return hi


def half_local_bound(nu: float, L: int, z: float) -> float:
    """B(L) for the half-integer local expansion with Chebyshev terms of
    degree up to 2L + e (see the module notes)."""
    n = int(round(nu - 0.5))
    e = n % 2
    k = 2 * L + 2 + e
    if k <= z:
        return math.inf
    total = 0.0
    for _ in range(100000):
        term = math.exp(k * psi(z / k))
        total += term
        if term <= 1e-20 * total:
            break
        k += 2
    return 2.0 * math.sqrt(2.0 * z / math.pi) * total


def half_local_rank(nu: float, eps: float, z: float, L_max: int = 100000) -> int:
    for L in range(0, L_max):
        if half_local_bound(nu, L, z) < eps:
            return L
    raise ValueError("no local rank below L_max")


def half_parameters(nu: float, eps: float, M: int = None):
    """(M, z, L) for nu = n + 1/2."""
    if M is None:
        M = half_num_asy_terms(nu, eps)
    z = half_crossover(nu, eps, M)
    return M, z, half_local_rank(nu, eps, z)


def any_parameters(nu, eps: float, M: int = None):
    """(M, z, L) for an integer or half-integer order."""
    return half_parameters(float(nu), eps, M) if is_half(nu) else parameters(int(nu), eps, M)
