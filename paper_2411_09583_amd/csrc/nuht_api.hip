// nuht_api.hip -- host side of libnuht: expansion parameters (Sec. 3.3), ES
// kernel set-up, plan construction (sort, staircase, Alg. 1) and the C ABI.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "nuht.h"
#include "nuht_launch.h"

namespace nuht {

// ===========================================================================
// Expansion parameters (Sec. 3.3).
// ===========================================================================

// M = min(floor(1 + nu/5 - log10(eps)/4), 20)   (eq. num-asy-terms)
static int num_asy_terms(double nu, double eps)
{
    int M = (int)std::floor(1.0 + std::fabs(nu) / 5.0 - std::log10(eps) / 4.0);
    return std::min(std::max(M, 1), 20);
}

// a_l(nu) = prod_{s=1}^{l} (4 nu^2 - (2s-1)^2) / (l! 8^l)   (Sec. 3.2)
static double hankel_coef(double nu, int l)
{
    double a = 1.0;
    for (int s = 1; s <= l; ++s) {
        double f = 2.0 * s - 1.0;
        a *= (4.0 * nu * nu - f * f) / (8.0 * s);
    }
    return a;
}

// Newton's method on xi(z) = B^asy(z) - eps, B^asy the first-neglected-terms
// bound of eq. asy-error.  xi is convex and decreasing; the iteration starts at
// the root of the first term alone, left of the root, and increases to it.
static double crossover(double nu, double eps, int M)
{
    const double s2p = std::sqrt(2.0 / M_PI);
    double a0 = s2p * std::fabs(hankel_coef(nu, 2 * M));
    double a1 = s2p * std::fabs(hankel_coef(nu, 2 * M + 1));
    double p0 = 2.0 * M + 0.5, p1 = 2.0 * M + 1.5;
    double z = std::pow(a0 / eps, 1.0 / p0);
    for (int it = 0; it < 200; ++it) {
        double xi = a0 * std::pow(z, -p0) + a1 * std::pow(z, -p1) - eps;
        double dxi = -p0 * a0 * std::pow(z, -p0 - 1.0) - p1 * a1 * std::pow(z, -p1 - 1.0);
        double zn = z - xi / dxi;
        if (std::fabs(zn - z) <= 1e-15 * z) return zn;
        z = zn;
    }
    return z;
}

// psi(p) = log p + sqrt(1-p^2) - log(1 + sqrt(1-p^2))   (Lemma 3.1)
static double psi_fn(double p)
{
    double s = std::sqrt(1.0 - p * p);
    return std::log(p) + s - std::log1p(s);
}

// Truncation bound of the Wimp expansion with terms l = 0..L on omega r <= z.
// Even nu: Lemma 3.1.  Odd nu: the same argument for the odd-order expansion
// sum_l 2 J_{(nu+1)/2+l}(x/2) J_{(nu-1)/2-l}(x/2) T_{2l+1}(y).  Outside the
// Lemma's hypotheses the bound is +inf.
static double local_bound(int nu, int L, double z)
{
    nu = std::abs(nu);
    double db, dg, lb, lg;
    bool g_applies;
    if (nu % 2 == 0) {
        db = 2.0 * L + 2 + nu; dg = 2.0 * L + 2 - nu; g_applies = (L + 1) >= nu / 2.0;
        lb = nu / 2.0; lg = nu / 2.0;
    } else {
        db = 2.0 * L + 3 + nu; dg = 2.0 * L + 3 - nu; g_applies = dg > 0;
        lb = (nu + 1) / 2.0; lg = (nu - 1) / 2.0;
    }
    double pb = z / db;
    if (pb >= 1.0) return INFINITY;
    double beta = psi_fn(pb), gamma = 0.0;
    if (g_applies) {
        if (dg <= 0.0) return INFINITY;
        double pg = z / dg;
        if (pg >= 1.0) return INFINITY;
        gamma = psi_fn(pg);
    }
    if (beta + gamma >= 0.0) return INFINITY;
    return 2.0 * std::exp(lb * beta - lg * gamma + (L + 1) * (beta + gamma)) / (1.0 - std::exp(beta + gamma));
}

static int local_rank(int nu, double eps, double z)
{
    for (int L = 0; L < 100000; ++L)
        if (local_bound(nu, L, z) < eps) return L;
    return -1;
}

// A tighter local rank: the smallest L whose dropped Wimp terms,
// sum_{l > L} |C_l(x)|, stay below eps / 2 at 512 equispaced x in (0, z]
// (every entry of a local block is off by at most that sum, |T_2l| <= 1),
// and never above L_lemma.  C_l(x) = delta_l J_{a+l}(x/2) J_{a-l}(x/2) for
// even nu and 2 J_{a+1+l}(x/2) J_{a-l}(x/2) for odd nu (a = floor(nu/2),
// |J_{-k}| = |J_k|), the J_k from Miller's backward recurrence in long
// double, normalised by J_0 + 2 sum_k J_2k = 1.
static int local_rank_tail(int nu, double eps, double z, int L_lemma)
{
    const int a = nu >> 1;
    const int lmax = L_lemma + 40;
    const int K = a + 2 + lmax;                     // highest order a term needs
    std::vector<long double> J(K + 1), C(lmax + 1);
    std::vector<double> tailmax(lmax + 1, 0.0);     // max over x of sum_{l' > l} |C_l'|
    const int G = 512;
    for (int g = 1; g <= G; ++g) {
        const long double y = 0.5L * (long double)z * g / G;
        const int N = K + 30 + (int)(y + 8.0L * std::cbrt(y));
        long double jp = 0.0L, jc = 1e-30L, S = 0.0L;
        for (int k = N; k >= 1; --k) {
            if (k <= K) J[k] = jc;
            if ((k & 1) == 0) S += 2.0L * jc;
            const long double jm = (2.0L * k / y) * jc - jp;
            jp = jc;
            jc = jm;
            if (std::fabs(jc) > 1e2000L) {          // rescale the running and stored values
                jp *= 1e-2000L; jc *= 1e-2000L; S *= 1e-2000L;
                for (int q = k - 1 > K ? K + 1 : k - 1; q <= K; ++q)
                    if (q >= 0) J[q] *= 1e-2000L;
            }
        }
        J[0] = jc;
        S += jc;
        for (int k = 0; k <= K; ++k) J[k] /= S;
        for (int l = 0; l <= lmax; ++l) {
            const int lo = a - l < 0 ? l - a : a - l;
            const long double hi = (nu & 1) ? J[a + 1 + l] : J[a + l];
            const long double f = ((nu & 1) || l > 0) ? 2.0L : 1.0L;
            C[l] = f * std::fabs(hi * J[lo]);
        }
        long double tail = 0.0L;
        for (int l = lmax; l >= 0; --l) {
            if ((double)tail > tailmax[l]) tailmax[l] = (double)tail;
            tail += C[l];
        }
    }
    for (int L = 0; L < L_lemma; ++L)
        if (tailmax[L] <= 0.5 * eps) return L;
    return L_lemma;
}

// ===========================================================================
// Half-integer orders nu = n + 1/2 (n >= 0).  The paper covers integer orders;
// for half-integers:
//  - Hankel's expansion ends at a_n (a_l(n + 1/2) = 0 for l > n), so M is the
//    eq. num-asy-terms value capped at ceil((n + 1) / 2); with 2M >= n + 1 the
//    expansion is exact and the crossover is set by conditioning: the smallest
//    z >= 1 where the retained terms' magnitudes sum_k |a_k| z^-k are at most
//    10 (the type-3 transforms run about a decade below eps); otherwise
//    Newton's root of B^asy = eps, at least 1;
//  - local blocks use J_{n+1/2}(x y) = sqrt(y) sqrt(2x/pi) j_n(x y), j_n the
//    spherical Bessel function (DLMF 10.47.3), expanded in Chebyshev
//    polynomials of y (j_n(x y) is entire in y with parity (-1)^n):
//      j_n(x y) = sum_l beta_{e+2l}(x) T_{e+2l}(y),  e = n mod 2,
//      beta_k(x) = eps_k (-1)^((k-n)/2) int_0^1 P_n(s) J_k(x s) ds
//    (from j_n(t) = (1/2) (-i)^n int_{-1}^{1} e^{i t s} P_n(s) ds and the
//    Jacobi-Anger expansion of e^{i x s cos theta}; eps_0 = 1, else 2);
//  - L is the smallest integer with
//      2 sqrt(2z/pi) sum_{k > 2L+e, k = e mod 2} exp(k psi(z/k)) < eps,
//    from |beta_k(x)| <= 2 max_{t<=x} |J_k(t)| and the Siegel bound
//    |J_k(k p)| <= exp(k psi(p)) of Lemma 3.1 (+inf while some k <= z).
// The beta_k are tabulated on panels of x in [0, z] (kHalfWidth wide, Chebyshev
// interpolants of degree kHalfDeg rewritten as monomials in the panel
// variable tau in [-1, 1]), computed on the host in long double: on the first
// panel by their power series, on the others by the Chebyshev transform of
// samples of j_n; the panels below x = n + 10 hold beta_k / x^n.
// ===========================================================================
static double half_crossover(double nu, double eps, int M)
{
    const int n = (int)(nu - 0.5 + 0.25);
    if (2 * M < n + 1) return std::max(crossover(nu, eps, M), 1.0);
    std::vector<double> a(n + 1);
    for (int k = 0; k <= n; ++k) a[k] = std::fabs(hankel_coef(nu, k));
    auto S = [&](double z) {          // sum_k a_k z^-k by Horner in 1/z
        double v = 0.0;
        for (int k = n; k >= 0; --k) v = v / z + a[k];
        return v;
    };
    auto dS = [&](double z) {         // S'(z) = -sum_k k a_k z^-k-1
        double v = 0.0;
        for (int k = n; k >= 1; --k) v = v / z + k * a[k];
        return -v / (z * z);
    };
    if (S(1.0) <= 10.0) return 1.0;
    // S is convex and decreasing: Newton from the left of the root increases
    // to it; the left start is 1 (S(1) > 10)
    double z = 1.0;
    for (int it = 0; it < 200; ++it) {
        const double zn = z - (S(z) - 10.0) / dS(z);
        if (std::fabs(zn - z) <= 1e-15 * zn) return zn;
        z = zn;
    }
    return z;
}

static double half_local_bound(int n, int L, double z)
{
    const int e = n & 1;
    int k = 2 * L + 2 + e;
    if (k <= z) return INFINITY;
    double total = 0.0;
    for (int i = 0; i < 100000; ++i, k += 2) {
        const double p = z / k, r = std::sqrt(1.0 - p * p);
        const double term = std::exp(k * (std::log(p) + r - std::log1p(r)));
        total += term;
        if (term <= 1e-20 * total) break;
    }
    return 2.0 * std::sqrt(2.0 * z / M_PI) * total;
}

static int half_local_rank(int n, double eps, double z)
{
    for (int L = 0; L < 100000; ++L)
        if (half_local_bound(n, L, z) < eps) return L;
    return -1;
}

// j_n(t) (spherical Bessel) in long double for t >= 0: upward recurrence from
// j_{-1} = cos t / t, j_0 = sin t / t above the turning point (t > n + 1),
// Miller's backward recurrence normalised by sum_k (2k+1) j_k^2 = 1 below it.
static long double sph_jn_ld(int n, long double t)
{
    if (t == 0.0L) return n == 0 ? 1.0L : 0.0L;
    if (t > n + 1.0L) {
        long double jm = cosl(t) / t, j = sinl(t) / t;
        for (int k = 0; k < n; ++k) {
            const long double jp = ((2.0L * k + 1.0L) / t) * j - jm;
            jm = j;
            j = jp;
        }
        return j;
    }
    const int N = (int)(n + t + 30.0L + 15.0L * cbrtl(t > 1.0L ? t : 1.0L));
    long double yk1 = 0.0L, yk = 1e-300L, S = 0.0L, rn = 0.0L;
    for (int k = N; k >= 0; --k) {
        if (k == n) rn = yk;
        S += (2.0L * k + 1.0L) * yk * yk;
        if (k == 0) break;
        const long double ykm1 = ((2.0L * k + 1.0L) / t) * yk - yk1;
        yk1 = yk;
        yk = ykm1;
        if (fabsl(yk) > 1e1000L) { yk *= 1e-1000L; yk1 *= 1e-1000L; S *= 1e-2000L; rn *= 1e-1000L; }
    }
    return rn / sqrtl(S);
}

// beta_{e+2l}(x) by the discrete Chebyshev transform of y -> j_n(x y) at the Q
// points y_q = cos theta_q, theta_q = pi (2q + 1) / (2Q), Q above the degrees
// involved; cos(k theta_q) from the integer k (2q + 1) reduced modulo 4Q.
// Every sample is accurate relative to itself, so the coefficients are
// accurate relative to the largest sample even when all are tiny (x < n); a
// quadrature of the integral form cancels there instead.
static void half_beta_dct(int n, int L, long double x, long double* beta)
{
    const int e = n & 1, K = e + 2 * L;
    const int Q = K + 2 * (int)x + 64;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<long double> f(Q), cs(4 * Q);
    for (int i = 0; i < 4 * Q; ++i) cs[i] = cosl(pi * i / (2.0L * Q));
    for (int q = 0; q < Q; ++q) {
        const long double t = x * cs[2 * q + 1];
        const long double v = sph_jn_ld(n, fabsl(t));
        f[q] = (t < 0.0L && (n & 1)) ? -v : v;
    }
    for (int l = 0; l <= L; ++l) {
        const int k = e + 2 * l;
        long double sm = 0.0L;
        for (int q = 0; q < Q; ++q) sm += f[q] * cs[(int)(((int64_t)k * (2 * q + 1)) % (4 * Q))];
        beta[l] = sm * (k == 0 ? 1.0L : 2.0L) / Q;
    }
}

// gamma_{e+2l}(x) = beta_{e+2l}(x) / x^n, l = 0 .. L, for small x by the power
// series of J_k, with the moments mu_m = int_0^1 s^m P_n(s) ds: zero for
// m < n (the terms that cancel in the integral), else
// 2^n m! ((m+n)/2)! / (((m-n)/2)! (m+n+1)!) (m + n even):
//   beta_k(x) = eps_k (-1)^((k-n)/2) sum_j (-1)^j (x/2)^(k+2j) mu_{k+2j} / (j! (k+j)!).
// beta_k is O(x^n), so gamma is entire and known to full relative accuracy at
// small x, where the quadrature's cancellation would leave only absolute
// accuracy.  Used on the first panel, x <= kHalfWidth.
static void half_gamma(int n, int L, long double x, long double* gam)
{
    const int e = n & 1;
    const long double h = 0.5L * x;
    for (int l = 0; l <= L; ++l) {
        const int k = e + 2 * l;
        int j = k >= n ? 0 : (n - k) / 2;            // first term with k + 2j >= n
        int m = k + 2 * j;
        // log of 2^-n (x/2)^(m-n) mu_m / (j! (k+j)!), the first term without its sign
        auto log_mu = [&](int mm) {
            return n * logl(2.0L) + lgammal(mm + 1.0L) + lgammal((mm + n) / 2 + 1.0L) -
                   lgammal((mm - n) / 2 + 1.0L) - lgammal(mm + n + 2.0L);
        };
        long double term;
        if (x == 0.0L) {
            term = m == n ? expl(-n * logl(2.0L) + log_mu(m) - lgammal(j + 1.0L) - lgammal(k + j + 1.0L)) : 0.0L;
        } else {
            term = expl(-n * logl(2.0L) + (m - n) * logl(h) + log_mu(m) - lgammal(j + 1.0L) -
                        lgammal(k + j + 1.0L));
        }
        if (j & 1) term = -term;
        long double sum = term;
        for (int it = 0; it < 4000 && x != 0.0L; ++it) {
            // mu_{m+2} / mu_m and the factorials' ratio
            const long double r = (long double)(m + 2) * (m + 1) * ((m + n) / 2 + 1) /
                                  ((long double)((m - n) / 2 + 1) * (m + n + 3) * (m + n + 2));
            term *= -h * h * r / ((long double)(j + 1) * (k + j + 1));
            ++j;
            m += 2;
            sum += term;
            if (fabsl(term) <= 1e-24L * fabsl(sum)) break;
        }
        const long double sg = (((k - n) / 2) & 1) ? -1.0L : 1.0L;
        gam[l] = (k == 0 ? 1.0L : 2.0L) * sg * sum;
    }
}

// The leading panels tabulated as beta / x^n: every panel below x = n + 10
// (there beta grows like x^n, by many orders of magnitude across a panel at
// large n, while beta / x^n varies slowly), at least the first.
static int half_scaled_panels(int n) { return std::max(1, (int)((n + 10.0) / kHalfWidth)); }

// The table: panels p = 0 .. np-1 covering [p h, (p+1) h], h = kHalfWidth,
// np = ceil(z / h); entry [p][l][d] = coefficient of tau^d in the degree
// kHalfDeg interpolant, at the panel's Chebyshev points, of gamma_{e+2l} =
// beta_{e+2l} / x^n on the leading half_scaled_panels(n) panels and of
// beta_{e+2l} on the others.
static void half_table(int n, int L, double z, std::vector<double>& tab, int& np)
{
    const int D = kHalfDeg;
    np = std::max(1, (int)std::ceil(z / kHalfWidth));
    const int ns = half_scaled_panels(n);
    tab.assign((size_t)np * (L + 1) * (D + 1), 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    long double T[kHalfDeg + 1][kHalfDeg + 1] = {};   // T[j][i]: coefficient of tau^i in T_j(tau)
    T[0][0] = 1.0L;
    T[1][1] = 1.0L;
    for (int j = 2; j <= D; ++j)
        for (int i = 0; i <= j; ++i) T[j][i] = (i > 0 ? 2.0L * T[j - 1][i - 1] : 0.0L) - T[j - 2][i];
    auto panel = [&](int p) {
        std::vector<long double> val((size_t)(D + 1) * (L + 1)), a(D + 1);
        for (int i = 0; i <= D; ++i) {
            const long double t = cosl(pi * (i + 0.5L) / (D + 1));
            const long double x = (p + 0.5L * (t + 1.0L)) * (long double)kHalfWidth;
            long double* v = &val[(size_t)i * (L + 1)];
            if (p == 0) {
                half_gamma(n, L, x, v);
            } else {
                half_beta_dct(n, L, x, v);
                if (p < ns) {
                    const long double inv = powl(x, -(long double)n);
                    for (int l = 0; l <= L; ++l) v[l] *= inv;
                }
            }
        }
        for (int l = 0; l <= L; ++l) {
            for (int j = 0; j <= D; ++j) {
                long double sm = 0.0L;
                for (int i = 0; i <= D; ++i)
                    sm += val[(size_t)i * (L + 1) + l] * cosl(pi * j * (i + 0.5L) / (D + 1));
                a[j] = sm * (j == 0 ? 1.0L : 2.0L) / (D + 1);
            }
            double* out = &tab[((size_t)p * (L + 1) + l) * (D + 1)];
            for (int i = 0; i <= D; ++i) {
                long double c = 0.0L;
                for (int j = i; j <= D; ++j) c += a[j] * T[j][i];
                out[i] = (double)c;
            }
        }
    };
    const int nt = std::max(1, std::min({np, 16, (int)std::thread::hardware_concurrency()}));
    std::vector<std::thread> pool;
    std::atomic<int> next{0};
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&]() { for (int p; (p = next++) < np;) panel(p); });
    for (auto& th : pool) th.join();
}

// J_n(x), integer n >= 0, x >= 0, in extended precision: Miller's backward
// recurrence J_{k-1} = (2k/x) J_k - J_{k+1} started well above max(x, n),
// normalised by J_0^2 + 2 sum_{k>=1} J_k^2 = 1 (DLMF 10.23.3 with the
// addition theorem at zero angle), rescaled by exact powers of ten before it
// can overflow.
static long double besselj_ld(int n, long double x)
{
    if (x == 0.0L) return n == 0 ? 1.0L : 0.0L;
    const long double top = x > n ? x : (long double)n;
    const int N = (int)(top + 30.0L + 15.0L * cbrtl(x > 1.0L ? x : 1.0L));
    long double yk1 = 0.0L, yk = 1e-300L, S = 0.0L, jn = 0.0L;
    for (int k = N; k >= 0; --k) {
        if (k == n) jn = yk;
        S += (k == 0 ? 1.0L : 2.0L) * yk * yk;
        if (k == 0) break;
        const long double ykm1 = (2.0L * k / x) * yk - yk1;
        yk1 = yk;
        yk = ykm1;
        if (fabsl(yk) > 1e1000L) { yk *= 1e-1000L; yk1 *= 1e-1000L; S *= 1e-2000L; jn *= 1e-1000L; }
    }
    return jn / sqrtl(S);
}

// The direct-block table of order nu2 / 2 (nu2 odd: the half-integer order,
// through J_{n+1/2}(x) = sqrt(2x/pi) j_n(x)): np panels of width kJtabWidth
// from x0; entry [p][j] = coefficient of u^j, u in [-1, 1] across the panel,
// of the degree kJtabCoef - 1 interpolant at the panel's Chebyshev points,
// from samples, DCT and the change of basis in extended precision.
static void jtab_host(int nu2, double x0, int np, std::vector<double>& tab)
{
    const int D = kJtabCoef;
    const bool half = (nu2 & 1) != 0;
    const int n = half ? (nu2 - 1) / 2 : std::abs(nu2 / 2);
    tab.assign((size_t)np * D, 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    long double cs[4 * kJtabCoef];                   // cos(pi i / (2 D))
    for (int i = 0; i < 4 * D; ++i) cs[i] = cosl(pi * i / (2.0L * D));
    long double T[kJtabCoef][kJtabCoef] = {};        // T[k][j]: coefficient of u^j in T_k(u)
    T[0][0] = 1.0L;
    T[1][1] = 1.0L;
    for (int k = 2; k < D; ++k)
        for (int j = 0; j <= k; ++j) T[k][j] = (j > 0 ? 2.0L * T[k - 1][j - 1] : 0.0L) - T[k - 2][j];
    auto panel = [&](int p) {
        long double f[kJtabCoef], c[kJtabCoef];
        const long double centre = (long double)x0 + kJtabWidth * (p + 0.5L);
        for (int l = 0; l < D; ++l) {
            const long double x = centre + 0.5L * kJtabWidth * cs[2 * l + 1];
            f[l] = half ? sqrtl(2.0L * x / pi) * sph_jn_ld(n, x) : besselj_ld(n, x);
        }
        for (int k = 0; k < D; ++k) {
            long double sm = 0.0L;
            for (int l = 0; l < D; ++l) sm += f[l] * cs[(k * (2 * l + 1)) % (4 * D)];
            c[k] = sm * (k == 0 ? 1.0L : 2.0L) / D;
        }
        for (int j = 0; j < D; ++j) {
            long double a = 0.0L;
            for (int k = D - 1; k >= j; --k) a += c[k] * T[k][j];
            tab[(size_t)p * D + j] = (double)a;
        }
    };
    const int nt = std::max(1, std::min({np / 8, 16, (int)std::thread::hardware_concurrency()}));
    if (nt == 1) {
        for (int p = 0; p < np; ++p) panel(p);
        return;
    }
    std::vector<std::thread> pool;
    std::atomic<int> next{0};
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&]() { for (int p; (p = next++) < np;) panel(p); });
    for (auto& th : pool) th.join();
}

// The direct-block table of (nu2, x0, np) on the current device: built and
// uploaded once per device and key, kept until the process ends.
static const double* jtab_device(int nu2, double x0, int np)
{
    struct Entry {
        int dev, nu2, np;
        double x0;
        const double* p;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    std::lock_guard<std::mutex> lock(mu);
    for (const Entry& e : cache)
        if (e.dev == dev && e.nu2 == nu2 && e.np == np && e.x0 == x0) return e.p;
    std::vector<double> host;
    jtab_host(nu2, x0, np, host);
    void* p = nullptr;
    const size_t bytes = sizeof(double) * host.size();
    if (hipMalloc(&p, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    if (hipMemcpy(p, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(p);
        return nullptr;
    }
    cache.push_back(Entry{dev, nu2, np, x0, (const double*)p});
    return (const double*)p;
}

// The table of (n, L, z) on the current device: built and uploaded once per
// device and key, kept until the process ends.
static const double* half_table_device(int n, int L, double z, int* np_out, int* ns_out)
{
    struct Entry {
        int dev, n, L;
        double z;
        int np;
        const double* p;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    std::lock_guard<std::mutex> lock(mu);
    for (const Entry& e : cache)
        if (e.dev == dev && e.n == n && e.L == L && e.z == z) {
            *np_out = e.np;
            *ns_out = half_scaled_panels(n);
            return e.p;
        }
    std::vector<double> host;
    int np = 0;
    half_table(n, L, z, host, np);
    void* p = nullptr;
    const size_t bytes = sizeof(double) * host.size();
    if (hipMalloc(&p, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    if (hipMemcpy(p, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(p);
        return nullptr;
    }
    cache.push_back(Entry{dev, n, L, z, np, (const double*)p});
    *np_out = np;
    *ns_out = half_scaled_panels(n);
    return (const double*)p;
}

// ===========================================================================
// Exponential-of-semicircle kernel: width and shape from eps, and the
// Chebyshev series of its Fourier transform ES^(kappa) on [0, w pi / 4].
// ===========================================================================
// The type-3 transforms are run about a decade tighter than eps: the method's
// own truncation error already reaches ~0.8 eps in the max norm, so the NUFFT
// error must stay near eps/10 for the total to stay within eps.
static int es_width(double eps, int precision)
{
    int digits = (int)std::ceil(-std::log10(eps) - 1e-9);
    int w = precision == NUHT_FP32_SPREAD ? digits + 2 : digits + 3;
    return std::min(std::max(w, 4), kMaxEsWidth);
}

static double es_beta(int w) { return 2.30 * w; }

static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& wt)
{
    x.resize(n);
    wt.resize(n);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            double dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1; p1 = p2;
        }
        double dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[i] = t;
        wt[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

// ES^ on [0, kappa_max] as a polynomial in s = 2 (kappa / kappa_max)^2 - 1:
// values at the kEshatTerms Chebyshev points in s (Gauss-Legendre quadrature
// of the kernel's cosine transform, which converges fast as the kernel is
// smooth and e^-beta small at the ends), their Chebyshev interpolant, then its
// monomial coefficients in s, all in long double.
static void eshat_poly(double beta, double kappa_max, double* coef)
{
    constexpr int n = kEshatTerms;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<double> x, wt;
    gauss_legendre(240, x, wt);
    long double f[n], c[n];
    for (int j = 0; j < n; ++j) {
        const long double t = std::cos(pi * (j + 0.5L) / n);
        const long double kappa = (long double)kappa_max * std::sqrt(0.5L * (t + 1.0L));
        long double s = 0.0L;
        for (size_t i = 0; i < x.size(); ++i) {
            const long double xx = x[i];
            const long double es = std::exp((long double)beta * (std::sqrt(std::max(0.0L, 1.0L - xx * xx)) - 1.0L));
            s += (long double)wt[i] * es * std::cos(kappa * xx);
        }
        f[j] = s;
    }
    for (int k = 0; k < n; ++k) {
        long double s = 0.0L;
        for (int j = 0; j < n; ++j) s += f[j] * std::cos(pi * k * (j + 0.5L) / n);
        c[k] = 2.0L * s / n;
    }
    c[0] *= 0.5L;
    // sum_k c_k T_k(s) in monomials: T_{k+1} = 2 s T_k - T_{k-1}
    long double Tm[n] = {}, T0[n] = {}, a[n] = {};
    T0[0] = 1.0L;                 // T_0
    for (int k = 0; k < n; ++k) {
        for (int i = 0; i < n; ++i) a[i] += c[k] * T0[i];
        long double Tn[n] = {};
        if (k == 0) {
            Tn[1] = 1.0L;             // T_1 = s
        } else {
            for (int i = 0; i + 1 < n; ++i) Tn[i + 1] = 2.0L * T0[i];
            for (int i = 0; i < n; ++i) Tn[i] -= Tm[i];
        }
        for (int i = 0; i < n; ++i) { Tm[i] = T0[i]; T0[i] = Tn[i]; }
    }
    for (int i = 0; i < n; ++i) coef[i] = (double)a[i];
}

// The ES kernel as w polynomial pieces.  A point at grid coordinate u reaches
// the w cells l0 + t (t = 0 .. w-1), l0 = floor(u - w/2) + 1; with
// f = l0 - (u - w/2) in (0, 1], cell l0 + t sees ES((2 (t + f) - w) / w).
// Piece t is that function of s = 2 f - 1 on [-1, 1], interpolated at the
// kEsDeg + 1 Chebyshev points and rewritten in monomials of s, all in long
// double; coefficients are stored [t][d] (d = 0 .. kEsDeg).  Rounded to double
// and evaluated by Horner's rule in double, degree 13 stays within 1.6 e^-beta
// of the kernel for every width 8 .. 16 (about 1.1e-15 of its peak at
// w = 16), the same as degree 15; degree 12 doubles the error at w = 15.
static void es_pieces(int w, double beta, double* coef)
{
    const int D = kEsDeg;
    const long double pi = 3.141592653589793238462643383279502884L;
    long double node[kEsDeg + 1], val[kEsDeg + 1], a[kEsDeg + 1];
    long double T[kEsDeg + 1][kEsDeg + 1] = {};   // T[j][i]: coefficient of s^i in T_j(s)
    T[0][0] = 1.0L;
    T[1][1] = 1.0L;
    for (int j = 2; j <= D; ++j)
        for (int i = 0; i <= j; ++i) T[j][i] = (i > 0 ? 2.0L * T[j - 1][i - 1] : 0.0L) - T[j - 2][i];
    for (int k = 0; k <= D; ++k) node[k] = std::cos(pi * (k + 0.5L) / (D + 1));
    for (int t = 0; t < w; ++t) {
        for (int k = 0; k <= D; ++k) {
            long double f = 0.5L * (node[k] + 1.0L);
            long double x = (2.0L * (t + f) - w) / w;
            long double r = 1.0L - x * x;
            val[k] = r > 0.0L ? std::exp((long double)beta * (std::sqrt(r) - 1.0L)) : 0.0L;
        }
        for (int j = 0; j <= D; ++j) {
            long double sm = 0.0L;
            for (int k = 0; k <= D; ++k) sm += val[k] * std::cos(pi * j * (k + 0.5L) / (D + 1));
            a[j] = sm * (j == 0 ? 1.0L : 2.0L) / (D + 1);
        }
        for (int i = 0; i <= D; ++i) {
            long double c = 0.0L;
            for (int j = i; j <= D; ++j) c += a[j] * T[j][i];
            coef[t * (D + 1) + i] = (double)c;
        }
    }
}

// Cached per kernel width (beta follows w).
static const double* es_pieces_cached(int w, double beta)
{
    static std::mutex mu;
    static double table[kMaxEsWidth + 1][kMaxEsWidth * (kEsDeg + 1)];
    static bool have[kMaxEsWidth + 1] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (!have[w]) {
        es_pieces(w, beta, table[w]);
        have[w] = true;
    }
    return table[w];
}

// The pieces of width w on the current device: uploaded once per device and
// width and kept until the process ends (w x (kEsDeg + 1) doubles each).
static const double* es_pieces_device(int w, double beta)
{
    static std::mutex mu;
    static const double* table[64][kMaxEsWidth + 1] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) { (void)hipGetLastError(); return nullptr; }
    const double* host = es_pieces_cached(w, beta);
    std::lock_guard<std::mutex> lock(mu);
    if (!table[dev][w]) {
        void* p = nullptr;
        size_t bytes = sizeof(double) * (size_t)w * (kEsDeg + 1);
        if (hipMalloc(&p, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
        if (hipMemcpy(p, host, bytes, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(p);
            return nullptr;
        }
        table[dev][w] = (const double*)p;
    }
    return table[dev][w];
}

// FFT twiddles of the large-transform passes, one table per device:
// entries 0..4095 hold e^(2 pi i j / 4096) and entries 4096..8191 hold
// e^(2 pi i j / 2^24), each rounded from an extended-precision evaluation.
static const double2* fft_twiddles_device()
{
    static std::mutex mu;
    static const double2* table[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) { (void)hipGetLastError(); return nullptr; }
    std::lock_guard<std::mutex> lock(mu);
    if (!table[dev]) {
        std::vector<double2> host(8192);
        const long double two_pi = 6.283185307179586476925286766559005768L;
        for (int j = 0; j < 4096; ++j) {
            long double a = two_pi * (long double)j / 4096.0L;
            long double b = two_pi * (long double)j / 16777216.0L;
            host[j] = make_double2((double)cosl(a), (double)sinl(a));
            host[4096 + j] = make_double2((double)cosl(b), (double)sinl(b));
        }
        void* p = nullptr;
        size_t bytes = sizeof(double2) * host.size();
        if (hipMalloc(&p, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
        if (hipMemcpy(p, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(p);
            return nullptr;
        }
        table[dev] = (const double2*)p;
    }
    return table[dev];
}

// -(2nu+1) pi/4 modulo 2 pi as a double-double in (0, 2 pi], from the
// integer t = 2 nu + 1 (odd for integer orders, even for half-integers).
static void phase_offset2(int t, double& hi, double& lo)
{
    int k = 8 - (t % 8);                      // -(2nu+1) = k - 8(...)  (mod 8)
    const double q_hi = 0.78539816339744827900;   // pi/4 rounded
    const double q_lo = 3.0616169978683830e-17;   // pi/4 - q_hi
    double p = k * q_hi;                           // exact: k <= 8
    hi = p;
    lo = k * q_lo;
}

void phase_offset_dd(int nu, double* hi, double* lo) { phase_offset2(2 * nu + 1, *hi, *lo); }

// ===========================================================================
// Plan.
// ===========================================================================
struct Geometry {
    int32_t n = 0, m = 0;
    const double* rs = nullptr;
    const double* ws = nullptr;
    const int32_t* perm_r = nullptr;
    const int32_t* perm_w = nullptr;
};

// Device memory comes from a stream-ordered pool per device (plans are made
// and dropped often, and the pool keeps the memory between them).  Each
// buffer remembers the stream it was allocated on and is released there.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
};

static hipMemPool_t device_pool()
{
    static std::mutex mu;
    static hipMemPool_t pools[64] = {};
    static bool tried[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) { (void)hipGetLastError(); return nullptr; }
    std::lock_guard<std::mutex> lock(mu);
    if (!tried[dev]) {
        tried[dev] = true;
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        if (hipMemPoolCreate(&pool, &props) == hipSuccess) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
            pools[dev] = pool;
        } else {
            (void)hipGetLastError();
        }
    }
    return pools[dev];
}

// Device blocks of released plans whose every use has completed, kept for
// reuse by later plans: taking one costs no HIP call, where an allocation from
// the stream-ordered pool costs tens of microseconds of host time (a plan
// makes three).  A request takes the smallest cached block of at least its
// size and at most twice it (plus 64 MiB); at most kBlockCacheCap bytes are
// kept, blocks beyond that go back to the pool.
struct CachedBlock {
    int dev;
    void* p;
    size_t bytes;
};
static std::mutex block_mu;
static std::vector<CachedBlock> block_cache;
static size_t block_cached = 0;
constexpr size_t kBlockCacheCap = size_t(16) << 30;

static bool block_take(int dev, size_t bytes, void** p, size_t* got)
{
    std::lock_guard<std::mutex> lock(block_mu);
    size_t best = block_cache.size();
    for (size_t i = 0; i < block_cache.size(); ++i) {
        const CachedBlock& c = block_cache[i];
        if (c.dev != dev || c.bytes < bytes || c.bytes > 2 * bytes + (size_t(64) << 20)) continue;
        if (best == block_cache.size() || c.bytes < block_cache[best].bytes) best = i;
    }
    if (best == block_cache.size()) return false;
    *p = block_cache[best].p;
    *got = block_cache[best].bytes;
    block_cached -= *got;
    block_cache[best] = block_cache.back();
    block_cache.pop_back();
    return true;
}

static bool block_put(int dev, void* p, size_t bytes)
{
    std::lock_guard<std::mutex> lock(block_mu);
    if (block_cached + bytes > kBlockCacheCap) return false;
    block_cache.push_back(CachedBlock{dev, p, bytes});
    block_cached += bytes;
    return true;
}

static int dev_alloc(DevBuf& b, size_t bytes, hipStream_t s)
{
    b = DevBuf{};
    if (bytes == 0) return NUHT_OK;
    void* p = nullptr;
    int dev = 0;
    size_t got = 0;
    if (hipGetDevice(&dev) == hipSuccess && block_take(dev, bytes, &p, &got)) {
        b.p = p; b.bytes = got; b.stream = s;   // every earlier use has completed
        return NUHT_OK;
    }
    (void)hipGetLastError();
    hipMemPool_t pool = device_pool();
    hipError_t e = pool ? hipMallocFromPoolAsync(&p, bytes, pool, s) : hipMalloc(&p, bytes);
    if (e != hipSuccess) { (void)hipGetLastError(); return NUHT_ENOMEM; }
    b.p = p; b.bytes = bytes; b.stream = pool ? s : nullptr;
    return NUHT_OK;
}

static void dev_free(DevBuf& b)
{
    if (b.p) {
        if (b.stream || device_pool()) (void)hipFreeAsync(b.p, b.stream);
        else (void)hipFree(b.p);
    }
    b = DevBuf{};
}

struct Partition {
    bool built = false;
    PlanDev P{};
    Summary sum{};
    std::vector<FftClass> cls;
    ExecBuffers B{};
    Arena A{};
    std::vector<DevBuf> bufs;
    int64_t bytes = 0;
    hipStream_t stream = nullptr;   // where this partition's memory lives

    // Hands the device buffers to `out` (whoever frees them) and resets.
    void take_bufs(std::vector<DevBuf>& out)
    {
        for (auto& b : bufs) out.push_back(b);
        bufs.clear();
        release();
    }

    void release()
    {
        for (auto& b : bufs) dev_free(b);
        bufs.clear();
        bytes = 0;
        built = false;
        cls.clear();
        B = ExecBuffers{};
        A = Arena{};
    }
    Partition() = default;
    Partition(const Partition&) = delete;             // owns device memory
    Partition& operator=(const Partition&) = delete;
    ~Partition() { release(); }
};

// Several device arrays carved out of one allocation (256-byte aligned), so a
// plan makes a handful of allocation calls instead of dozens.
class Slab {
public:
    template <class T>
    void add(T*& out, size_t count)
    {
        reqs_.push_back(Req{(void**)&out, count * sizeof(T)});
    }
    size_t bytes() const
    {
        size_t t = 0;
        for (const Req& r : reqs_) t += round(r.bytes);
        return t;
    }
    // Allocates on stream s into b and assigns every requested pointer (null
    // for empty requests).
    int commit(DevBuf& b, hipStream_t s)
    {
        int rc = dev_alloc(b, bytes(), s);
        if (rc != NUHT_OK) return rc;
        char* base = (char*)b.p;
        for (const Req& r : reqs_) {
            *r.out = r.bytes ? (void*)base : nullptr;
            base += round(r.bytes);
        }
        return NUHT_OK;
    }
    int commit(Partition& Pt)
    {
        DevBuf b;
        int rc = commit(b, Pt.stream);
        if (rc != NUHT_OK) return rc;
        if (b.p) Pt.bufs.push_back(b);
        Pt.bytes += (int64_t)b.bytes;
        return NUHT_OK;
    }

private:
    struct Req {
        void** out;
        size_t bytes;
    };
    static size_t round(size_t x) { return (x + 255) & ~(size_t)255; }
    std::vector<Req> reqs_;
};

// Pinned host staging for the plan's one device-to-host read (the planning
// summary and the input-check flag).  Allocated once per process; a plan holds
// the lock from the copy to the read.
struct HostStage {
    Summary sum;
    int32_t flag;
};

static HostStage* host_stage(std::unique_lock<std::mutex>& lock)
{
    static std::mutex mu;
    static HostStage* stage = nullptr;
    lock = std::unique_lock<std::mutex>(mu);
    if (!stage) {
        void* p = nullptr;
        if (hipHostMalloc(&p, sizeof(HostStage), hipHostMallocPortable) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        stage = (HostStage*)p;
    }
    return stage;
}

}  // namespace nuht

using namespace nuht;

struct nuht_plan_s {
    int nu2_req = 0;             // twice the order (odd: a half-integer order)
    double eps = 0.0;
    nuht_opts opts{};            // opts.tune_cache is not kept (see cache_path)
    std::string cache_path;      // the tuning cache file, empty for none
    int64_t n = 0, m = 0;
    // Planning (sort, partitions) runs on `ps`, a stream of the library's, so
    // it overlaps work already queued on the caller's streams; ev_use marks
    // the last use of the plan's buffers on a caller stream, and anything the
    // plan frees is ordered after it.
    hipStream_t ps = nullptr;
    hipEvent_t ev_use = nullptr;
    hipEvent_t ev_plan = nullptr;  // marks the planning stream's queued work when the plan is released
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;   // an execution's fork to the side stream and back
    bool used = false;
    DevBuf b_geom;               // keys, values, sort scratch, summary, flag
    uint64_t* keys = nullptr;    // sorted points then sorted frequencies (bit patterns)
    int32_t* vals = nullptr;     // matching caller indices
    uint64_t* keys2 = nullptr;
    int32_t* vals2 = nullptr;
    int32_t* hist = nullptr;
    Summary* d_sum = nullptr;
    int32_t* d_flag = nullptr;   // domain error flag of the input check (plans with n = 0 or m = 0)
    int32_t* errs = nullptr;     // per sort tile: 1 if the tile holds an invalid input
    int32_t n_errs = 0;
    int64_t geom_bytes = 0;
    Geometry fwd, adj;
    // Partitions by order: forward and transposed, built on first use and kept
    // (the gradient runs orders nu - 1 and nu + 1 on the same sorted geometry).
    struct OrderParts {
        int nu = 0;
        uint64_t used = 0;
        Partition f, a;
    };
    std::vector<std::unique_ptr<OrderParts>> orders;
    uint64_t clock = 0;
    DevBuf b_grad;               // gradient temporaries (two of n, two of m)
    double* grad_t[4] = {nullptr, nullptr, nullptr, nullptr};
    // stage timing (diagnostics): kStages + 1 event slots per profiled call,
    // the boundaries of the stages in prof_mask filled
    bool prof = false;
    uint32_t prof_mask = 0;
    std::vector<hipEvent_t> prof_events;
    int64_t prof_calls = 0;
};

static void prof_clear(nuht_plan_t p)
{
    for (hipEvent_t e : p->prof_events)
        if (e) (void)hipEventDestroy(e);
    p->prof_events.clear();
    p->prof_calls = 0;
}

// Events for one profiled execute call, or null when profiling is off.
static hipEvent_t* prof_marks(nuht_plan_t p)
{
    if (!p->prof) return nullptr;
    size_t base = p->prof_events.size();
    for (int i = 0; i <= kStages; ++i) {
        hipEvent_t e = nullptr;
        const bool used = (i < kStages && ((p->prof_mask >> i) & 1)) || (i > 0 && ((p->prof_mask >> (i - 1)) & 1));
        if (used && hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            p->prof_events.resize(base);
            return nullptr;
        }
        p->prof_events.push_back(e);
    }
    p->prof_calls++;
    return p->prof_events.data() + base;
}

#define HIP_TRY(x)                                   \
    do {                                             \
        hipError_t e_ = (x);                         \
        if (e_ != hipSuccess) { (void)hipGetLastError(); return NUHT_EHIP; } \
    } while (0)

#define NUHT_TRY(x)                                  \
    do {                                             \
        int r_ = (x);                                \
        if (r_ != NUHT_OK) return r_;                \
    } while (0)

// Channel counts the spreading and row kernels are instantiated for: every
// even count up to 16, then multiples of 4 up to 40.  2M is padded up to the
// next instance; padding channels carry a zero factor.
static int padded_channels(int nch)
{
    return nch <= 16 ? nch : ((nch + 3) / 4) * 4;
}

// The tolerance the expansion orders and the NUFFT width are chosen for: the
// requested eps, or eps / margin when the caller asks for a margin (the
// paper's choice bounds every matrix entry by eps, which leaves the normwise
// maximum of the output error at up to ~1.3 eps at high orders).
static double design_eps(double eps, const nuht_opts& o)
{
    return o.margin > 1.0 ? eps / o.margin : eps;
}

// nu2 = 2 nu: even for integer orders (any sign), odd (>= 1) for nu = n + 1/2.
// Returns NUHT_ENOMEM if the half-integer table could not be made.
static int fill_params(PlanDev& P, int nu2, double eps_req, const nuht_opts& o)
{
    const bool half = (nu2 & 1) != 0;
    const int anu = half ? (nu2 - 1) / 2 : std::abs(nu2 / 2);
    const double nu = half ? anu + 0.5 : (double)anu;
    P.nu = anu;
    P.half = half ? 1 : 0;
    P.sign = (!half && nu2 < 0 && (anu & 1)) ? -1 : 1;
    P.eps = eps_req;
    const double eps = design_eps(eps_req, o);
    int M = o.M_override > 0 ? std::min(o.M_override, 20) : num_asy_terms(nu, eps);
    if (half && o.M_override <= 0) M = std::min(M, (anu + 2) / 2);
    P.M = M;
    P.nch = padded_channels(2 * M);
    if (half) {
        P.z = half_crossover(nu, eps, M);
        P.L = o.local_rank > 0 ? o.local_rank : half_local_rank(anu, eps, P.z);
        if (P.L >= 0) {
            int np = 0, ns = 0;
            P.half_tab = half_table_device(anu, P.L, P.z, &np, &ns);
            if (!P.half_tab) return NUHT_ENOMEM;
            P.half_np = np;
            P.half_ns = ns;
            P.half_inv_h = 1.0 / kHalfWidth;
        }
    } else {
        P.z = crossover(anu, eps, M);
        P.L = local_rank(anu, eps, P.z);
        if (o.local_rank > 0) P.L = o.local_rank;
        else if (o.local_rank == -1 && P.L >= 0) P.L = local_rank_tail(anu, eps, P.z, P.L);
    }
    P.w = es_width(eps, o.precision);
    P.fp32 = o.precision == NUHT_FP32_SPREAD ? 1 : 0;
    P.mfma = (!P.fp32 && P.w <= 16 && P.nch <= kMfmaMaxChannels && !o.vector_spread) ? 1 : 0;
    P.beta = es_beta(P.w);
    for (int p = 0; p < 2 * M + 2; ++p) P.hank[p] = hankel_coef(nu, p);
    for (int p = 0; p < kMaxChannels; ++p)
        P.chan[p] = p < 2 * M ? (((p >> 1) & 1) ? -P.hank[p] : P.hank[p]) : 0.0;
    phase_offset2(half ? nu2 + 1 : 2 * anu + 1, P.phi_hi, P.phi_lo);
    P.kappa_max = P.w * M_PI / 4.0 * (1.0 + 1e-9);
    P.eshat_s = 2.0 / (P.kappa_max * P.kappa_max);
    P.spread_chunk = o.spread_chunk > 0 ? o.spread_chunk : kSpreadChunk;
    // the polynomial depends only on the kernel width (beta follows w); at
    // kEshatTerms = 16 terms it is within about 1e-14 of ES^, relative, for
    // every width up to kMaxEsWidth
    static std::mutex mu;
    static double cache[32][kEshatTerms];
    static bool have[32] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (!have[P.w]) {
        eshat_poly(P.beta, P.kappa_max, cache[P.w]);
        have[P.w] = true;
    }
    for (int i = 0; i < kEshatTerms; ++i) P.eshat[i] = cache[P.w][i];
    return NUHT_OK;
}

// The direct-block J_nu table of P: panels of width kJtabWidth covering
// [0.8 z - 8, 1.2 z + 8] rounded out to multiples of 32 (a direct block holds
// entries on both sides of z, and at the finest subdivision level its entries
// lie within a few percent of z; the rounding lets plans of nearby z share a
// table); half-integer orders start at x = 8 or above, away from the branch
// point of J at 0.
static int direct_table(PlanDev& P)
{
    constexpr double q = 32.0;
    double lo = std::max(0.0, std::floor((0.8 * P.z - 8.0) / q) * q);
    if (P.half) lo = std::max(lo, 8.0);
    const double hi = std::ceil((1.2 * P.z + 8.0) / q) * q;
    P.jtab_x0 = lo;
    P.jtab_np = hi > lo ? (int32_t)((hi - lo) / kJtabWidth) : 0;
    P.jtab = nullptr;
    if (P.jtab_np == 0) return NUHT_OK;
    P.jtab = jtab_device(P.half ? 2 * P.nu + 1 : 2 * P.nu, lo, P.jtab_np);
    return P.jtab ? NUHT_OK : NUHT_ENOMEM;
}

// Building a partition takes two steps around one host synchronisation:
// part_begin fills the parameters, allocates the planning tables (with the
// current capacity guesses), launches the planning kernels and queues the copy
// of the summary and the input-check flag into a pinned slot; after the caller
// has synchronised, part_finish reads the slot and either asks for another
// attempt with larger tables or allocates the execution buffers.
struct PendingPart {
    Partition* Pt = nullptr;
    const Geometry* G = nullptr;
    hipStream_t s = nullptr;
    int32_t cap = 0, icap = 0;
    int attempt = 0;
    Arena A{};
    Partition tmp;   // the current attempt's tables
    PendingPart() = default;
    PendingPart(const PendingPart&) = delete;
    PendingPart& operator=(const PendingPart&) = delete;
};

static int part_begin(nuht_plan_t pl, PendingPart& pp, Partition& Pt, const Geometry& G, int nu, hipStream_t s,
                      HostStage* h, bool first)
{
    PlanDev& P = Pt.P;
    if (first) {
        Pt.release();
        Pt.stream = s;
        P = PlanDev{};
        NUHT_TRY(fill_params(P, nu, pl->eps, pl->opts));
        if (P.L < 0) return NUHT_EINVAL;
        NUHT_TRY(direct_table(P));
        P.n = G.n; P.m = G.m;
        P.rs = G.rs; P.ws = G.ws; P.perm_r = G.perm_r; P.perm_w = G.perm_w;
        Pt.sum = Summary{};
        pp.tmp.release();
        pp.attempt = 0;
        pp.Pt = &Pt; pp.G = &G; pp.s = s;
        int64_t tot = (int64_t)G.n + G.m;
        pp.cap = (int32_t)std::min<int64_t>(tot / 32 + 4096, 1 << 28);
        pp.icap = (int32_t)std::min<int64_t>(64 * (tot / P.spread_chunk) + 2 * (int64_t)pp.cap, 1 << 28);
    }
    if (G.n == 0 || G.m == 0) {
        if (pl->n_errs > 0) {
            HIP_TRY(launch_reduce_errs(pl->errs, pl->n_errs, pl->d_flag, s));
            HIP_TRY(hipMemcpyAsync(&h->flag, pl->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        } else {
            h->flag = 0;
        }
        return NUHT_OK;
    }
    const nuht_opts& o = pl->opts;
    int64_t min_size = o.min_size > 0 ? o.min_size : default_min_size(G.n, G.m);
    // -1: every row of a block is a candidate (the exact split optimum)
    int ncand = o.split_candidates == -1 ? INT32_MAX : (o.split_candidates > 1 ? o.split_candidates : 16);
    int dft_max = o.dft_max == 0 ? 48 : o.dft_max;
    const double sigma = 2.0;
    pp.tmp.release();
    pp.tmp.stream = s;
    Arena& A = pp.A;
    A = Arena{};
    A.node_cap = pp.cap; A.l_cap = pp.cap; A.a_cap = pp.cap; A.d_cap = 2 * pp.cap; A.q_cap = pp.cap;
    A.litem_cap = pp.icap; A.aitem_cap = pp.icap;
    int32_t *K = nullptr, *Jc = nullptr, *a_cells = nullptr;
    Slab slab;
    slab.add(K, (size_t)G.m);
    slab.add(Jc, (size_t)G.n);
    slab.add(a_cells, (size_t)A.aitem_cap);
    slab.add(A.nodes, (size_t)A.node_cap);
    slab.add(A.lb, (size_t)A.l_cap);
    slab.add(A.ab, (size_t)A.a_cap);
    slab.add(A.db, (size_t)A.d_cap);
    slab.add(A.q0, (size_t)A.q_cap);
    slab.add(A.q1, (size_t)A.q_cap);
    slab.add(A.litems, (size_t)A.litem_cap);
    slab.add(A.aitems, (size_t)A.aitem_cap);
    slab.add(A.alist, (size_t)A.aitem_cap);
    slab.add(A.fft_list, (size_t)A.a_cap);
    slab.add(A.gslot, (size_t)A.a_cap + 1);
    NUHT_TRY(slab.commit(pp.tmp));
    P.nodes = A.nodes; P.lb = A.lb; P.ab = A.ab; P.db = A.db;
    P.litems = A.litems; P.aitems = A.aitems; P.alist = A.alist; P.fft_list = A.fft_list; P.gslot = A.gslot;
    HIP_TRY(launch_planning(P, A, K, Jc, a_cells, min_size, ncand, dft_max, sigma, pl->d_sum, pl->errs, pl->n_errs,
                            s));
    HIP_TRY(hipMemcpyAsync(&h->sum, pl->d_sum, sizeof(Summary), hipMemcpyDeviceToHost, s));
    return NUHT_OK;
}

// After the synchronisation.  *again is set when the tables overflowed and
// part_begin must run once more (with first = false).
static int part_finish(PendingPart& pp, const HostStage* h, bool* again)
{
    *again = false;
    Partition& Pt = *pp.Pt;
    const Geometry& G = *pp.G;
    PlanDev& P = Pt.P;
    if (G.n == 0 || G.m == 0) {
        if (h->flag) return NUHT_EDOMAIN;
        Pt.built = true;
        return NUHT_OK;
    }
    if (h->sum.domain_error) return NUHT_EDOMAIN;
    Summary& S = Pt.sum;
    S = h->sum;
    if (S.overflow == 2) return NUHT_ECAPACITY;   // subdivision deeper than kMaxLevels
    if (S.grid_error) return NUHT_ECAPACITY;
    if (S.overflow) {
        if (++pp.attempt >= 6) return NUHT_ECAPACITY;
        int64_t need = std::max<int64_t>({(int64_t)S.n_nodes, (int64_t)S.n_l, (int64_t)S.n_a, (int64_t)S.n_d / 2});
        if (need >= pp.cap) pp.cap = (int32_t)std::min<int64_t>(2 * need + 1024, 1 << 29);
        int64_t ineed = std::max<int64_t>((int64_t)S.n_litems, (int64_t)S.n_aitems);
        if (ineed >= pp.icap) pp.icap = (int32_t)std::min<int64_t>(2 * ineed + 1024, 1 << 29);
        if (need < pp.cap && ineed < pp.icap) { pp.cap *= 2; pp.icap *= 2; }
        *again = true;
        return NUHT_OK;
    }
    // keep this attempt's tables
    for (auto& b : pp.tmp.bufs) Pt.bufs.push_back(b);
    Pt.bytes += pp.tmp.bytes;
    pp.tmp.bufs.clear();
    pp.tmp.bytes = 0;
    Pt.A = pp.A;
    P.n_nodes = S.n_nodes; P.n_l = S.n_l; P.n_a = S.n_a; P.n_d = S.n_d;
    P.n_litems = S.n_litems; P.n_aitems = S.n_aitems; P.n_adense = S.n_adense; P.n_amed = S.n_amed;

    // execution buffers
    ExecBuffers& B = Pt.B;
    Slab slab;
    slab.add(B.cs, (size_t)G.n);
    slab.add(B.lpart, (size_t)S.n_litems * (P.L + 1));
    slab.add(B.lmom, (size_t)S.n_l * (P.L + 1));
    slab.add(B.part, (size_t)S.part_cells * P.nch);
    slab.add(B.grids, (size_t)S.grid_cells * P.nch);
    slab.add(B.gd, (size_t)G.m);
    slab.add(B.ga, (size_t)G.m);
    B.grid_cells = S.grid_cells;
    int64_t scratch = 0;
    for (int c = 6; c <= kMaxFftLog2; ++c) {
        if (S.fft_count[c] == 0) continue;
        FftClass fc;
        fc.log2n = c; fc.count = S.fft_count[c]; fc.first = S.fft_first[c];
        fc.scratch_off = scratch;
        if (c > 12) scratch += (int64_t)fc.count * P.nch << c;
        Pt.cls.push_back(fc);
    }
    slab.add(B.scratch, (size_t)scratch);
    NUHT_TRY(slab.commit(Pt));
    B.es_poly = es_pieces_device(P.w, P.beta);
    if (!B.es_poly) return NUHT_ENOMEM;
    B.fft_tw = fft_twiddles_device();
    if (!B.fft_tw) return NUHT_ENOMEM;
    P.es_poly = B.es_poly;
    P.cs = B.cs; P.lpart = B.lpart; P.lmom = B.lmom; P.part = B.part; P.grids = B.grids;
    P.scratch = B.scratch; P.gd = B.gd; P.ga = B.ga; P.fft_tw = B.fft_tw;
    P.grid_cells = B.grid_cells;
    small_fft_table(P, Pt.cls.data(), (int)Pt.cls.size());
    Pt.built = true;
    return NUHT_OK;
}

// Both steps with the process-wide pinned slot; synchronises `s` once per
// attempt (once unless the capacity guesses were too small).
static int build_partition(nuht_plan_t pl, Partition& Pt, const Geometry& G, int nu, hipStream_t s)
{
    PendingPart pp;
    bool first = true;
    for (;;) {
        std::unique_lock<std::mutex> lock;
        HostStage* h = host_stage(lock);
        if (!h) return NUHT_ENOMEM;
        NUHT_TRY(part_begin(pl, pp, Pt, G, nu, s, h, first));
        first = false;
        HIP_TRY(hipStreamSynchronize(s));
        bool again = false;
        NUHT_TRY(part_finish(pp, h, &again));
        if (!again) return NUHT_OK;
    }
}

// Frees on the plan stream happen after the last use on a caller stream.
static void before_free(nuht_plan_t p)
{
    if (p->used && p->ps && p->ev_use) (void)hipStreamWaitEvent(p->ps, p->ev_use, 0);
}

static void note_use(nuht_plan_t p, hipStream_t s)
{
    if (p->ev_use && hipEventRecord(p->ev_use, s) == hipSuccess) p->used = true;
    else (void)hipGetLastError();
}

static hipStream_t plan_stream();

// Memory of released plans: kept with the events that mark its last uses
// (the last execution on a caller stream, the work queued on the planning
// stream) and, once both have completed, put in the block cache (or freed on
// the library's planning stream).  Releasing a plan therefore never makes the
// planning stream wait for an execution, and the next plan reuses the memory
// without an allocation call.  Completion is checked whenever a plan is made
// or released.
struct Retired {
    int dev = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<DevBuf> bufs;
};

static std::mutex retired_mu;
static std::vector<Retired> retired;

static void reap_retired()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { (void)hipGetLastError(); return; }
    hipStream_t ls = plan_stream();
    std::lock_guard<std::mutex> lock(retired_mu);
    for (size_t i = 0; i < retired.size();) {
        Retired& r = retired[i];
        // anything but "not ready" ends a wait (an error leaves nothing to protect)
        bool done = r.dev == dev;
        for (hipEvent_t e : r.ev)
            if (done && e && hipEventQuery(e) == hipErrorNotReady) done = false;
        (void)hipGetLastError();
        if (!done) { ++i; continue; }
        for (DevBuf& b : r.bufs) {
            if (!b.p || block_put(r.dev, b.p, b.bytes)) continue;
            if (b.stream || device_pool()) (void)hipFreeAsync(b.p, ls);
            else (void)hipFree(b.p);
        }
        for (hipEvent_t e : r.ev)
            if (e) (void)hipEventDestroy(e);
        retired[i] = std::move(retired.back());
        retired.pop_back();
    }
    (void)hipGetLastError();
}

static void free_plan(nuht_plan_t p)
{
    if (!p) return;
    prof_clear(p);
    Retired r;
    bool retire = hipGetDevice(&r.dev) == hipSuccess && plan_stream() != nullptr;
    if (retire && p->ps) {
        // the planning stream's queued work (none after a completed plan, but a
        // plan that failed midway may leave some)
        if (p->ev_plan && hipEventRecord(p->ev_plan, p->ps) == hipSuccess) {
            r.ev[0] = p->ev_plan;
            p->ev_plan = nullptr;
        } else if (hipStreamSynchronize(p->ps) != hipSuccess) {
            retire = false;
        }
    }
    (void)hipGetLastError();
    if (retire) {
        if (p->used && p->ev_use) {
            r.ev[1] = p->ev_use;
            p->ev_use = nullptr;
        }
        for (auto& o : p->orders) {
            o->f.take_bufs(r.bufs);
            o->a.take_bufs(r.bufs);
        }
        for (DevBuf* b : {&p->b_grad, &p->b_geom}) {
            if (b->p) r.bufs.push_back(*b);
            *b = DevBuf{};
        }
        p->orders.clear();
        if (p->ev_use) (void)hipEventDestroy(p->ev_use);
        if (p->ev_plan) (void)hipEventDestroy(p->ev_plan);
        if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
        if (p->ev_join) (void)hipEventDestroy(p->ev_join);
        delete p;
        {
            std::lock_guard<std::mutex> lock(retired_mu);
            retired.push_back(std::move(r));
        }
        reap_retired();
        return;
    }
    before_free(p);
    p->orders.clear();
    dev_free(p->b_grad);
    dev_free(p->b_geom);
    if (p->ev_use) (void)hipEventDestroy(p->ev_use);
    if (p->ev_plan) (void)hipEventDestroy(p->ev_plan);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    delete p;
    reap_retired();
}

// The library's planning stream of the current device (default priority).
static hipStream_t plan_stream()
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) { (void)hipGetLastError(); return nullptr; }
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        streams[dev] = nullptr;
    }
    return streams[dev];
}

// The library's side stream for executions (per device, default priority):
// the local moments and direct blocks of an execution run there, beside the
// spreading chain on the caller's stream.  Made when a plan is made
// (create), only looked up by executions, which allocate nothing.
static hipStream_t exec_side_stream(bool create)
{
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) { (void)hipGetLastError(); return nullptr; }
    std::lock_guard<std::mutex> lock(mu);
    if (create && !streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        streams[dev] = nullptr;
    }
    return streams[dev];
}

// At most this many orders keep their partitions; the least recently used
// other order is dropped to make room.
constexpr size_t kMaxOrders = 4;

static nuht_plan_s::OrderParts* order_parts(nuht_plan_t p, int nu)
{
    for (auto& o : p->orders)
        if (o->nu == nu) { o->used = ++p->clock; return o.get(); }
    if (p->orders.size() >= kMaxOrders) {
        size_t victim = p->orders.size();
        for (size_t i = 0; i < p->orders.size(); ++i)
            if (p->orders[i]->nu != p->nu2_req &&
                (victim == p->orders.size() || p->orders[i]->used < p->orders[victim]->used))
                victim = i;
        if (victim < p->orders.size()) {
            before_free(p);
            p->orders.erase(p->orders.begin() + victim);
        }
    }
    auto o = std::unique_ptr<nuht_plan_s::OrderParts>(new (std::nothrow) nuht_plan_s::OrderParts());
    if (!o) return nullptr;
    o->nu = nu;
    o->used = ++p->clock;
    p->orders.push_back(std::move(o));
    return p->orders.back().get();
}

// The partition of order nu, forward (A) or transposed (A^T), built if needed
// (building synchronises `s` once).
static int get_partition(nuht_plan_t p, int nu, bool transposed, hipStream_t s, Partition** out)
{
    nuht_plan_s::OrderParts* o = order_parts(p, nu);
    if (!o) return NUHT_ENOMEM;
    Partition& Pt = transposed ? o->a : o->f;
    if (!Pt.built) {
        (void)s;
        int rc = build_partition(p, Pt, transposed ? p->adj : p->fwd, nu, p->ps);
        if (rc != NUHT_OK) {
            Pt.release();
            return rc;
        }
    }
    *out = &Pt;
    return NUHT_OK;
}

static const Partition* current_forward(nuht_plan_t p)
{
    for (auto& o : p->orders)
        if (o->nu == p->nu2_req && o->f.built) return &o->f;
    return nullptr;
}

static int run(nuht_plan_t p, const Partition& Pt, const double* in, double* out, bool scale, hipStream_t s)
{
    IoArgs io;
    io.c = in;
    io.g = out;
    io.scale_by_points = scale;
    // The fork needs the plan's events and the side stream; it is left out
    // while `s` is being captured into a graph (the capture stays one stream)
    // and while the local moments, direct blocks or local rows are timed
    // (their intervals are taken on `s`).
    ExecFork fork;
    const ExecFork* fk = nullptr;
    constexpr uint32_t kSerialStages = (1u << 1) | (1u << 5) | (1u << 7);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) {
        (void)hipGetLastError();
        cap = hipStreamCaptureStatusActive;
    }
    if (p->ev_fork && p->ev_join && cap == hipStreamCaptureStatusNone && !(p->prof && (p->prof_mask & kSerialStages))) {
        fork.side = exec_side_stream(false);
        fork.ev_fork = p->ev_fork;
        fork.ev_join = p->ev_join;
        if (fork.side) fk = &fork;
    }
    HIP_TRY(launch_execute(Pt.P, Pt.sum, Pt.B, Pt.cls.data(), (int)Pt.cls.size(), io, s, prof_marks(p), fk));
    note_use(p, s);
    return NUHT_OK;
}

static bool valid_eps(double eps) { return eps >= 1e-15 && eps <= 1e-2; }

static bool valid_common(int nu, double eps) { return nu >= -100 && nu <= 100 && valid_eps(eps); }

// An order given as twice its value: integers |nu| <= 100, half-integers
// 1/2 <= nu <= 199/2.
static bool valid_order2(int nu2)
{
    if (nu2 & 1) return nu2 >= 1 && nu2 <= 199;
    return nu2 >= -200 && nu2 <= 200;
}

extern "C" {

const char* nuht_strerror(int code)
{
    switch (code) {
        case NUHT_OK: return "success";
        case NUHT_EINVAL: return "invalid argument";
        case NUHT_EDOMAIN: return "a point or frequency is negative, NaN or infinite";
        case NUHT_EPRECISION: return "FP32 spreading needs eps >= 1e-7";
        case NUHT_ENOMEM: return "device allocation failed";
        case NUHT_EHIP: return "HIP runtime error";
        case NUHT_ECAPACITY: return "partition exceeds internal table limits";
        case NUHT_ENOTREADY: return "a partition the call needs has not been built";
        default: return "unknown error";
    }
}

// Validated options of a plan call.
static int check_opts(const nuht_opts* opts, nuht_opts& o)
{
    o = nuht_opts{};
    if (opts) o = *opts;
    if (o.precision != NUHT_FP64 && o.precision != NUHT_FP32_SPREAD) return NUHT_EINVAL;

    if (o.min_size < 0 || o.M_override < 0 || o.M_override > 20 || o.split_candidates < -1 || o.local_rank < -1 ||
        o.local_rank > 2000)
        return NUHT_EINVAL;
    if (o.spread_chunk != 0 && (o.spread_chunk < 64 || o.spread_chunk > 16384)) return NUHT_EINVAL;
    if (o.margin != 0.0 && !(o.margin >= 1.0 && o.margin <= 1e3)) return NUHT_EINVAL;
    return NUHT_OK;
}

// Host-side checks of one plan's arguments (no HIP call).
static int check_plan_args(int nu2, double eps, int64_t n, const double* r_dev, int64_t m,
                           const double* omega_dev, const nuht_opts& o)
{
    if (!valid_order2(nu2) || !valid_eps(eps)) return NUHT_EINVAL;
    if (design_eps(eps, o) < 1e-15) return NUHT_EINVAL;
    if (o.precision == NUHT_FP32_SPREAD && design_eps(eps, o) < 1e-7) return NUHT_EPRECISION;
    if (n < 0 || m < 0 || n > INT32_MAX / 2 || m > INT32_MAX / 2) return NUHT_EINVAL;
    if ((n > 0 && !r_dev) || (m > 0 && !omega_dev)) return NUHT_EINVAL;
    return NUHT_OK;
}

// A plan with its geometry: storage allocated, input check and sort launched
// on `s` (no partition yet, no synchronisation).
// s: the stream the plan works on (its planning stream); wait_on, if set, is
// the caller's stream, after whose queued work the inputs are read.
static int plan_create(nuht_plan_t* out, int nu2, double eps, int64_t n, const double* r_dev, int64_t m,
                       const double* omega_dev, const nuht_opts& o, hipStream_t s, hipStream_t wait_on)
{
    *out = nullptr;
    NUHT_TRY(check_plan_args(nu2, eps, n, r_dev, m, omega_dev, o));
    reap_retired();
    nuht_plan_s* p = new (std::nothrow) nuht_plan_s();
    if (!p) return NUHT_ENOMEM;
    p->nu2_req = nu2; p->eps = eps; p->opts = o; p->n = n; p->m = m;
    if (o.tune_cache) p->cache_path = o.tune_cache;
    p->opts.tune_cache = nullptr;
    p->ps = s;
    int64_t tot = n + m;
    auto fail = [&](int code) { free_plan(p); return code; };
    if (hipEventCreateWithFlags(&p->ev_use, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        p->ev_use = nullptr;
        return fail(NUHT_EHIP);
    }
    if (hipEventCreateWithFlags(&p->ev_plan, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        p->ev_plan = nullptr;
        return fail(NUHT_EHIP);
    }
    // the fork events and side stream are optional: without them executions
    // stay on one stream
    if (hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess || !exec_side_stream(true)) {
        (void)hipGetLastError();
        if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
        if (p->ev_join) (void)hipEventDestroy(p->ev_join);
        p->ev_fork = p->ev_join = nullptr;
    }
    if (wait_on) {
        if (hipEventRecord(p->ev_use, wait_on) != hipSuccess) return fail(NUHT_EHIP);
        if (hipStreamWaitEvent(s, p->ev_use, 0) != hipSuccess) return fail(NUHT_EHIP);
    }
    {
        Slab slab;
        slab.add(p->d_sum, 1);
        slab.add(p->d_flag, 1);
        p->n_errs = sort_tiles((int32_t)n, (int32_t)m);
        slab.add(p->errs, (size_t)p->n_errs);
        if (tot > 0) {
            slab.add(p->keys, (size_t)tot);
            slab.add(p->vals, (size_t)tot);
            slab.add(p->keys2, (size_t)tot);
            slab.add(p->vals2, (size_t)tot);
            slab.add(p->hist, (size_t)sort_hist_len((int32_t)n, (int32_t)m));
        }
        if (slab.commit(p->b_geom, s) != NUHT_OK) return fail(NUHT_ENOMEM);
        p->geom_bytes = (int64_t)p->b_geom.bytes;
    }
    if (launch_keys_and_sort(r_dev, (int32_t)n, omega_dev, (int32_t)m, p->keys, p->vals, p->keys2, p->vals2, p->hist,
                             p->errs, s) != hipSuccess)
        return fail(NUHT_EHIP);
    p->fwd.n = (int32_t)n; p->fwd.m = (int32_t)m;
    p->fwd.rs = (const double*)p->keys;
    p->fwd.ws = (const double*)(p->keys + n);
    p->fwd.perm_r = p->vals;
    p->fwd.perm_w = p->vals + n;
    p->adj.n = (int32_t)m; p->adj.m = (int32_t)n;
    p->adj.rs = p->fwd.ws; p->adj.ws = p->fwd.rs;
    p->adj.perm_r = p->fwd.perm_w; p->adj.perm_w = p->fwd.perm_r;
    *out = p;
    return NUHT_OK;
}

int nuht_plan_half(nuht_plan_t* out, int nu2, double eps, int64_t n, const double* r_dev, int64_t m,
                   const double* omega_dev, const nuht_opts* opts, void* stream)
{
    if (!out) return NUHT_EINVAL;
    *out = nullptr;
    nuht_opts o;
    NUHT_TRY(check_opts(opts, o));
    NUHT_TRY(check_plan_args(nu2, eps, n, r_dev, m, omega_dev, o));
    hipStream_t s = (hipStream_t)stream;
    hipStream_t ps = plan_stream();
    if (!ps) return NUHT_EHIP;
    nuht_plan_t p = nullptr;
    NUHT_TRY(plan_create(&p, nu2, eps, n, r_dev, m, omega_dev, o, ps, s));
    // the one synchronisation of the plan happens inside (it also reads the
    // input check's flag)
    Partition* Pt = nullptr;
    int rc = get_partition(p, nu2, false, s, &Pt);
    if (rc != NUHT_OK) {
        free_plan(p);
        return rc;
    }
    *out = p;
    return NUHT_OK;
}

int nuht_plan(nuht_plan_t* out, int nu, double eps, int64_t n, const double* r_dev, int64_t m,
              const double* omega_dev, const nuht_opts* opts, void* stream)
{
    if (!out) return NUHT_EINVAL;
    *out = nullptr;
    if (nu < -100 || nu > 100) return NUHT_EINVAL;
    return nuht_plan_half(out, 2 * nu, eps, n, r_dev, m, omega_dev, opts, stream);
}

int nuht_execute(nuht_plan_t p, const double* c_dev, double* g_dev, void* stream)
{
    if (!p) return NUHT_EINVAL;
    const Partition* Pt = current_forward(p);
    if (!Pt) return NUHT_EINVAL;
    if ((p->n > 0 && !c_dev) || (p->m > 0 && !g_dev)) return NUHT_EINVAL;
    return run(p, *Pt, c_dev, g_dev, false, (hipStream_t)stream);
}

int nuht_adjoint(nuht_plan_t p, const double* y_dev, double* cbar_dev, void* stream)
{
    if (!p || !current_forward(p)) return NUHT_EINVAL;
    if ((p->m > 0 && !y_dev) || (p->n > 0 && !cbar_dev)) return NUHT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Partition* Pt = nullptr;
    int rc = get_partition(p, p->nu2_req, true, s, &Pt);
    if (rc != NUHT_OK) return rc;
    return run(p, *Pt, y_dev, cbar_dev, false, s);
}

int nuht_gradient(nuht_plan_t p, const double* c_dev, const double* gbar_dev, double* dc_dev, double* dr_dev,
                  double* domega_dev, void* stream)
{
    if (!p || !current_forward(p)) return NUHT_EINVAL;
    const bool want_r = dr_dev != nullptr, want_w = domega_dev != nullptr;
    if (p->m > 0 && !gbar_dev) return NUHT_EINVAL;
    if ((want_r || want_w) && p->n > 0 && !c_dev) return NUHT_EINVAL;
    const int nu = p->nu2_req;       // twice the order; orders nu -+ 1 are nu -+ 2 here
    if ((want_r || want_w) && !(valid_order2(nu - 2) && valid_order2(nu + 2))) return NUHT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if ((want_r || want_w) && !p->b_grad.p && p->n + p->m > 0) {
        Slab slab;
        slab.add(p->grad_t[0], (size_t)p->n);
        slab.add(p->grad_t[1], (size_t)p->n);
        slab.add(p->grad_t[2], (size_t)p->m);
        slab.add(p->grad_t[3], (size_t)p->m);
        if (slab.commit(p->b_grad, s) != NUHT_OK) return NUHT_ENOMEM;
    }
    Partition* Pt = nullptr;
    int rc;
    if (dc_dev) {                        // dL/dc = A^T gbar
        if ((rc = get_partition(p, nu, true, s, &Pt)) != NUHT_OK) return rc;
        if ((rc = run(p, *Pt, gbar_dev, dc_dev, false, s)) != NUHT_OK) return rc;
    }
    if (want_r && p->n > 0) {            // dL/dr = (c/2) (A_{nu-1}^T - A_{nu+1}^T)(omega gbar)
        if ((rc = get_partition(p, nu - 2, true, s, &Pt)) != NUHT_OK) return rc;
        if ((rc = run(p, *Pt, gbar_dev, p->grad_t[0], true, s)) != NUHT_OK) return rc;
        if ((rc = get_partition(p, nu + 2, true, s, &Pt)) != NUHT_OK) return rc;
        if ((rc = run(p, *Pt, gbar_dev, p->grad_t[1], true, s)) != NUHT_OK) return rc;
        HIP_TRY(launch_half_difference(c_dev, p->grad_t[0], p->grad_t[1], dr_dev, (int32_t)p->n, s));
    }
    if (want_w && p->m > 0) {            // dL/domega = (gbar/2) (A_{nu-1} - A_{nu+1})(r c)
        if ((rc = get_partition(p, nu - 2, false, s, &Pt)) != NUHT_OK) return rc;
        if ((rc = run(p, *Pt, c_dev, p->grad_t[2], true, s)) != NUHT_OK) return rc;
        if ((rc = get_partition(p, nu + 2, false, s, &Pt)) != NUHT_OK) return rc;
        if ((rc = run(p, *Pt, c_dev, p->grad_t[3], true, s)) != NUHT_OK) return rc;
        HIP_TRY(launch_half_difference(gbar_dev, p->grad_t[2], p->grad_t[3], domega_dev, (int32_t)p->m, s));
    }
    return NUHT_OK;
}

// ---------------------------------------------------------------------------
// The gradient without allocation: its four temporaries (two of n, two of m
// doubles) live in `scratch`, one array per device for the whole process,
// instead of the plan's own buffer.  Host code never passes the array's name
// to a kernel (in host code it is only a stand-in for the symbol); it uses the
// device address hipGetSymbolAddress returns, looked up once per device.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocDoubles = size_t(8) << 20;     // 64 MiB: n + m <= 4 194 304

static __device__ __align__(256) __attribute__((used)) double scratch[kNoAllocDoubles];

// Device address of this device's copy of `scratch`, or null on failure.
static double* scratch_address()
{
    static std::mutex mu;
    static double* addr[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) { (void)hipGetLastError(); return nullptr; }
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        addr[dev] = (double*)ptr;
    }
    return addr[dev];
}

// The partition of order nu (forward or transposed) if it is already built;
// never builds one.
static const Partition* built_partition(nuht_plan_t p, int nu, bool transposed)
{
    for (auto& o : p->orders) {
        if (o->nu != nu) continue;
        const Partition& Pt = transposed ? o->a : o->f;
        return Pt.built ? &Pt : nullptr;
    }
    return nullptr;
}

int nuht_gradient_noalloc(nuht_plan_t p, const double* c_dev, const double* gbar_dev, double* dc_dev,
                          double* dr_dev, double* domega_dev, void* stream)
{
    if (!p || !current_forward(p)) return NUHT_EINVAL;
    const bool want_r = dr_dev != nullptr, want_w = domega_dev != nullptr;
    if (p->m > 0 && !gbar_dev) return NUHT_EINVAL;
    if ((want_r || want_w) && p->n > 0 && !c_dev) return NUHT_EINVAL;
    const int nu = p->nu2_req;       // twice the order
    if ((want_r || want_w) && !(valid_order2(nu - 2) && valid_order2(nu + 2))) return NUHT_EINVAL;
    if ((want_r || want_w) && 2 * (p->n + p->m) > (int64_t)kNoAllocDoubles) return NUHT_ECAPACITY;
    // every partition the call runs must exist already: building one allocates
    const Partition *pc = nullptr, *pr0 = nullptr, *pr1 = nullptr, *pw0 = nullptr, *pw1 = nullptr;
    if (dc_dev && !(pc = built_partition(p, nu, true))) return NUHT_ENOTREADY;
    if (want_r && p->n > 0) {
        if (!(pr0 = built_partition(p, nu - 2, true)) || !(pr1 = built_partition(p, nu + 2, true)))
            return NUHT_ENOTREADY;
    }
    if (want_w && p->m > 0) {
        if (!(pw0 = built_partition(p, nu - 2, false)) || !(pw1 = built_partition(p, nu + 2, false)))
            return NUHT_ENOTREADY;
    }
    double* t = (want_r || want_w) ? scratch_address() : nullptr;
    if ((want_r || want_w) && !t) return NUHT_EHIP;
    hipStream_t s = (hipStream_t)stream;
    auto go = [&](const Partition* Pt, const double* in, double* out, bool scale) -> int {
        IoArgs io;
        io.c = in;
        io.g = out;
        io.scale_by_points = scale;
        HIP_TRY(launch_execute(Pt->P, Pt->sum, Pt->B, Pt->cls.data(), (int)Pt->cls.size(), io, s, nullptr));
        return NUHT_OK;
    };
    if (pc) NUHT_TRY(go(pc, gbar_dev, dc_dev, false));
    if (pr0) {                           // t[0 .. n) and t[n .. 2n): the two transposed transforms
        NUHT_TRY(go(pr0, gbar_dev, t, true));
        NUHT_TRY(go(pr1, gbar_dev, t + p->n, true));
        HIP_TRY(launch_half_difference(c_dev, t, t + p->n, dr_dev, (int32_t)p->n, s));
    }
    if (pw0) {                           // t[2n .. 2n + m) and t[2n + m .. 2n + 2m)
        double* a = t + 2 * p->n;
        NUHT_TRY(go(pw0, c_dev, a, true));
        NUHT_TRY(go(pw1, c_dev, a + p->m, true));
        HIP_TRY(launch_half_difference(gbar_dev, a, a + p->m, domega_dev, (int32_t)p->m, s));
    }
    note_use(p, s);
    return NUHT_OK;
}

int nuht_plan_set_order(nuht_plan_t p, int nu, void* stream)
{
    if (!p) return NUHT_EINVAL;
    if (!valid_common(nu, p->eps)) return NUHT_EINVAL;
    const int prev = p->nu2_req;
    p->nu2_req = 2 * nu;
    Partition* Pt = nullptr;
    int rc = get_partition(p, 2 * nu, false, (hipStream_t)stream, &Pt);
    if (rc != NUHT_OK) p->nu2_req = prev;
    return rc;
}

// ---------------------------------------------------------------------------
// Autotuning: the spreading work-item size (points per item), the direct-block
// threshold min_size, the direct-sum/FFT threshold dft_max and the number of
// candidate rows of SplitIndices (unless the exact split was asked for), by
// coordinate descent over a few candidates each, every candidate planned on
// the plan's own sorted geometry and timed over `reps` executes (after one
// warm-up) with HIP events on `s`.
// ---------------------------------------------------------------------------
static int tune_plan(nuht_plan_t p, const double* c_dev, int reps, nuht_opts* best, double* best_ms, hipStream_t s)
{
    if (reps < 1) reps = 3;
    DevBuf ones, out;
    if (!c_dev && p->n > 0) {
        NUHT_TRY(dev_alloc(ones, sizeof(double) * (size_t)p->n, s));
        HIP_TRY(launch_fill((double*)ones.p, p->n, 1.0, s));
        c_dev = (const double*)ones.p;
    }
    if (p->m > 0) NUHT_TRY(dev_alloc(out, sizeof(double) * (size_t)p->m, s));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const nuht_opts saved = p->opts;
    nuht_opts cur = saved;
    if (cur.spread_chunk == 0) cur.spread_chunk = kSpreadChunk;
    if (cur.min_size == 0) cur.min_size = default_min_size(p->n, p->m);
    if (cur.dft_max == 0) cur.dft_max = 48;
    if (cur.split_candidates == 0) cur.split_candidates = 16;
    int rc = NUHT_OK;
    auto time_opts = [&](const nuht_opts& o, double* ms) -> int {
        p->opts = o;
        Partition T;
        int r = build_partition(p, T, p->fwd, p->nu2_req, p->ps);
        if (r != NUHT_OK) return r;
        IoArgs io;
        io.c = c_dev;
        io.g = (double*)out.p;
        HIP_TRY(launch_execute(T.P, T.sum, T.B, T.cls.data(), (int)T.cls.size(), io, s, nullptr));
        HIP_TRY(hipEventRecord(e0, s));
        for (int k = 0; k < reps; ++k)
            HIP_TRY(launch_execute(T.P, T.sum, T.B, T.cls.data(), (int)T.cls.size(), io, s, nullptr));
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        *ms = (double)t / reps;
        return NUHT_OK;
    };
    double cur_ms = 0.0;
    rc = time_opts(cur, &cur_ms);
    const int chunks[] = {512, 1024, 2048, 4096};
    const int64_t sizes[] = {1024, 4096, 8192, 32768};
    const int dfts[] = {24, 48, 96};
    const int splits[] = {8, 16, 32};
    const int nparam = cur.split_candidates == -1 ? 3 : 4;
    for (int param = 0; param < nparam && rc == NUHT_OK; ++param) {
        int ncand = (param == 0 || param == 1) ? 4 : 3;
        for (int q = 0; q < ncand && rc == NUHT_OK; ++q) {
            nuht_opts o = cur;
            if (param == 0) { if (o.spread_chunk == chunks[q]) continue; o.spread_chunk = chunks[q]; }
            if (param == 1) { if (o.min_size == sizes[q]) continue; o.min_size = sizes[q]; }
            if (param == 2) { if (o.dft_max == dfts[q]) continue; o.dft_max = dfts[q]; }
            if (param == 3) { if (o.split_candidates == splits[q]) continue; o.split_candidates = splits[q]; }
            double ms = 0.0;
            rc = time_opts(o, &ms);
            if (rc == NUHT_OK && ms < cur_ms) { cur = o; cur_ms = ms; }
        }
    }
    p->opts = saved;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dev_free(ones);
    dev_free(out);
    if (rc != NUHT_OK) return rc;
    cur.tune = 0;
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return NUHT_OK;
}

// ---------------------------------------------------------------------------
// The tuning cache: a JSON file of tuned options by key, so that a size class
// is timed once (the paper builds its parameter tables once, when the library
// is installed) and later plans and batches read the result.  The key is what
// the tuned options depend on: the size class floor(log10(n + m)), the channel
// count, the local rank, the ES width, the spreading precision and whether
// the split is exact.  One entry per line:
//   {"key": "...", "spread_chunk": 1024, "min_size": 1024, "dft_max": 48,
//    "split_candidates": 16, "ms": 0.93}
// The file is read whole and rewritten through a temporary file and a rename;
// an unreadable file counts as empty, and a failed write only loses the entry.
// ---------------------------------------------------------------------------
struct TuneEntry {
    std::string key;
    int64_t spread_chunk = 0, min_size = 0, dft_max = 0, split_candidates = 0;
    double ms = 0.0;
};

static std::mutex& cache_mutex()
{
    static std::mutex mu;
    return mu;
}

static std::string tune_key(const nuht_plan_s* p, const PlanDev& P)
{
    int cls = 0;
    for (int64_t t = p->n + p->m; t >= 10 && cls < 9; t /= 10) ++cls;
    char buf[160];
    std::snprintf(buf, sizeof buf, "v1 class %d nch %d L %d w %d fp32 %d exact %d%s", cls, P.nch, P.L, P.w, P.fp32,
                  p->opts.split_candidates == -1 ? 1 : 0, P.half ? " half" : "");
    return buf;
}

static std::vector<TuneEntry> cache_read(const std::string& path)
{
    std::vector<TuneEntry> out;
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f) return out;
    std::string text;
    char chunk[4096];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof chunk, f)) > 0) text.append(chunk, got);
    std::fclose(f);
    const std::string tag = "{\"key\": \"";
    for (size_t at = text.find(tag); at != std::string::npos; at = text.find(tag, at + 1)) {
        const size_t k0 = at + tag.size(), k1 = text.find('"', k0), end = text.find('}', k0);
        if (k1 == std::string::npos || end == std::string::npos || k1 > end) break;
        TuneEntry e;
        e.key = text.substr(k0, k1 - k0);
        auto num = [&](const char* name, double* v) {
            const std::string pat = std::string("\"") + name + "\": ";
            const size_t q = text.find(pat, k1);
            if (q == std::string::npos || q > end) return false;
            *v = std::strtod(text.c_str() + q + pat.size(), nullptr);
            return true;
        };
        double a, b, c, d, ms;
        if (num("spread_chunk", &a) && num("min_size", &b) && num("dft_max", &c) && num("split_candidates", &d) &&
            num("ms", &ms)) {
            e.spread_chunk = (int64_t)a; e.min_size = (int64_t)b; e.dft_max = (int64_t)c;
            e.split_candidates = (int64_t)d; e.ms = ms;
            out.push_back(e);
        }
    }
    return out;
}

static bool cache_lookup(const std::string& path, const std::string& key, TuneEntry& hit)
{
    std::lock_guard<std::mutex> lock(cache_mutex());
    for (const TuneEntry& e : cache_read(path))
        if (e.key == key) { hit = e; return true; }
    return false;
}

static void cache_store(const std::string& path, const TuneEntry& entry)
{
    std::lock_guard<std::mutex> lock(cache_mutex());
    std::vector<TuneEntry> all = cache_read(path);
    bool found = false;
    for (TuneEntry& e : all)
        if (e.key == entry.key) { e = entry; found = true; }
    if (!found) all.push_back(entry);
    std::sort(all.begin(), all.end(), [](const TuneEntry& x, const TuneEntry& y) { return x.key < y.key; });
    const std::string tmp = path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    std::fprintf(f, "{\"format\": \"libnuht tuning cache 1\", \"entries\": [\n");
    for (size_t i = 0; i < all.size(); ++i) {
        const TuneEntry& e = all[i];
        std::fprintf(f, "{\"key\": \"%s\", \"spread_chunk\": %lld, \"min_size\": %lld, \"dft_max\": %lld, "
                        "\"split_candidates\": %lld, \"ms\": %.6g}%s\n",
                     e.key.c_str(), (long long)e.spread_chunk, (long long)e.min_size, (long long)e.dft_max,
                     (long long)e.split_candidates, e.ms, i + 1 < all.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) (void)std::remove(tmp.c_str());
}

// The tuned options of plan p: from the cache when it holds p's key, else by
// tune_plan (then stored).  The options that are not tuned come from p.
static int tune_cached(nuht_plan_t p, const double* c_dev, int reps, nuht_opts* best, double* best_ms, hipStream_t s)
{
    const Partition* cur = current_forward(p);
    if (!cur) return NUHT_EINVAL;
    const std::string key = tune_key(p, cur->P);
    nuht_opts o = p->opts;
    TuneEntry e;
    if (!p->cache_path.empty() && cache_lookup(p->cache_path, key, e)) {
        o.spread_chunk = (int32_t)e.spread_chunk;
        o.min_size = e.min_size;
        o.dft_max = (int32_t)e.dft_max;
        if (o.split_candidates != -1) o.split_candidates = (int32_t)e.split_candidates;
        o.tune = 0;
        *best = o;
        if (best_ms) *best_ms = e.ms;
        return NUHT_OK;
    }
    double ms = 0.0;
    NUHT_TRY(tune_plan(p, c_dev, reps, &o, &ms, s));
    if (!p->cache_path.empty()) {
        e.key = key;
        e.spread_chunk = o.spread_chunk; e.min_size = o.min_size; e.dft_max = o.dft_max;
        e.split_candidates = o.split_candidates; e.ms = ms;
        cache_store(p->cache_path, e);
    }
    *best = o;
    if (best_ms) *best_ms = ms;
    return NUHT_OK;
}

int nuht_tune(nuht_plan_t p, const double* c_dev, int reps, nuht_opts* best, double* best_ms, void* stream)
{
    if (!p || !best || !current_forward(p)) return NUHT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    nuht_opts o;
    NUHT_TRY(tune_cached(p, c_dev, reps, &o, best_ms, s));
    // adopt the best options: the plan's partitions are rebuilt with them
    o.precision = p->opts.precision;
    o.M_override = p->opts.M_override;
    o.vector_spread = p->opts.vector_spread;
    o.local_rank = p->opts.local_rank;
    o.margin = p->opts.margin;
    o.tune_cache = nullptr;
    p->opts = o;
    p->orders.clear();
    Partition* Pt = nullptr;
    NUHT_TRY(get_partition(p, p->nu2_req, false, s, &Pt));
    *best = o;
    return NUHT_OK;
}

// ---------------------------------------------------------------------------
// Batches: many independent plans, planned with one synchronisation and
// executed as one captured graph.
// ---------------------------------------------------------------------------
constexpr int kBatchStreams = 4;

struct nuht_batch_s {
    std::vector<nuht_plan_t> plans;
    std::vector<int> stream_of;          // planning stream of each transform
    std::vector<int> order;              // transforms by decreasing n + m
    hipStream_t aux[kBatchStreams] = {};
    hipStream_t cap = nullptr;           // capture and replay stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;   // the captured graph's branch to aux[0] and back
    DevBuf b_ptrs;                       // device tables of input and output pointers
    void** c_table = nullptr;
    void** g_table = nullptr;
    BatchSchedule sched;                 // the batched launches, stage by stage
    DevBuf b_table;                      // their device tables (PlanDev array, segments)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<nuht_opts> class_opts;   // tuned options per size class (when tuned)
};

static void free_batch(nuht_batch_t b)
{
    if (!b) return;
    for (hipStream_t st : b->aux) if (st) (void)hipStreamSynchronize(st);
    if (b->cap) (void)hipStreamSynchronize(b->cap);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (nuht_plan_t p : b->plans) free_plan(p);   // stream-ordered frees on the batch's streams
    dev_free(b->b_ptrs);
    dev_free(b->b_table);
    for (hipStream_t st : b->aux) if (st) (void)hipStreamSynchronize(st);
    if (b->cap) (void)hipStreamSynchronize(b->cap);
    for (hipStream_t st : b->aux) if (st) (void)hipStreamDestroy(st);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    delete b;
}

// size class of a transform for tuning: floor(log10(n + m)), 0 .. 9
static int size_class(int64_t tot)
{
    int c = 0;
    while (tot >= 10 && c < 9) { tot /= 10; ++c; }
    return c;
}

int nuht_plan_many(nuht_batch_t* out, int count, const int* nu, double eps, const int64_t* n,
                   const double* const* r_dev, const int64_t* m, const double* const* omega_dev,
                   const nuht_opts* opts, void* stream)
{
    if (!out) return NUHT_EINVAL;
    *out = nullptr;
    if (count < 0 || count > (1 << 20)) return NUHT_EINVAL;
    if (count > 0 && (!nu || !n || !r_dev || !m || !omega_dev)) return NUHT_EINVAL;
    nuht_opts o;
    NUHT_TRY(check_opts(opts, o));
    if (design_eps(eps, o) < 1e-15) return NUHT_EINVAL;
    if (o.precision == NUHT_FP32_SPREAD && design_eps(eps, o) < 1e-7) return NUHT_EPRECISION;
    for (int i = 0; i < count; ++i) {
        if (!valid_common(nu[i], eps)) return NUHT_EINVAL;
        if (n[i] < 0 || m[i] < 0 || n[i] > INT32_MAX / 2 || m[i] > INT32_MAX / 2) return NUHT_EINVAL;
        if ((n[i] > 0 && !r_dev[i]) || (m[i] > 0 && !omega_dev[i])) return NUHT_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    nuht_batch_s* b = new (std::nothrow) nuht_batch_s();
    if (!b) return NUHT_ENOMEM;
    auto fail = [&](int code) { free_batch(b); return code; };
    auto hip_ok = [](hipError_t e) { if (e != hipSuccess) { (void)hipGetLastError(); return false; } return true; };
    for (int k = 0; k < kBatchStreams; ++k) {
        if (!hip_ok(hipStreamCreateWithFlags(&b->aux[k], hipStreamNonBlocking))) return fail(NUHT_EHIP);
    }
    if (!hip_ok(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking))) return fail(NUHT_EHIP);
    if (!hip_ok(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming))) return fail(NUHT_EHIP);
    if (!hip_ok(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming))) return fail(NUHT_EHIP);
    if (!hip_ok(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming))) return fail(NUHT_EHIP);
    if (!hip_ok(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming))) return fail(NUHT_EHIP);
    // the inputs are ready once the caller's stream reaches this point
    if (!hip_ok(hipEventRecord(b->ev_in, s))) return fail(NUHT_EHIP);
    for (int k = 0; k < kBatchStreams; ++k)
        if (!hip_ok(hipStreamWaitEvent(b->aux[k], b->ev_in, 0))) return fail(NUHT_EHIP);
    // longest-processing-time assignment of the transforms to the streams
    b->order.resize(count);
    for (int i = 0; i < count; ++i) b->order[i] = i;
    std::sort(b->order.begin(), b->order.end(), [&](int x, int y) { return n[x] + m[x] > n[y] + m[y]; });
    b->stream_of.assign(count, 0);
    {
        int64_t load[kBatchStreams] = {};
        for (int t : b->order) {
            int k = (int)(std::min_element(load, load + kBatchStreams) - load);
            b->stream_of[t] = k;
            load[k] += n[t] + m[t] + 20000;   // a fixed cost per transform for its launches
        }
    }
    b->plans.assign(count, nullptr);
    for (int i = 0; i < count; ++i) {
        int rc = plan_create(&b->plans[i], 2 * nu[i], eps, n[i], r_dev[i], m[i], omega_dev[i], o,
                             b->aux[b->stream_of[i]], nullptr);
        if (rc != NUHT_OK) return fail(rc);
    }
    if (o.tune) {
        // one representative (the largest) per size class is tuned; its options
        // serve the whole class
        nuht_opts oc = o;
        oc.tune_cache = nullptr;
        b->class_opts.assign(10, oc);
        std::vector<int> rep(10, -1);
        for (int t : b->order) {
            int c = size_class(n[t] + m[t]);
            if (rep[c] < 0) rep[c] = t;
        }
        for (int c = 0; c < 10; ++c) {
            if (rep[c] < 0) continue;
            nuht_plan_t p = b->plans[rep[c]];
            hipStream_t st = b->aux[b->stream_of[rep[c]]];
            Partition* Pt = nullptr;
            int rc = get_partition(p, p->nu2_req, false, st, &Pt);
            if (rc != NUHT_OK) return fail(rc);
            nuht_opts best;
            rc = tune_cached(p, nullptr, 3, &best, nullptr, st);
            if (rc != NUHT_OK) return fail(rc);
            best.precision = o.precision; best.M_override = o.M_override;
            best.vector_spread = o.vector_spread;
            best.tune_cache = nullptr;
            best.local_rank = o.local_rank;
            best.margin = o.margin;
            b->class_opts[c] = best;
        }
        for (int i = 0; i < count; ++i) {
            nuht_plan_t p = b->plans[i];
            p->opts = b->class_opts[size_class(n[i] + m[i])];
            p->orders.clear();
        }
    }
    // every partition's planning launched, then one synchronisation
    HostStage* slots = nullptr;
    if (count > 0 && !hip_ok(hipHostMalloc((void**)&slots, sizeof(HostStage) * (size_t)count, hipHostMallocPortable)))
        return fail(NUHT_ENOMEM);
    std::vector<std::unique_ptr<PendingPart>> pend(count);
    std::vector<Partition*> parts(count, nullptr);
    int rc = NUHT_OK;
    for (int i = 0; i < count && rc == NUHT_OK; ++i) {
        nuht_plan_t p = b->plans[i];
        nuht_plan_s::OrderParts* op = order_parts(p, p->nu2_req);
        if (!op) { rc = NUHT_ENOMEM; break; }
        parts[i] = &op->f;
        pend[i].reset(new (std::nothrow) PendingPart());
        if (!pend[i]) { rc = NUHT_ENOMEM; break; }
        rc = part_begin(p, *pend[i], *parts[i], p->fwd, p->nu2_req, b->aux[b->stream_of[i]], &slots[i], true);
    }
    for (int k = 0; k < kBatchStreams && rc == NUHT_OK; ++k)
        if (!hip_ok(hipStreamSynchronize(b->aux[k]))) rc = NUHT_EHIP;
    for (int i = 0; i < count && rc == NUHT_OK; ++i) {
        bool again = false;
        rc = part_finish(*pend[i], &slots[i], &again);
        while (rc == NUHT_OK && again) {   // tables too small: this one again, on its own
            hipStream_t st = b->aux[b->stream_of[i]];
            rc = part_begin(b->plans[i], *pend[i], *parts[i], b->plans[i]->fwd, b->plans[i]->nu2_req, st,
                            &slots[i], false);
            if (rc == NUHT_OK && !hip_ok(hipStreamSynchronize(st))) rc = NUHT_EHIP;
            if (rc == NUHT_OK) rc = part_finish(*pend[i], &slots[i], &again);
        }
    }
    pend.clear();
    if (slots) (void)hipHostFree(slots);
    if (rc != NUHT_OK) return fail(rc);
    // pointer tables for the graph
    if (count > 0) {
        Slab slab;
        slab.add(b->c_table, (size_t)count);
        slab.add(b->g_table, (size_t)count);
        if (slab.commit(b->b_ptrs, b->cap) != NUHT_OK) return fail(NUHT_ENOMEM);
    }
    // the launch list and its device tables
    {
        std::vector<BatchTransform> tr(count);
        for (int i = 0; i < count; ++i) {
            const Partition* Pt = current_forward(b->plans[i]);
            if (!Pt) return fail(NUHT_EINVAL);
            tr[i] = BatchTransform{&Pt->P, &Pt->sum, Pt->cls.data(), (int)Pt->cls.size()};
        }
        build_batch_schedule(tr.data(), count, b->order.data(), b->sched);
        if (!b->sched.launches.empty()) {
            if (dev_alloc(b->b_table, b->sched.table.size(), b->cap) != NUHT_OK) return fail(NUHT_ENOMEM);
            if (!hip_ok(hipMemcpyAsync(b->b_table.p, b->sched.table.data(), b->sched.table.size(),
                                       hipMemcpyHostToDevice, b->cap)))
                return fail(NUHT_EHIP);
        }
    }
    for (int k = 0; k < kBatchStreams; ++k)
        if (!hip_ok(hipStreamSynchronize(b->aux[k]))) return fail(NUHT_EHIP);
    if (!hip_ok(hipStreamSynchronize(b->cap))) return fail(NUHT_EHIP);
    *out = b;
    return NUHT_OK;
}

// Captures the batch's execution into one graph: the batched launches, stage
// by stage (each launch covers every transform with work in its stage), on
// the capture stream, with the local moments and direct blocks on a branch
// of their own (the batch's first planning stream, idle by now, joins the
// capture through the fork event); inputs and outputs come from the pointer
// tables.
static int capture_batch(nuht_batch_t b)
{
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return NUHT_EHIP;
    }
    ExecFork fork;
    fork.side = b->aux[0];
    fork.ev_fork = b->ev_fork;
    fork.ev_join = b->ev_join;
    hipError_t e = launch_execute_many(b->sched, b->b_table.p, b->c_table, b->g_table, b->cap, &fork);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return NUHT_EHIP;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(g);
        return NUHT_EHIP;
    }
    b->graph = g;
    b->exec = x;
    return NUHT_OK;
}

int nuht_execute_many(nuht_batch_t b, const double* const* c_dev, double* const* g_dev, void* stream)
{
    if (!b) return NUHT_EINVAL;
    const int count = (int)b->plans.size();
    if (count == 0) return NUHT_OK;
    if (!c_dev || !g_dev) return NUHT_EINVAL;
    for (int i = 0; i < count; ++i) {
        if (b->plans[i]->n > 0 && !c_dev[i]) return NUHT_EINVAL;
        if (b->plans[i]->m > 0 && !g_dev[i]) return NUHT_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if (b->sched.launches.empty()) return NUHT_OK;   // every transform has m = 0
    if (!b->exec) NUHT_TRY(capture_batch(b));
    HIP_TRY(hipEventRecord(b->ev_in, s));
    HIP_TRY(hipStreamWaitEvent(b->cap, b->ev_in, 0));
    for (int off = 0; off < count; off += 224) {
        int cnt = std::min(224, count - off);
        HIP_TRY(launch_set_pointers(b->c_table + off, (const void* const*)(c_dev + off), cnt, b->cap));
        HIP_TRY(launch_set_pointers(b->g_table + off, (const void* const*)(g_dev + off), cnt, b->cap));
    }
    HIP_TRY(hipGraphLaunch(b->exec, b->cap));
    HIP_TRY(hipEventRecord(b->ev_out, b->cap));
    HIP_TRY(hipStreamWaitEvent(s, b->ev_out, 0));
    return NUHT_OK;
}

int nuht_batch_info(nuht_batch_t b, int index, nuht_info* info)
{
    if (!b || index < 0 || index >= (int)b->plans.size()) return NUHT_EINVAL;
    return nuht_plan_info(b->plans[index], info);
}

int nuht_batch_destroy(nuht_batch_t b)
{
    free_batch(b);
    return NUHT_OK;
}

int nuht_plan_order(nuht_plan_t p, double* r_sorted, int32_t* perm_r, double* omega_sorted, int32_t* perm_omega,
                    void* stream)
{
    if (!p) return NUHT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const Geometry& G = p->fwd;   // sorted by plan creation, which synchronised on that work
    if (r_sorted && G.n > 0) HIP_TRY(hipMemcpyAsync(r_sorted, G.rs, sizeof(double) * (size_t)G.n,
                                                    hipMemcpyDeviceToDevice, s));
    if (perm_r && G.n > 0) HIP_TRY(hipMemcpyAsync(perm_r, G.perm_r, sizeof(int32_t) * (size_t)G.n,
                                                  hipMemcpyDeviceToDevice, s));
    if (omega_sorted && G.m > 0) HIP_TRY(hipMemcpyAsync(omega_sorted, G.ws, sizeof(double) * (size_t)G.m,
                                                        hipMemcpyDeviceToDevice, s));
    if (perm_omega && G.m > 0) HIP_TRY(hipMemcpyAsync(perm_omega, G.perm_w, sizeof(int32_t) * (size_t)G.m,
                                                      hipMemcpyDeviceToDevice, s));
    note_use(p, s);
    return NUHT_OK;
}

int nuht_plan_info(nuht_plan_t p, nuht_info* info)
{
    if (!p || !info) return NUHT_EINVAL;
    const Partition* cur = current_forward(p);
    if (!cur) return NUHT_EINVAL;
    const Partition& Pt = *cur;
    const PlanDev& P = Pt.P;
    const Summary& S = Pt.sum;
    std::memset(info, 0, sizeof(*info));
    info->nu = p->nu2_req >> 1; info->M = P.M; info->L = P.L; info->es_width = P.w;
    info->half_order = p->nu2_req & 1;
    info->eps = P.eps; info->z = P.z; info->es_beta = P.beta;
    info->levels = S.levels; info->n_nodes = S.n_nodes; info->n_local = S.n_l; info->n_asy = S.n_a;
    info->n_direct = S.n_d; info->n_fft_blocks = S.n_fft;
    info->local_row_members = S.l_row; info->local_col_members = S.l_col;
    info->asy_row_members = S.a_row; info->asy_col_members = S.a_col;
    info->direct_entries = S.d_ent;
    info->grid_cells = S.grid_cells; info->fft_points = S.fft_points;
    info->dft_row_cells = S.dft_row_cells; info->fft_row_members = S.fft_rows;
    int64_t bytes = p->geom_bytes + (int64_t)p->b_grad.bytes;
    for (auto& o : p->orders) bytes += o->f.bytes + o->a.bytes;
    info->workspace_bytes = bytes;
    info->min_size = p->opts.min_size > 0 ? p->opts.min_size : default_min_size(p->n, p->m);
    info->dft_max = p->opts.dft_max == 0 ? 48 : p->opts.dft_max;
    info->spread_chunk = P.spread_chunk;
    info->spread_items = S.n_aitems;
    info->dense_items = S.n_adense + S.n_amed;
    info->split_candidates = p->opts.split_candidates == -1 ? -1
                             : (p->opts.split_candidates > 1 ? p->opts.split_candidates : 16);
    return NUHT_OK;
}

int nuht_profile_stages(nuht_plan_t p, uint32_t mask)
{
    if (!p) return NUHT_EINVAL;
    if (mask >> kStages) return NUHT_EINVAL;
    prof_clear(p);
    p->prof = mask != 0;
    p->prof_mask = mask;
    return NUHT_OK;
}

int nuht_profile(nuht_plan_t p, int enable)
{
    return nuht_profile_stages(p, enable ? (1u << kStages) - 1 : 0u);
}

int nuht_profile_read(nuht_plan_t p, double* stage_ms, int64_t* calls)
{
    if (!p || !stage_ms) return NUHT_EINVAL;
    for (int i = 0; i < kStages; ++i) stage_ms[i] = 0.0;
    int64_t nc = (int64_t)p->prof_events.size() / (kStages + 1);
    if (nc > 0) {   // the last call's last recorded event
        hipEvent_t* e = p->prof_events.data() + (nc - 1) * (kStages + 1);
        for (int i = kStages; i >= 0; --i)
            if (e[i]) { HIP_TRY(hipEventSynchronize(e[i])); break; }
    }
    for (int64_t c = 0; c < nc; ++c) {
        hipEvent_t* e = p->prof_events.data() + c * (kStages + 1);
        for (int i = 0; i < kStages; ++i) {
            if (!e[i] || !e[i + 1]) continue;
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, e[i], e[i + 1]));
            stage_ms[i] += ms;
        }
    }
    if (calls) *calls = nc;
    return NUHT_OK;
}

int nuht_destroy(nuht_plan_t p)
{
    free_plan(p);
    return NUHT_OK;
}

int nuht_direct(int nu, double eps, int64_t n, const double* r_dev, const double* c_dev, int64_t m,
                const double* omega_dev, double* g_dev, void* stream)
{
    if (!valid_common(nu, eps)) return NUHT_EINVAL;
    if (n < 0 || m < 0 || n > INT32_MAX || m > INT32_MAX) return NUHT_EINVAL;
    if ((n > 0 && (!r_dev || !c_dev)) || (m > 0 && (!omega_dev || !g_dev))) return NUHT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    PlanDev P{};
    nuht_opts o{};
    NUHT_TRY(fill_params(P, 2 * nu, eps, o));
    if (m == 0) return NUHT_OK;
    if (n == 0) { HIP_TRY(hipMemsetAsync(g_dev, 0, sizeof(double) * (size_t)m, s)); return NUHT_OK; }
    HIP_TRY(launch_direct(P, r_dev, c_dev, (int32_t)n, omega_dev, (int32_t)m, g_dev, s));
    return NUHT_OK;
}

}  // extern "C"
