/*
 * oracle/bessel.c -- CPU reference for the discrete Hankel transform.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain FP64 oracle that the
 * GPU library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code with the GPU
 * library and the GPU library never calls it.
 *
 * What it computes (Beckman & O'Neil, "A Nonuniform Fast Hankel Transform"):
 *   g_j = sum_k c_k J_nu(omega_j r_k)                       (Sec. 1, eq. DHT)
 * for integer order nu, by direct O(nm) summation.  Every argument omega_j r_k
 * is formed exactly as an unevaluated double-double sum hi + lo (TwoProduct
 * with fma), so the reference does not inherit the rounding of fl(omega r),
 * which at arguments near 1e5 is the dominant FP64 error of any direct sum.
 *
 * J_n(x) for integer n >= 0 is evaluated by whichever textbook method is
 * accurate at (n, x):
 *   x == 0            J_n(0) = [n == 0]
 *   0 < x < 2         the power series  sum_s (-1)^s (x/2)^(2s+n) / (s! (s+n)!)
 *   x >= 25 and the   Hankel's large-argument expansion (Sec. 3.2, eq.
 *   series converges  asymptotic-expansion), summed until its terms fall below
 *                     1e-17 (the expansion is divergent, so it is used only
 *                     where its smallest term is that small)
 *   otherwise         Miller's backward recurrence J_{k-1} = (2k/x) J_k - J_{k+1},
 *                     normalised by J_0^2 + 2 sum_{k>=1} J_k^2 = 1
 * The low part of the argument enters as a first-order Taylor correction
 * (Hankel: in the phase; the other branches: through J_n').
 *
 * Negative integer orders use J_{-n} = (-1)^n J_n.
 *
 * Half-integer orders nu = n + 1/2 (n >= 0; the radial Fourier transform in
 * odd dimension d has nu = d/2 - 1) go through the spherical Bessel function,
 * J_{n+1/2}(x) = sqrt(2x/pi) j_n(x) (DLMF 10.47.3), in long double:
 *   x > n + 1         upward recurrence j_{k+1} = ((2k+1)/x) j_k - j_{k-1} from
 *                     j_{-1} = cos x / x and j_0 = sin x / x (stable while k < x)
 *   otherwise         Miller's backward recurrence with the same relation,
 *                     normalised by sum_k (2k+1) j_k^2 = 1 (DLMF 10.60.11)
 * and the low part of the argument through J_nu' = J_{nu-1} - (nu/x) J_nu.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_PI 3.14159265358979323846

/* a*b == *hi + *lo exactly (no overflow/underflow assumed). */
static inline void two_prod(double a, double b, double *hi, double *lo)
{
    *hi = a * b;
    *lo = fma(a, b, -*hi);
}

/* ------------------------------------------------------------------------ */
/* Power series, used for 0 < x < 2 where its terms decrease monotonically.   */
/* ------------------------------------------------------------------------ */
static double series_j(int n, double x)
{
    double half = 0.5 * x;
    double lead = 1.0;                 /* (x/2)^n / n!  built as a product */
    for (int i = 1; i <= n; ++i) {
        lead *= half / (double)i;
        if (lead == 0.0) return 0.0;   /* below the smallest double: J_n(x) ~ 0 */
    }
    double q = -half * half;
    double term = lead, sum = lead;
    for (int s = 1; s < 200; ++s) {
        term *= q / ((double)s * (double)(s + n));
        sum += term;
        if (fabs(term) <= 1e-18 * fabs(sum)) break;
    }
    return sum;
}

/* ------------------------------------------------------------------------ */
/* Hankel's expansion with real order (also used at half-integer orders by   */
/* the tests, where it terminates and is exact).                             */
/*   J_nu(x) ~ sqrt(2/(pi x)) [ P cos(x+phi) - Q sin(x+phi) ],               */
/*   P = sum_l (-1)^l a_{2l}/x^{2l},  Q = sum_l (-1)^l a_{2l+1}/x^{2l+1},     */
/*   phi = -(2 nu + 1) pi / 4,                                               */
/*   a_k(nu) = prod_{s=1..k} (4nu^2 - (2s-1)^2) / (k! 8^k).                   */
/* nterms > 0 keeps exactly terms k = 0 .. nterms-1 (for tests);             */
/* nterms == 0 sums until |term| < 1e-17 and returns 0 if a term exceeds 1e3  */
/* or the terms start to grow first (argument too small for this order).      */
/* ------------------------------------------------------------------------ */
static int hankel_pq(double nu, double x, int nterms, double *P, double *Q)
{
    double mu = 4.0 * nu * nu;
    double t = 1.0;                     /* a_k / x^k */
    double p = 1.0, q = 0.0;
    double prev = INFINITY;
    int kmax = nterms > 0 ? nterms : 400;
    for (int k = 1; k < kmax; ++k) {
        double f = (double)(2 * k - 1);
        t *= (mu - f * f) / (8.0 * (double)k * x);
        /* k = 2l -> P gets (-1)^l t ; k = 2l+1 -> Q gets (-1)^l t */
        int l = k / 2;
        double sgn = (l & 1) ? -1.0 : 1.0;
        if (k & 1) q += sgn * t; else p += sgn * t;
        if (nterms == 0) {
            double at = fabs(t);
            if (at < 1e-17) { *P = p; *Q = q; return 1; }
            /* growing terms: divergence has set in, or the sum would cancel
               terms far larger than its result; leave it to Miller */
            if ((at > prev && k > 2) || at > 1e3) return 0;
            prev = at;
        }
    }
    *P = p; *Q = q;
    return nterms > 0;
}

static double hankel_value(double nu, double xh, double xl, double P, double Q)
{
    /* phi modulo 2 pi: (2nu+1) is reduced mod 8 exactly before scaling by pi/4,
       so large orders do not carry the rounding of a large multiple of pi */
    double phi = -fmod(2.0 * nu + 1.0, 8.0) * ORC_PI / 4.0;
    double cp = cos(phi), sp = sin(phi);
    double cx = cos(xh), sx = sin(xh);
    /* first-order correction for the low part of the argument */
    double c = cx - xl * sx;
    double s = sx + xl * cx;
    double cph = c * cp - s * sp;     /* cos(x + phi) */
    double sph = s * cp + c * sp;     /* sin(x + phi) */
    double x = xh + xl;
    return sqrt(2.0 / (ORC_PI * x)) * (P * cph - Q * sph);
}

/* ------------------------------------------------------------------------ */
/* Miller's backward recurrence for J_{n-1}, J_n, J_{n+1} at x > 0.          */
/* ------------------------------------------------------------------------ */
static void miller_j(int n, double x, double *jm1, double *j0, double *jp1)
{
    double top = (double)(n + 1) > x ? (double)(n + 1) : x;
    int N = (int)(top + 20.0 + 15.0 * cbrt(x > 1.0 ? x : 1.0));
    if (N & 1) ++N;
    double yk1 = 0.0;        /* y_{k+1} */
    double yk = 1.0;         /* y_k, k = N */
    double S = 0.0;          /* y_0^2 + 2 sum_{k>=1} y_k^2 */
    double rm1 = 0.0, r0 = 0.0, rp1 = 0.0;
    for (int k = N; k >= 0; --k) {
        /* yk holds y_k here */
        if (k == n + 1) rp1 = yk;
        if (k == n) r0 = yk;
        if (k == n - 1) rm1 = yk;
        S += (k == 0 ? 1.0 : 2.0) * yk * yk;
        if (k == 0) break;
        double ykm1 = (2.0 * (double)k / x) * yk - yk1;
        yk1 = yk;
        yk = ykm1;
        if (fabs(yk) > 1e100) {
            const double f = 1e-100;
            yk *= f; yk1 *= f; S *= f * f;
            rm1 *= f; r0 *= f; rp1 *= f;
        }
    }
    double lam = sqrt(S);
    *jm1 = rm1 / lam;
    *j0 = r0 / lam;
    *jp1 = rp1 / lam;
}

/* J_n(xh + xl) for integer n >= 0, xh >= 0. */
static double besselj_nonneg(int n, double xh, double xl)
{
    if (xh == 0.0 && xl == 0.0) return n == 0 ? 1.0 : 0.0;
    if (xh >= 25.0) {
        double P, Q;
        if (hankel_pq((double)n, xh, 0, &P, &Q)) return hankel_value((double)n, xh, xl, P, Q);
    }
    if (xh < 2.0) {
        double jn = series_j(n, xh);
        double jn1 = series_j(n + 1, xh);
        double d = (double)n / xh * jn - jn1;           /* J_n'(x) */
        return jn + xl * d;
    }
    double jm1, jn, jp1;
    miller_j(n, xh, &jm1, &jn, &jp1);
    double d = n == 0 ? -jp1 : 0.5 * (jm1 - jp1);
    return jn + xl * d;
}

static double besselj_int(int nu, double xh, double xl)
{
    if (nu >= 0) return besselj_nonneg(nu, xh, xl);
    double v = besselj_nonneg(-nu, xh, xl);
    return ((-nu) & 1) ? -v : v;
}

/* J_{n+1/2}(xh + xl) for n >= 0, xh >= 0 (see the header). */
static double besselj_half(int n, double xh, double xl)
{
    if (xh == 0.0 && xl == 0.0) return 0.0;
    const long double x = (long double)xh;
    const long double sx = sinl(x), cx = cosl(x);
    long double jn, jnm1;                      /* j_n(x), j_{n-1}(x) */
    if (x > (long double)n + 1.0L) {
        long double jm = cx / x, j = sx / x;   /* j_{-1}, j_0 */
        for (int k = 0; k < n; ++k) {
            const long double jp = ((long double)(2 * k + 1) / x) * j - jm;
            jm = j;
            j = jp;
        }
        jn = j;
        jnm1 = jm;
    } else {
        const int N = (int)((long double)n + x + 30.0L + 15.0L * cbrtl(x > 1.0L ? x : 1.0L));
        long double yk1 = 0.0L, yk = 1e-300L, S = 0.0L, rn = 0.0L, rnm1 = 0.0L;
        for (int k = N; k >= 0; --k) {
            if (k == n) rn = yk;
            if (k == n - 1) rnm1 = yk;
            S += (long double)(2 * k + 1) * yk * yk;
            if (k == 0) break;
            const long double ykm1 = ((long double)(2 * k + 1) / x) * yk - yk1;
            yk1 = yk;
            yk = ykm1;
            if (fabsl(yk) > 1e1000L) {
                const long double f = 1e-1000L;
                yk *= f; yk1 *= f; S *= f * f; rn *= f; rnm1 *= f;
            }
        }
        const long double lam = sqrtl(S);
        jn = rn / lam;
        jnm1 = n == 0 ? cx / x : rnm1 / lam;
    }
    const long double amp = sqrtl(2.0L * x / 3.141592653589793238462643383279502884L);
    const long double J = amp * jn;
    const long double dJ = amp * (jnm1 - (((long double)n + 0.5L) / x) * jn);
    return (double)(J + (long double)xl * dJ);
}

/* J_{nu2/2}: integer orders for even nu2, n + 1/2 (n = (nu2 - 1) / 2 >= 0) for odd nu2 >= 1. */
static double besselj_twice(int nu2, double xh, double xl)
{
    if ((nu2 & 1) == 0) return besselj_int(nu2 / 2, xh, xl);
    return besselj_half((nu2 - 1) / 2, xh, xl);
}

/* ======================================================================== */
/* Exported entry points (called through ctypes).                           */
/* ======================================================================== */

/* out[i] = J_{nu2/2}(xh[i] + xl[i]): integer or half-integer (nu2 odd, >= 1) orders. */
void orc_besselj_twice(int nu2, const double *xh, const double *xl, int64_t n, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = besselj_twice(nu2, xh[i], xl ? xl[i] : 0.0);
}

/* out[i] = J_nu(xh[i] + xl[i]). */
void orc_besselj(int nu, const double *xh, const double *xl, int64_t n, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = besselj_int(nu, xh[i], xl ? xl[i] : 0.0);
}

/* Hankel's expansion at real order nu with exactly nterms terms (k < nterms). */
void orc_hankel_series(double nu, const double *x, int64_t n, int nterms, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double P, Q;
        hankel_pq(nu, x[i], nterms, &P, &Q);
        out[i] = hankel_value(nu, x[i], 0.0, P, Q);
    }
}

/* Hankel coefficient a_k(nu) (Sec. 3.2), by its product definition. */
double orc_hankel_coef(double nu, int k)
{
    double a = 1.0;
    for (int s = 1; s <= k; ++s) {
        double f = (double)(2 * s - 1);
        a *= (4.0 * nu * nu - f * f) / (8.0 * (double)s);
    }
    return a;
}

/*
 * Direct discrete Hankel transform (Sec. 1, eq. DHT):
 *   g[j] = sum_k c[k] J_nu(w[j] * r[k]),  j < m,  k < n,
 * with exact double-double arguments and Neumaier-compensated summation.
 * Parallel over outputs; nthreads <= 0 uses the OpenMP default.
 */
void orc_dht_twice(int nu2, int64_t n, const double *r, const double *c,
                   int64_t m, const double *w, double *g, int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < m; ++j) {
        double sum = 0.0, comp = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            if (c[k] == 0.0) continue;
            double xh, xl;
            two_prod(w[j], r[k], &xh, &xl);
            double t = c[k] * besselj_twice(nu2, xh, xl);
            double s = sum + t;
            if (fabs(sum) >= fabs(t)) comp += (sum - s) + t; else comp += (t - s) + sum;
            sum = s;
        }
        g[j] = sum + comp;
    }
}

/* The same for integer orders. */
void orc_dht(int nu, int64_t n, const double *r, const double *c,
             int64_t m, const double *w, double *g, int nthreads)
{
    orc_dht_twice(2 * nu, n, r, c, m, w, g, nthreads);
}

/* Number of OpenMP threads a parallel region would use. */
int orc_max_threads(void) { return omp_get_max_threads(); }

/*
 * Staircase of the local region (Sec. 4.1): for sorted r (ascending) and each
 * frequency w[j], K[j] = #{k : w[j] * r[k] <= z}, where the product is the
 * exact real product (decided from its double-double representation).
 */
static inline int exact_le(double a, double b, double z)
{
    double hi, lo;
    two_prod(a, b, &hi, &lo);
    if (hi < z) return 1;
    if (hi > z) return 0;
    return lo <= 0.0;
}

void orc_staircase(int64_t n, const double *r_sorted, int64_t m, const double *w,
                   double z, int64_t *K)
{
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j) {
        int64_t lo = 0, hi = n;          /* first k with w r_k > z lies in [lo, hi] */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (exact_le(w[j], r_sorted[mid], z)) lo = mid + 1; else hi = mid;
        }
        K[j] = lo;
    }
}

/* 1 if w*r <= z exactly, else 0 (vectorised helper for tests). */
void orc_exact_le(const double *w, const double *r, int64_t n, double z, int32_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = exact_le(w[i], r[i], z);
}

/*
 * M-term Hankel approximation of one matrix block (integer or half-integer
 * order nu), applied to a vector by direct summation (the asymptotic block
 * formula of Sec. 3.2, eq. asy-error, written entry-wise):
 *   H_M(x) = sqrt(2/pi) sum_{l<M} (-1)^l [ a_{2l} x^{-2l-1/2} cos(x+phi)
 *                                        - a_{2l+1} x^{-2l-3/2} sin(x+phi) ],
 *   g[i] += sum_k c[k] H_M(w[i] r[k]),  x = w r formed exactly.
 */
void orc_asy_block(double nu, int M, int64_t mb, const double *w, int64_t nb,
                   const double *r, const double *c, double *g)
{
    double a[64];
    for (int k = 0; k < 2 * M && k < 64; ++k) a[k] = orc_hankel_coef(nu, k);
    double phi = -fmod(2.0 * nu + 1.0, 8.0) * ORC_PI / 4.0;
    double cp = cos(phi), sp = sin(phi);
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < mb; ++i) {
        double sum = 0.0, comp = 0.0;
        for (int64_t k = 0; k < nb; ++k) {
            if (c[k] == 0.0) continue;
            double xh, xl;
            two_prod(w[i], r[k], &xh, &xl);
            double cx = cos(xh), sx = sin(xh);
            double cc = cx - xl * sx, ss = sx + xl * cx;
            double cph = cc * cp - ss * sp, sph = ss * cp + cc * sp;
            double x = xh + xl;
            double inv = 1.0 / x;
            double pw = 1.0 / sqrt(x);      /* x^{-1/2} */
            double h = 0.0;
            for (int l = 0; l < M; ++l) {
                double sg = (l & 1) ? -1.0 : 1.0;
                h += sg * a[2 * l] * pw * cph;
                pw *= inv;
                h -= sg * a[2 * l + 1] * pw * sph;
                pw *= inv;
            }
            double t = c[k] * sqrt(2.0 / ORC_PI) * h;
            double s = sum + t;
            if (fabs(sum) >= fabs(t)) comp += (sum - s) + t; else comp += (t - s) + sum;
            sum = s;
        }
        g[i] += sum + comp;
    }
}
