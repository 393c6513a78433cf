// nuht_device.h -- device helpers: double-double arithmetic, phase reduction,
// the exponential-of-semicircle kernel, and Bessel-function evaluation.
#pragma once

#include "nuht_internal.h"

namespace nuht {

struct dd {
    double hi, lo;
};

// a*b == hi + lo exactly (TwoProduct with a fused multiply-add).
__device__ __forceinline__ dd two_prod(double a, double b)
{
    double p = a * b;
    return {p, __builtin_fma(a, b, -p)};
}

// a+b == hi + lo exactly (Knuth's TwoSum).
__device__ __forceinline__ dd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

// a b + c with c the same in every lane (a constant, or a value read through
// the scalar unit), as one FMA with c its scalar-register addend.  The
// compiler would keep such an addend in vector registers and copy it before
// each two-operand FMA, an extra instruction per term of a polynomial.
__device__ __forceinline__ double fma_uniform_addend(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// 1/sqrt(x) and 1/x for positive normal x: the hardware estimate refined by two
// Newton steps (to within an ulp or two; cheaper than IEEE division and sqrt).
__device__ __forceinline__ double rsqrt_refined(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    #pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double h = 0.5 * x * y;
        y = __builtin_fma(y, __builtin_fma(-h, y, 0.5), y);    // y (3/2 - x y^2 / 2)
    }
    return y;
}

__device__ __forceinline__ double rcp_refined(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    #pragma unroll
    for (int k = 0; k < 2; ++k) y = __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
    return y;
}

constexpr double kTwoPiHi = 6.283185307179586232;        // 2 pi rounded to double
constexpr double kTwoPiLo = 2.4492935982947064e-16;       // 2 pi - kTwoPiHi
constexpr double kInvTwoPi = 0.15915494309189535;        // 1/(2 pi) rounded to double
constexpr double kInvTwoPiLo = -9.8393383375912433e-18;   // 1/(2 pi) - kInvTwoPi
constexpr double kPi = 3.141592653589793116;
constexpr double kSqrt2OverPi = 0.79788456080286541;

// sin x and cos x for |x| <= 64: x is reduced by the nearest multiple q of
// pi/2 (pi/2 split into two doubles, each product taken inside an FMA), and
// sin, cos of the remainder |r| <= pi/4 are the Taylor polynomials through
// r^17 and r^18 (truncation below 1e-19), chosen by q mod 4.  No
// large-argument reduction, which keeps the register footprint small.
__device__ __forceinline__ void sincos_small(double x, double* sp, double* cp)
{
    constexpr double kPio2Hi = 1.5707963267948966;       // pi/2 rounded to double
    constexpr double kPio2Lo = 6.123233995736766e-17;    // pi/2 - kPio2Hi
    constexpr double kTwoOverPi = 0.6366197723675814;
    double q = rint(x * kTwoOverPi);
    double r = __builtin_fma(-q, kPio2Hi, x);
    r = __builtin_fma(-q, kPio2Lo, r);
    double r2 = r * r;
    double ps = 1.0 / 355687428096000.0;                  // 1/17!
    ps = fma_uniform_addend(ps, r2, -1.0 / 1307674368000.0);
    ps = fma_uniform_addend(ps, r2, 1.0 / 6227020800.0);
    ps = fma_uniform_addend(ps, r2, -1.0 / 39916800.0);
    ps = fma_uniform_addend(ps, r2, 1.0 / 362880.0);
    ps = fma_uniform_addend(ps, r2, -1.0 / 5040.0);
    ps = fma_uniform_addend(ps, r2, 1.0 / 120.0);
    ps = fma_uniform_addend(ps, r2, -1.0 / 6.0);
    double sn = __builtin_fma(r * r2, ps, r);
    double pc = -1.0 / 6402373705728000.0;                // -1/18!
    pc = fma_uniform_addend(pc, r2, 1.0 / 20922789888000.0);
    pc = fma_uniform_addend(pc, r2, -1.0 / 87178291200.0);
    pc = fma_uniform_addend(pc, r2, 1.0 / 479001600.0);
    pc = fma_uniform_addend(pc, r2, -1.0 / 3628800.0);
    pc = fma_uniform_addend(pc, r2, 1.0 / 40320.0);
    pc = fma_uniform_addend(pc, r2, -1.0 / 720.0);
    pc = fma_uniform_addend(pc, r2, 1.0 / 24.0);
    pc = __builtin_fma(pc, r2, -0.5);                     // -0.5 is an inline constant
    double cs = __builtin_fma(r2, pc, 1.0);
    int k = (int)q & 3;
    double s0 = (k & 1) ? cs : sn;
    double c0 = (k & 1) ? sn : cs;
    *sp = (k & 2) ? -s0 : s0;
    *cp = ((k + 1) & 2) ? -c0 : c0;
}

// (cos t, sin t) for t = hi + lo, |hi| < 2^52.  t is reduced by the nearest
// multiple k of 2 pi: hi - k*kTwoPiHi is exact (k*kTwoPiHi is formed exactly
// and lies within a factor two of hi), the low parts are added afterwards, and
// the residual low part enters as a first-order correction.
__device__ __forceinline__ void cis_dd(double hi, double lo, double& c, double& s)
{
    double k = rint(hi * kInvTwoPi);
    dd p = two_prod(k, kTwoPiHi);
    double r = hi - p.hi;
    double rl = (lo - p.lo) - k * kTwoPiLo;
    dd t = two_sum(r, rl);
    double sn, cs;
    sincos_small(t.hi, &sn, &cs);
    c = __builtin_fma(-t.lo, sn, cs);
    s = __builtin_fma(t.lo, cs, sn);
}

// 1/k for k < 128 (exact to the last bit: every entry is the double nearest 1/k).
__device__ __constant__ static const double kInvInt[128] = {
    0.0, 1.0 / 1, 1.0 / 2, 1.0 / 3, 1.0 / 4, 1.0 / 5, 1.0 / 6, 1.0 / 7, 1.0 / 8, 1.0 / 9, 1.0 / 10, 1.0 / 11,
    1.0 / 12, 1.0 / 13, 1.0 / 14, 1.0 / 15, 1.0 / 16, 1.0 / 17, 1.0 / 18, 1.0 / 19, 1.0 / 20, 1.0 / 21, 1.0 / 22,
    1.0 / 23, 1.0 / 24, 1.0 / 25, 1.0 / 26, 1.0 / 27, 1.0 / 28, 1.0 / 29, 1.0 / 30, 1.0 / 31, 1.0 / 32, 1.0 / 33,
    1.0 / 34, 1.0 / 35, 1.0 / 36, 1.0 / 37, 1.0 / 38, 1.0 / 39, 1.0 / 40, 1.0 / 41, 1.0 / 42, 1.0 / 43, 1.0 / 44,
    1.0 / 45, 1.0 / 46, 1.0 / 47, 1.0 / 48, 1.0 / 49, 1.0 / 50, 1.0 / 51, 1.0 / 52, 1.0 / 53, 1.0 / 54, 1.0 / 55,
    1.0 / 56, 1.0 / 57, 1.0 / 58, 1.0 / 59, 1.0 / 60, 1.0 / 61, 1.0 / 62, 1.0 / 63, 1.0 / 64, 1.0 / 65, 1.0 / 66,
    1.0 / 67, 1.0 / 68, 1.0 / 69, 1.0 / 70, 1.0 / 71, 1.0 / 72, 1.0 / 73, 1.0 / 74, 1.0 / 75, 1.0 / 76, 1.0 / 77,
    1.0 / 78, 1.0 / 79, 1.0 / 80, 1.0 / 81, 1.0 / 82, 1.0 / 83, 1.0 / 84, 1.0 / 85, 1.0 / 86, 1.0 / 87, 1.0 / 88,
    1.0 / 89, 1.0 / 90, 1.0 / 91, 1.0 / 92, 1.0 / 93, 1.0 / 94, 1.0 / 95, 1.0 / 96, 1.0 / 97, 1.0 / 98, 1.0 / 99,
    1.0 / 100, 1.0 / 101, 1.0 / 102, 1.0 / 103, 1.0 / 104, 1.0 / 105, 1.0 / 106, 1.0 / 107, 1.0 / 108, 1.0 / 109,
    1.0 / 110, 1.0 / 111, 1.0 / 112, 1.0 / 113, 1.0 / 114, 1.0 / 115, 1.0 / 116, 1.0 / 117, 1.0 / 118, 1.0 / 119,
    1.0 / 120, 1.0 / 121, 1.0 / 122, 1.0 / 123, 1.0 / 124, 1.0 / 125, 1.0 / 126, 1.0 / 127};

// ES^(kappa) = int_{-1}^{1} ES(x) e^{i kappa x} dx for 0 <= kappa <= kappa_max.
// ES^ is even in kappa, so on that range it is a smooth function of
// s = 2 (kappa / kappa_max)^2 - 1 in [-1, 1]: the plan holds the monomial
// coefficients in s of its Chebyshev interpolant of degree kEshatTerms - 1
// (for widths 4 .. 18 coefficients at most 0.63 in magnitude against values
// 0.035 .. 0.8, so Horner's rule loses nothing to cancellation; within 1e-14
// of ES^, relative), the same for every lane.
__device__ __forceinline__ double eshat(const PlanDev& P, double kappa)
{
    const double s = __builtin_fma(kappa * kappa, P.eshat_s, -1.0);
    double v = P.eshat[kEshatTerms - 1];
    #pragma unroll
    for (int i = kEshatTerms - 2; i >= 0; --i) v = __builtin_fma(v, s, P.eshat[i]);
    return v;
}

// Starting index of Miller's backward recurrence at argument y: started there,
// the recurrence reproduces J_0(y) .. J_40(y) to the FP64 rounding floor
// (checked against 30-digit values for 0.01 <= y <= 160).
__device__ __forceinline__ int miller_start(double y)
{
    return (int)(y + 8.0 * cbrt(y) + 12.0);
}

// J_nu(x) for 0 <= x (nu >= 0) by Miller's backward recurrence
// J_{k-1} = (2k/x) J_k - J_{k+1}, normalised by J_0^2 + 2 sum J_k^2 = 1,
// with the first-order correction for the low part of x = xh + xl.
__device__ inline double besselj_miller(int nu, double xh, double xl)
{
    if (xh == 0.0) return nu == 0 ? 1.0 : 0.0;
    if (xh < 1e-30) return nu == 0 ? 1.0 : 0.0;
    int N = miller_start(xh);
    if (nu > N) return 0.0;
    if (N < nu + 1) N = nu + 1;
    double rec = 2.0 / xh;
    double yk1 = 0.0, yk = 1e-100, S = 0.0;
    double jm = 0.0, j0 = 0.0, jp = 0.0;
    for (int k = N; k >= 0; --k) {
        if (k == nu + 1) jp = yk;
        if (k == nu) j0 = yk;
        if (k == nu - 1) jm = yk;
        S = __builtin_fma(k == 0 ? yk : 2.0 * yk, yk, S);
        if (k == 0) break;
        double ykm1 = __builtin_fma((double)k * rec, yk, -yk1);
        yk1 = yk;
        yk = ykm1;
        if (fabs(yk) > 1e100) {
            yk *= 1e-100; yk1 *= 1e-100; S *= 1e-200;
            jm *= 1e-100; j0 *= 1e-100; jp *= 1e-100;
        }
    }
    double inv = 1.0 / sqrt(S);
    double d = nu == 0 ? -jp : 0.5 * (jm - jp);
    return __builtin_fma(xl, d, j0) * inv;
}

// The M-term Hankel approximation of J_nu at x = xh + xl (Sec. 3.2):
//   sqrt(2/(pi x)) [ P cos(x + phi) - Q sin(x + phi) ],
//   P = sum_{l<M} (-1)^l a_{2l} / x^{2l},  Q = sum_{l<M} (-1)^l a_{2l+1} / x^{2l+1}.
__device__ inline double besselj_hankel(const PlanDev& P, double xh, double xl)
{
    dd ph = two_sum(xh, P.phi_hi);
    double c, s;
    cis_dd(ph.hi, ph.lo + xl + P.phi_lo, c, s);
    double inv = 1.0 / xh;
    double inv2 = inv * inv;
    double p = 0.0, q = 0.0;
    for (int l = P.M - 1; l >= 0; --l) {
        double sg = (l & 1) ? -1.0 : 1.0;
        p = __builtin_fma(p, inv2, sg * P.hank[2 * l]);
        q = __builtin_fma(q, inv2, sg * P.hank[2 * l + 1]);
    }
    q *= inv;
    return sqrt(2.0 / (kPi * xh)) * __builtin_fma(p, c, -q * s);
}

// J_nu(x) accurate to the plan's eps: Hankel's M-term formula above the
// crossover z (where it is eps-accurate by the choice of z), Miller below.
__device__ __forceinline__ double besselj_eps(const PlanDev& P, double xh, double xl)
{
    return xh > P.z ? besselj_hankel(P, xh, xl) : besselj_miller(P.nu, xh, xl);
}

// One step k -> k-1 of Miller's backward recurrence y_{k-1} = (2k/x) y_k - y_{k+1}
// (kd = k as a double, rec = 2/x), adding 2 y_k^2 to the normalisation sum
// S = y_0^2 + 2 sum_{k>=1} y_k^2.  When y_k grows past 2^332 everything held
// (the recurrence pair, S and the values kept so far) is scaled by 2^-332,
// exactly, so the result does not depend on where the scaling happens.
__device__ __forceinline__ void miller_step(double kd, double rec, double& yk, double& yk1, double& S,
                                            double& a, double& b, double& c)
{
    S = __builtin_fma(yk + yk, yk, S);
    const double ykm1 = __builtin_fma(kd * rec, yk, -yk1);
    yk1 = yk;
    yk = ykm1;
    if (fabs(yk) > 0x1p332) {
        yk *= 0x1p-332; yk1 *= 0x1p-332; S *= 0x1p-664;
        a *= 0x1p-332; b *= 0x1p-332; c *= 0x1p-332;
    }
}

// J_nu(x) (nu >= 0, phase offset -(2 nu + 1) pi / 4 as phi_hi + phi_lo) to
// full FP64 accuracy: Hankel's expansion summed until its terms
// fall below 1e-17 where it converges that far (x >= 25, terms never above
// 1e3), Miller's recurrence otherwise.  Used for the direct blocks.
__device__ inline double besselj_core(int nu, double phi_hi, double phi_lo, double xh, double xl)
{
    if (xh >= 25.0) {
        // terms t_k = prod_{i<=k} (mu - (2i-1)^2) / (8 x i); odd k go to Q, even
        // k to P, with sign (-1)^floor(k/2): one odd and one even term per step
        const double mu = 4.0 * (double)nu * (double)nu;
        const double inv8x = 0.125 / xh;
        double t = 1.0, p = 1.0, q = 0.0, prev = 1e300;
        bool ok = false;
        for (int k = 1; k < 119; k += 2) {
            const double f1 = 2.0 * k - 1.0, f2 = f1 + 2.0;
            const double sg = ((k >> 1) & 1) ? -1.0 : 1.0;       // (-1)^floor(k/2); the even term k+1 has -sg
            const double t1 = t * ((mu - f1 * f1) * inv8x * kInvInt[k]);
            const double t2 = t1 * ((mu - f2 * f2) * inv8x * kInvInt[k + 1]);
            const double a1 = fabs(t1), a2 = fabs(t2);
            q = __builtin_fma(sg, t1, q);
            if (a1 < 1e-17) { ok = true; break; }
            if ((a1 > prev && k > 2) || a1 > 1e3) break;
            p = __builtin_fma(-sg, t2, p);
            if (a2 < 1e-17) { ok = true; break; }
            if ((k > 1 && a2 > a1) || a2 > 1e3) break;
            prev = a2;
            t = t2;
        }
        if (ok) {
            dd ph = two_sum(xh, phi_hi);
            double c, s;
            cis_dd(ph.hi, ph.lo + xl + phi_lo, c, s);
            return sqrt(2.0 / (kPi * xh)) * __builtin_fma(p, c, -q * s);
        }
    }
    if (xh < 1e-30) return nu == 0 ? 1.0 : 0.0;
    const double top = (double)(nu + 1) > xh ? (double)(nu + 1) : xh;
    const int N = (int)(top + 12.0 + 8.0 * cbrt(xh > 1.0 ? xh : 1.0));   // >= nu + 13
    const double rec = 2.0 / xh;
    double yk1 = 0.0, yk = 1e-100, S = 0.0;
    double jm = 0.0, j0 = 0.0, jp = 0.0;
    double kd = (double)N;
    // k = N .. nu + 2: nothing kept
    for (int k = N; k > nu + 1; --k, kd -= 1.0) miller_step(kd, rec, yk, yk1, S, jm, j0, jp);
    jp = yk;                                                     // y_{nu+1}
    miller_step(kd, rec, yk, yk1, S, jm, j0, jp);
    kd -= 1.0;
    j0 = yk;                                                     // y_nu
    if (nu > 0) {
        miller_step(kd, rec, yk, yk1, S, jm, j0, jp);
        kd -= 1.0;
        jm = yk;                                                 // y_{nu-1}
        for (int k = nu - 1; k > 0; --k, kd -= 1.0) miller_step(kd, rec, yk, yk1, S, jm, j0, jp);
    }
    S = __builtin_fma(yk, yk, S);                                // k = 0 counts once
    const double d = nu == 0 ? -jp : 0.5 * (jm - jp);
    return __builtin_fma(xl, d, j0) / sqrt(S);
}

// J_{n+1/2}(x) (n >= 0, phase offset -(n+1) pi/2 as phi_hi + phi_lo) to full
// FP64 accuracy through the spherical Bessel function, J_{n+1/2}(x) =
// sqrt(2x/pi) j_n(x) (DLMF 10.47.3):
//   x >= 25 with Hankel's terms never above 1e3: Hankel's expansion, which ends
//     at a_n at half-integer orders and is then exact;
//   x > n + 1: the upward recurrence j_{k+1} = ((2k+1)/x) j_k - j_{k-1} from
//     j_{-1} = cos x / x, j_0 = sin x / x (stable while k < x; the low part of
//     x enters through the double-double sine and cosine);
//   otherwise: Miller's backward recurrence with the same relation, normalised
//     by sum_k (2k+1) j_k^2 = 1 (DLMF 10.60.11), scaled by exact powers of two,
//     and the low part through J' = sqrt(2x/pi) (j_{n-1} - ((n + 1/2)/x) j_n).
__device__ inline double besselj_half_core(int n, double phi_hi, double phi_lo, double xh, double xl)
{
    if (xh < 1e-300) return 0.0;
    if (xh >= 25.0) {
        const double mu = (2.0 * n + 1.0) * (2.0 * n + 1.0);
        const double inv8x = 0.125 / xh;
        double t = 1.0, p = 1.0, q = 0.0;
        bool ok = true;
        for (int k = 1; k <= n; ++k) {
            const double f = 2.0 * k - 1.0;
            t *= (mu - f * f) * inv8x * kInvInt[k];
            if (fabs(t) > 1e3) { ok = false; break; }
            const double sg = ((k >> 1) & 1) ? -1.0 : 1.0;       // (-1)^floor(k/2)
            if (k & 1) q = __builtin_fma(sg, t, q);
            else p = __builtin_fma(sg, t, p);
        }
        if (ok) {
            dd ph = two_sum(xh, phi_hi);
            double c, s;
            cis_dd(ph.hi, ph.lo + xl + phi_lo, c, s);
            return sqrt(2.0 / (kPi * xh)) * __builtin_fma(p, c, -q * s);
        }
    }
    const double amp = sqrt(2.0 * xh / kPi);
    const double inv = 1.0 / xh;
    if (xh > n + 1.0) {
        double c, s;
        cis_dd(xh, xl, c, s);
        double jm = c * inv, j = s * inv;                        // j_{-1}, j_0
        for (int k = 0; k < n; ++k) {
            const double jp = __builtin_fma((2.0 * k + 1.0) * inv, j, -jm);
            jm = j;
            j = jp;
        }
        return amp * j;
    }
    const int N = (int)(n + xh + 20.0 + 8.0 * cbrt(xh > 1.0 ? xh : 1.0));
    double yk1 = 0.0, yk = 1e-100, S = 0.0, rn = 0.0, rnm1 = 0.0;
    for (int k = N; k >= 0; --k) {
        if (k == n) rn = yk;
        if (k == n - 1) rnm1 = yk;
        S = __builtin_fma((2.0 * k + 1.0) * yk, yk, S);
        if (k == 0) break;
        const double ykm1 = __builtin_fma((2.0 * k + 1.0) * inv, yk, -yk1);
        yk1 = yk;
        yk = ykm1;
        if (fabs(yk) > 0x1p332) {
            yk *= 0x1p-332; yk1 *= 0x1p-332; S *= 0x1p-664; rn *= 0x1p-332; rnm1 *= 0x1p-332;
        }
    }
    const double lam = 1.0 / sqrt(S);
    const double jn = rn * lam;
    double jnm1;
    if (n == 0) {
        double c, s;
        sincos_small(xh, &s, &c);                                // xh <= 1 here
        jnm1 = c * inv;
    } else {
        jnm1 = rnm1 * lam;
    }
    const double d = amp * __builtin_fma(-(n + 0.5) * inv, jn, jnm1);
    return __builtin_fma(xl, d, amp * jn);
}

// The same for the plan's order and phase offset.
__device__ __forceinline__ double besselj_full(const PlanDev& P, double xh, double xl)
{
    if (P.half) return besselj_half_core(P.nu, P.phi_hi, P.phi_lo, xh, xl);
    return besselj_core(P.nu, P.phi_hi, P.phi_lo, xh, xl);
}

// ---------------------------------------------------------------------------
// FFT: X[k] = sum_n x[n] e^{+2 pi i n k / N}, N a power of two, in LDS.
// Stockham autosort, radix 4 (one radix-2 stage first when log2 N is odd).
// Element (line, n) of the tile lives at sm[line * ls + n * es].  The tile
// holds at most 4096 points and the block 256 threads, so a thread carries at
// most 8 radix-2 or 4 radix-4 butterflies per stage.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(__builtin_fma(a.x, b.x, -a.y * b.y), __builtin_fma(a.x, b.y, a.y * b.x));
}

__device__ inline void lds_fft(double2* sm, int N, int logN, int lines, int ls, int es)
{
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    int Ns = 1;
    if (logN & 1) {
        const int half = N >> 1;
        const int nb = lines * half;
        double2 v[8][2];
        #pragma unroll
        for (int c = 0; c < 8; ++c) {
            int b = tid + c * nt;
            if (b < nb) {
                int line = b / half, j = b - line * half;
                v[c][0] = sm[line * ls + j * es];
                v[c][1] = sm[line * ls + (j + half) * es];
            }
        }
        __syncthreads();
        #pragma unroll
        for (int c = 0; c < 8; ++c) {
            int b = tid + c * nt;
            if (b < nb) {
                int line = b / half, j = b - line * half;
                double2 a = v[c][0], d = v[c][1];
                sm[line * ls + (2 * j) * es] = make_double2(a.x + d.x, a.y + d.y);
                sm[line * ls + (2 * j + 1) * es] = make_double2(a.x - d.x, a.y - d.y);
            }
        }
        __syncthreads();
        Ns = 2;
    }
    const int q4 = N >> 2;
    while (Ns < N) {
        const int nb = lines * q4;
        double2 v[4][4];
        #pragma unroll
        for (int c = 0; c < 4; ++c) {
            int b = tid + c * nt;
            if (b < nb) {
                int line = b / q4, j = b - line * q4;
                #pragma unroll
                for (int r = 0; r < 4; ++r) v[c][r] = sm[line * ls + (j + r * q4) * es];
            }
        }
        __syncthreads();
        #pragma unroll
        for (int c = 0; c < 4; ++c) {
            int b = tid + c * nt;
            if (b < nb) {
                int line = b / q4, j = b - line * q4;
                int k = j & (Ns - 1);
                double s, co;
                sincospi(2.0 * (double)k / (double)(4 * Ns), &s, &co);
                double2 w1 = make_double2(co, s);
                double2 w2 = cmul(w1, w1);
                double2 w3 = cmul(w2, w1);
                double2 x0 = v[c][0];
                double2 x1 = cmul(v[c][1], w1);
                double2 x2 = cmul(v[c][2], w2);
                double2 x3 = cmul(v[c][3], w3);
                double2 a0 = make_double2(x0.x + x2.x, x0.y + x2.y);
                double2 a1 = make_double2(x0.x - x2.x, x0.y - x2.y);
                double2 a2 = make_double2(x1.x + x3.x, x1.y + x3.y);
                double2 a3 = make_double2(-(x1.y - x3.y), x1.x - x3.x);   // i (x1 - x3)
                int d0 = (j - k) * 4 + k;
                sm[line * ls + (d0) * es] = make_double2(a0.x + a2.x, a0.y + a2.y);
                sm[line * ls + (d0 + Ns) * es] = make_double2(a1.x + a3.x, a1.y + a3.y);
                sm[line * ls + (d0 + 2 * Ns) * es] = make_double2(a0.x - a2.x, a0.y - a2.y);
                sm[line * ls + (d0 + 3 * Ns) * es] = make_double2(a1.x - a3.x, a1.y - a3.y);
            }
        }
        __syncthreads();
        Ns <<= 2;
    }
}


}  // namespace nuht
