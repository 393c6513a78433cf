// exec.hip -- execution of a planned transform (Alg. 2): local blocks by the
// Wimp expansion (Sec. 3.1), asymptotic blocks by type-3 NUFFTs of Hankel's
// expansion (Sec. 3.2), direct blocks entry by entry.
//
// Column side (reductions over points):  gather c -> local moments ->
//   ES spreading of 2M weight channels onto each asymptotic block's grid.
// Grid stage:  reduce spread partials; for large grids deconvolve by the
//   inner kernel's transform, zero-pad and FFT.
// Row side (one thread per frequency): walk the block tree from the root and
//   add, level by level, the row's local, asymptotic and (at the end) direct
//   contributions; write g once, in the caller's order.
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <utility>
#include <vector>

#include "nuht_device.h"
#include "nuht_launch.h"

namespace nuht {

// ---------------------------------------------------------------------------
// Every execution kernel is a body taking the transform (P) and the index of
// its workgroup within that transform's work.  A single transform's kernel
// passes P by value and blockIdx.x; a batched kernel covers every transform
// of a batch in one launch: its workgroup finds its transform in a table of
// segments (WorkSeg, ascending g0) and runs the body on that transform's
// PlanDev, kept in device memory, as its workgroup blockIdx.x - g0.
// ---------------------------------------------------------------------------
// A batch's PlanDev array is written once, before the graph that reads it is
// recorded, and never while a batched kernel runs: it is read through the
// constant address space, like a kernel argument, so that the compiler may
// load its fields through the scalar unit.
typedef const __attribute__((address_space(4))) PlanDev ConstPlanDev;
__device__ __forceinline__ const PlanDev& plan_of(const PlanDev* plans, int t)
{
    return *(const PlanDev*)((ConstPlanDev*)plans + t);
}

// The segment of this workgroup (the last one with g0 <= blockIdx.x).
template <class Seg>
__device__ __forceinline__ int find_seg_index(const Seg* __restrict__ segs, int nseg)
{
    const int g = blockIdx.x;
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].g0 <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The transform of this workgroup and the workgroup's index within it.
__device__ __forceinline__ WorkSeg find_seg(const WorkSeg* __restrict__ segs, int nseg)
{
    const int s = find_seg_index(segs, nseg);
    return WorkSeg{segs[s].t, (int32_t)blockIdx.x - segs[s].g0};
}

// cs[k] = c[perm[k]] (times the sorted point r_k when scale is set).
__device__ __forceinline__ void gather_body(const PlanDev& P, int bid, const double* c, bool scale)
{
    const int32_t k = bid * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    const double v = c[P.perm_r[k]];
    P.cs[k] = scale ? v * P.rs[k] : v;
}

// c is read from c_slot when that is set.
__global__ void k_gather(PlanDev P, const double* c, const double* const* c_slot, int scale)
{
    gather_body(P, blockIdx.x, c_slot ? *c_slot : c, scale != 0);
}

__global__ void k_gather_many(const PlanDev* __restrict__ plans, const WorkSeg* __restrict__ segs, int nseg,
                              const double* const* c_table)
{
    const WorkSeg w = find_seg(segs, nseg);
    gather_body(plan_of(plans, w.t), w.g0, c_table[w.t], false);
}

// A transform with no points: the output is zero.
__global__ void k_zero_output(double* g, double* const* g_slot, int64_t m)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double* gp = g_slot ? *g_slot : g;
    gp[i] = 0.0;
}

__global__ void k_zero_output_many(const PlanDev* __restrict__ plans, const WorkSeg* __restrict__ segs, int nseg,
                                   double* const* g_table)
{
    const WorkSeg w = find_seg(segs, nseg);
    const int64_t i = (int64_t)w.g0 * blockDim.x + threadIdx.x;
    if (i < plan_of(plans, w.t).m) g_table[w.t][i] = 0.0;
}

// gd = 0 ahead of the direct blocks.
__global__ void k_zero_gd_many(const PlanDev* __restrict__ plans, const WorkSeg* __restrict__ segs, int nseg)
{
    const WorkSeg w = find_seg(segs, nseg);
    const PlanDev& P = plan_of(plans, w.t);
    const int64_t i = (int64_t)w.g0 * blockDim.x + threadIdx.x;
    if (i < P.m) P.gd[i] = 0.0;
}

__global__ void k_fill_value(double* __restrict__ x, int64_t n, double v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

struct PtrArgs {
    void* p[224];
};

__global__ void k_set_pointers(void** table, PtrArgs a, int count)
{
    int i = threadIdx.x;
    if (i < count) table[i] = a.p[i];
}

// out = w (a - b) / 2: the derivative J_nu' = (J_{nu-1} - J_{nu+1}) / 2 applied
// to the two shifted-order transforms.
__global__ void k_half_difference(const double* __restrict__ w, const double* __restrict__ a,
                                  const double* __restrict__ b, double* __restrict__ out, int32_t n)
{
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = 0.5 * w[k] * (a[k] - b[k]);
}

// ---------------------------------------------------------------------------
// Local moments t_l = sum_k c_k T_{2l(+1)}(r_k / R) of one chunk of a local
// block's columns (Sec. 3.1: T^T applied first).  The Chebyshev polynomials
// come from the recurrence in u = 2y^2 - 1:  T_{2(l+1)+e}(y) = 2u T_{2l+e}(y) - T_{2(l-1)+e}(y).
// Moments are produced in passes of up to 64 (a multiple of 8: all L + 1 in
// one pass up to L = 63, so no pass repeats the recurrence through an earlier
// pass's moments there).  One 64-lane wave per item: each lane accumulates its
// points' moments in registers (points strided over the lanes), and the wave
// reduces them with cross-lane sums, in chunks of 64, 32, 16 and 8 moments.
// ---------------------------------------------------------------------------
// One reduce-scatter level: v[0 .. 2H) -> v[0 .. H), lanes with bit H set
// keeping the upper half; partner lane ^ H holds the other copy.
template <int H, int NQ>
__device__ __forceinline__ void reduce_scatter_half(double (&v)[NQ], int lane)
{
    const bool upper = (lane & H) != 0;
    #pragma unroll
    for (int i = 0; i < H; ++i) {
        double keep = upper ? v[i + H] : v[i];
        double send = upper ? v[i] : v[i + H];
        v[i] = keep + __shfl_xor(send, H);
    }
}

// Sum over the wave of the C moments acc[off .. off + C) (C a power of two,
// 8 to 64): a reduce-scatter at offsets C/2 .. 1 leaves lane q with moment
// off + (q mod C) summed over the lanes congruent to q; exchanges at offsets
// C .. 32 complete the sums.
template <int C, int NQ>
__device__ __forceinline__ double reduce_chunk(const double (&acc)[NQ], int off, int lane)
{
    double v[C];
    #pragma unroll
    for (int i = 0; i < C; ++i) v[i] = acc[off + i];
    if constexpr (C >= 64) reduce_scatter_half<32>(v, lane);
    if constexpr (C >= 32) reduce_scatter_half<16>(v, lane);
    if constexpr (C >= 16) reduce_scatter_half<8>(v, lane);
    reduce_scatter_half<4>(v, lane);
    reduce_scatter_half<2>(v, lane);
    reduce_scatter_half<1>(v, lane);
    double mine = v[0];
    #pragma unroll
    for (int o = C; o < 64; o <<= 1) mine += __shfl_xor(mine, o);
    return mine;
}

// Stores the chunk of C moments starting at s0 + off (those up to L).
template <int C, int NQ>
__device__ __forceinline__ void store_chunk(const double (&acc)[NQ], int off, int s0, int L, int lane,
                                            double* __restrict__ dst)
{
    const double mine = reduce_chunk<C>(acc, off, lane);
    if (lane < C && s0 + off + lane <= L) dst[s0 + off + lane] = mine;
}

// Moments s0 .. s0 + NQ - 1 of the item (those up to L are stored); NQ a
// multiple of 8 up to 64.
template <int NQ>
__device__ __forceinline__ void lmom_pass(const PlanDev& P, const Item& I, const LBlock& B, const double* __restrict__ cs,
                                          double* __restrict__ lpart, int s0, int lane, int bid)
{
    static_assert(NQ % 8 == 0 && NQ >= 8 && NQ <= 64, "pass width");
    const int L = P.L;
    const int odd = P.nu & 1;
    double acc[NQ];
    #pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    // y = r / R through the block's reciprocal (within an ulp of the
    // quotient; y only enters the Chebyshev recurrence)
    const double inv_R = 1.0 / B.R;
    // two points per lane per step (the second with weight 0 past the end):
    // both loads issue together and the recurrences are independent chains
    for (int k = I.ka + lane; k < I.kb; k += 128) {
        const bool two = k + 64 < I.kb;
        const int k2 = two ? k + 64 : k;
        const double ya = P.rs[k] * inv_R, yb = P.rs[k2] * inv_R;
        double ca = cs[k], cb = two ? cs[k2] : 0.0;
        if (P.half) {          // half-integer orders: weights c sqrt(r / R)
            ca *= sqrt(ya);
            cb *= sqrt(yb);
        }
        const double ua2 = 2.0 * __builtin_fma(2.0 * ya, ya, -1.0);
        const double ub2 = 2.0 * __builtin_fma(2.0 * yb, yb, -1.0);
        double a0, a1, b0, b1;
        if (odd) { a0 = ya; a1 = ya * (ua2 - 1.0); b0 = yb; b1 = yb * (ub2 - 1.0); }
        else { a0 = 1.0; a1 = 0.5 * ua2; b0 = 1.0; b1 = 0.5 * ub2; }
        for (int l = 0; l < s0; ++l) {
            const double a2 = __builtin_fma(ua2, a1, -a0), b2 = __builtin_fma(ub2, b1, -b0);
            a0 = a1; a1 = a2; b0 = b1; b1 = b2;
        }
        #pragma unroll
        for (int q = 0; q < NQ; ++q) {
            acc[q] = __builtin_fma(cb, b0, __builtin_fma(ca, a0, acc[q]));
            const double a2 = __builtin_fma(ua2, a1, -a0), b2 = __builtin_fma(ub2, b1, -b0);
            a0 = a1; a1 = a2; b0 = b1; b1 = b2;
        }
    }
    // the pass's moments in chunks of 64, 32, 16 and 8 (NQ's binary digits)
    double* __restrict__ dst = lpart + (int64_t)bid * (L + 1);
    constexpr int c64 = NQ & 64, c32 = NQ & 32, c16 = NQ & 16, c8 = NQ & 8;
    if constexpr (c64) store_chunk<64>(acc, 0, s0, L, lane, dst);
    if constexpr (c32) store_chunk<32>(acc, c64, s0, L, lane, dst);
    if constexpr (c16) store_chunk<16>(acc, c64 + c32, s0, L, lane, dst);
    if constexpr (c8) store_chunk<8>(acc, c64 + c32 + c16, s0, L, lane, dst);
}

// MAXQ: the widest pass (32 or 64).  A kernel's registers follow its widest
// pass, so orders with L < 32 run the 32-wide instance at twice the waves.
template <int MAXQ>
__device__ __forceinline__ void lmom_body(const PlanDev& P, int bid)
{
    const Item I = P.litems[bid];
    const LBlock B = P.lb[I.blk];
    const int L = P.L;
    const int lane = threadIdx.x;
    const double* __restrict__ cs = P.cs;
    double* __restrict__ lpart = P.lpart;
    // passes of up to MAXQ moments, each the multiple of 8 that covers what is left
    for (int s0 = 0; s0 <= L;) {
        const int rem = L + 1 - s0;
        const int nq = rem >= MAXQ ? MAXQ : (rem + 7) / 8 * 8;
        if (nq == 8) lmom_pass<8>(P, I, B, cs, lpart, s0, lane, bid);
        else if (nq == 16) lmom_pass<16>(P, I, B, cs, lpart, s0, lane, bid);
        else if (nq == 24) lmom_pass<24>(P, I, B, cs, lpart, s0, lane, bid);
        else if (nq == 32) lmom_pass<32>(P, I, B, cs, lpart, s0, lane, bid);
        else if constexpr (MAXQ > 32) {
            if (nq == 40) lmom_pass<40>(P, I, B, cs, lpart, s0, lane, bid);
            else if (nq == 48) lmom_pass<48>(P, I, B, cs, lpart, s0, lane, bid);
            else if (nq == 56) lmom_pass<56>(P, I, B, cs, lpart, s0, lane, bid);
            else lmom_pass<64>(P, I, B, cs, lpart, s0, lane, bid);
        }
        s0 += nq;
    }
}

// The instance for an order's local rank L.
constexpr int lmom_width(int L) { return L + 1 <= 32 ? 32 : 64; }

template <int MAXQ>
__global__ __launch_bounds__(64) void k_lmom(PlanDev P) { lmom_body<MAXQ>(P, blockIdx.x); }

template <int MAXQ>
__global__ __launch_bounds__(64) void k_lmom_many(const PlanDev* __restrict__ plans,
                                                  const WorkSeg* __restrict__ segs, int nseg)
{
    const WorkSeg w = find_seg(segs, nseg);
    lmom_body<MAXQ>(plan_of(plans, w.t), w.g0);
}

// Sum of a local block's item partials, in a fixed order: eight running sums
// over the items (item i into sum i mod 8), combined pairwise.  A block can
// hold a few hundred items (the top-level local block spans most columns),
// and eight independent sums keep eight loads in flight instead of one.
__device__ __forceinline__ void lmom_reduce_body(const PlanDev& P, int bid)
{
    const int32_t t = bid * (int32_t)blockDim.x + (int32_t)threadIdx.x;
    const int32_t Lp = P.L + 1;
    if (t >= P.n_l * Lp) return;
    const int32_t b = t / Lp;
    const int32_t l = t - b * Lp;
    const LBlock B = P.lb[b];
    const double* __restrict__ col = P.lpart + (int64_t)B.item0 * Lp + l;
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int32_t it = 0;
    for (; it + 8 <= B.nitems; it += 8) {
        #pragma unroll
        for (int q = 0; q < 8; ++q) a[q] += col[(int64_t)(it + q) * Lp];
    }
    #pragma unroll
    for (int q = 0; q < 7; ++q)
        if (it + q < B.nitems) a[q] += col[(int64_t)(it + q) * Lp];
    const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    // stored as the row pass uses them: u_0 = t_0, u_l = 2 (-1)^l t_l (integer
    // orders), t_l itself (half-integer orders: the factors are in the table)
    P.lmom[t] = (l == 0 || P.half) ? s : ((l & 1) ? -2.0 * s : 2.0 * s);
}

__global__ void k_lmom_reduce(PlanDev P) { lmom_reduce_body(P, blockIdx.x); }

__global__ void k_lmom_reduce_many(const PlanDev* __restrict__ plans, const WorkSeg* __restrict__ segs, int nseg)
{
    const WorkSeg w = find_seg(segs, nseg);
    lmom_reduce_body(plan_of(plans, w.t), w.g0);
}

// ---------------------------------------------------------------------------
// ES spreading of one chunk of an asymptotic block's points (type-3 NUFFT,
// step one).  Point k of the block carries the 2M channel weights
//   x_k^(p) = c_k (r0/r_k)^(p+1/2) e^{i D (r_k - C)},   p = 0 .. 2M-1
// (the weights c_k r_k^(-p-1/2) of Sec. 3.2, normalised by the block's
// smallest point r0, times the type-3 pre-phase), placed at grid coordinate
// u_k = (r_k - C)/h.  Cell l receives sum_k x_k^(p) ES((l - u_k) 2/w).
//
// The points of an item are taken in sub-chunks of kSpreadSub.
// Phase 1: one thread per point forms the offset r - C and the phase
// D (r - C) as double-doubles (so the kernel position and the phase are exact
// to FP64 relative to themselves), the weight and the ratio r0 / r, the first
// cell l0 it reaches, and its w kernel values from the polynomial pieces
// (sums of coefficients common to all lanes times powers of the point's
// offset), all into LDS.
// Phase 2: threads own (cell, slice) pairs; the points reaching cell l are
// those with l - w < l0 <= l, a contiguous range (points are sorted), found by
// binary search; slices of one cell are adjacent lanes and are summed with
// cross-lane shuffles after the last sub-chunk.
// ---------------------------------------------------------------------------
constexpr int kSpreadSub = 256;

// T is the type of the weights, kernel values and channel sums: double, or
// float in the FP32-spreading mode (positions and phases stay double-double
// either way); partials are stored as the matching two-component vector.
// One point of a sub-chunk in LDS: weight (real, imaginary), ratio r0 / r and
// first cell reached, read with two (one for float) 16-byte loads.
template <typename T>
struct alignas(16) SpreadPoint {
    T wr, wi, q;
    int32_t l0;
};

// Dynamic LDS of k_spread: kSpreadSub point records, then w kernel values per point.
template <typename T>
constexpr size_t spread_lds_bytes(int w)
{
    return (size_t)kSpreadSub * (sizeof(SpreadPoint<T>) + (size_t)w * sizeof(T));
}

// One point of a block for spreading: weight c sqrt(r0/r) e^{i D (r - C)}
// (real, imaginary), ratio q = r0 / r, first cell reached l0, and the kernel
// argument s = 2 f - 1 of the polynomial pieces.  The phase is a double-double
// product; the cell position (r - C) / h is formed from the double-double
// difference (the scaling by h is exact).
struct PointEval {
    double wr, wi, q, s;
    int l0;
};

__device__ __forceinline__ PointEval eval_point(const ABlock& B, double r, double c, double inv_h, double hw)
{
    dd tp = two_sum(r, -B.C);
    dd ph = two_prod(B.D, tp.hi);
    double cth, sth;
    cis_dd(ph.hi, __builtin_fma(B.D, tp.lo, ph.lo), cth, sth);
    // q = r0 / r in (0, 1] and its square root through the refined hardware
    // estimates (within an ulp or two; no IEEE division or square root)
    const double q = B.r0 * rcp_refined(r);
    const double w0 = c * (q * rsqrt_refined(q));
    // u - w/2 = (tp.hi + tp.lo)/h - w/2
    dd a = two_sum(tp.hi * inv_h, -hw);
    double lo = a.lo + tp.lo * inv_h;
    double fl = floor(a.hi);
    double frac = (a.hi - fl) + lo;          // a.hi - fl is exact
    if (frac < 0.0) { fl -= 1.0; frac += 1.0; }
    else if (frac >= 1.0) { fl += 1.0; frac -= 1.0; }
    PointEval e;
    e.wr = w0 * cth;
    e.wi = w0 * sth;
    e.q = q;
    e.l0 = (int)fl + 1;
    e.s = 1.0 - 2.0 * frac;                  // s = 2 f - 1, f = 1 - frac
    return e;
}

__device__ __forceinline__ double typed_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float typed_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int NCH, typename T>
__device__ __forceinline__ void spread_body(const PlanDev& P, int bid)
{
    using T2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
    T2* part = reinterpret_cast<T2*>(P.part);
    const double* __restrict__ cs = P.cs;
    const double* __restrict__ es_poly = P.es_poly;
    extern __shared__ double4 spread_lds[];
    SpreadPoint<T>* s_pt = reinterpret_cast<SpreadPoint<T>*>(spread_lds);
    T* s_k = reinterpret_cast<T*>(s_pt + kSpreadSub);
    // the items not spread on the matrix cores, from the back of the order
    const Item I = P.aitems[P.alist[P.n_aitems - 1 - bid]];
    const ABlock B = P.ab[I.blk];
    const int tid = threadIdx.x;
    const int w = P.w;
    const double hw = 0.5 * w;
    const double inv_h = 1.0 / B.h;      // exact: h is a power of two
    const int sub_n = I.sub_n;
    int slices = 1;
    while (slices < 64 && slices * 2 * sub_n <= 256) slices <<= 1;
    const int cells_par = 256 / slices;
    for (int cbase = 0; cbase < sub_n; cbase += cells_par) {
        const int cell = cbase + tid / slices;
        const int sl = tid & (slices - 1);
        const int l = I.sub_lo + cell;
        T ar[NCH], ai[NCH];
        #pragma unroll
        for (int p = 0; p < NCH; ++p) { ar[p] = T(0); ai[p] = T(0); }
        for (int k0 = I.ka; k0 < I.kb; k0 += kSpreadSub) {
            const int np = (I.kb - k0) < kSpreadSub ? (I.kb - k0) : kSpreadSub;
            __syncthreads();
            // every thread evaluates a point (the last one when tid >= np) so
            // that the coefficient loads below stay wave-uniform (scalar)
            {
                const bool own = tid < np;
                const int k = k0 + (own ? tid : np - 1);
                const PointEval e = eval_point(B, P.rs[k], cs[k], inv_h, hw);
                if (own) {
                    SpreadPoint<T> rec;
                    rec.wr = (T)e.wr;
                    rec.wi = (T)e.wi;
                    rec.q = (T)e.q;
                    rec.l0 = e.l0;
                    s_pt[tid] = rec;
                }
                const double sv = e.s;
                // powers s^0 .. s^h once per point (h = ceil(kEsDeg / 2));
                // each piece is then sum_{d<=h} c_d s^d + s^h sum_{d>h} c_d
                // s^(d-h), with the (scalar) coefficients as multiplicands
                constexpr int kHalf = (kEsDeg + 1) / 2;
                double spow[kHalf + 1];
                spow[0] = 1.0;
                #pragma unroll
                for (int d = 1; d <= kHalf; ++d) spow[d] = spow[d - 1] * sv;
                T* kv = s_k + tid * w;
                for (int t = 0; t < w; ++t) {
                    const double* cf = es_poly + t * (kEsDeg + 1);
                    double vlo = cf[0], vhi = cf[kHalf + 1] * spow[1];
                    #pragma unroll
                    for (int d = 1; d <= kHalf; ++d) vlo = __builtin_fma(cf[d], spow[d], vlo);
                    #pragma unroll
                    for (int d = kHalf + 2; d <= kEsDeg; ++d) vhi = __builtin_fma(cf[d], spow[d - kHalf], vhi);
                    double v = __builtin_fma(spow[kHalf], vhi, vlo);
                    if (own) kv[t] = (T)v;
                }
            }
            __syncthreads();
            if (cell < sub_n) {
                // points with l0 in (l - w, l]
                int lo = 0, hi = np;
                while (lo < hi) { int mid = (lo + hi) >> 1; if (s_pt[mid].l0 <= l - w) lo = mid + 1; else hi = mid; }
                int first = lo;
                hi = np;
                while (lo < hi) { int mid = (lo + hi) >> 1; if (s_pt[mid].l0 <= l) lo = mid + 1; else hi = mid; }
                int last = lo;
                for (int i = first + sl; i < last; i += slices) {
                    const SpreadPoint<T> rec = s_pt[i];
                    T phi = s_k[i * w + (l - rec.l0)];
                    const T vr = phi * rec.wr, vi = phi * rec.wi;
                    const T q = rec.q;
                    // one chain of powers q^p serves both parts
                    T qp = T(1);
                    #pragma unroll
                    for (int p = 0; p < NCH; ++p) {
                        ar[p] = typed_fma(vr, qp, ar[p]);
                        ai[p] = typed_fma(vi, qp, ai[p]);
                        qp *= q;
                    }
                }
            }
        }
        for (int o = slices >> 1; o >= 1; o >>= 1) {
            #pragma unroll
            for (int p = 0; p < NCH; ++p) {
                ar[p] += __shfl_xor(ar[p], o);
                ai[p] += __shfl_xor(ai[p], o);
            }
        }
        if (cell < sub_n && sl == 0) {
            T2* dst = part + I.off + (int64_t)cell * NCH;
            #pragma unroll
            for (int p = 0; p < NCH; ++p) { dst[p].x = ar[p]; dst[p].y = ai[p]; }
        }
    }
}

template <int NCH, typename T>
__global__ __launch_bounds__(256) void k_spread(PlanDev P)
{
    spread_body<NCH, T>(P, blockIdx.x);
}

template <int NCH, typename T>
__global__ __launch_bounds__(256) void k_spread_many(const PlanDev* __restrict__ plans,
                                                     const WorkSeg* __restrict__ segs, int nseg)
{
    const WorkSeg w = find_seg(segs, nseg);
    spread_body<NCH, T>(plan_of(plans, w.t), w.g0);
}

// ---------------------------------------------------------------------------
// Spreading on the matrix cores (FP64), for items whose points reach the grid
// from at most kSpreadAnchors first cells (dense items: many points per cell)
// and, in a launch of their own with room for more cell sums, from at most
// kSpreadAnchorsMed (medium items: tens of points per cell).
// With the points of an item split by their first cell a (anchor), the
// item's partial subgrid is
//   G[a + t][col] = sum over anchors a, over points k with anchor a, of
//                   phi_t(s_k) V_k[col],
// t the tap (0 .. w-1), phi_t the kernel's polynomial piece for tap t and
// V_k[2p + {0,1}] = (re, im) of c_k sqrt(q_k) e^{i D (r_k - C)} q_k^p.  For
// each anchor this is a (16 taps) x (points) x (16 NCT columns) product: one
// v_mfma_f64_16x16x4f64 per four points and column tile.  In an MFMA step,
// lane (row = lane % 16, k = lane / 16) supplies A[row][k] = phi_row(s) of
// point k, evaluated in the lane with the coefficients of piece `row` held in
// its registers, and B[k][col] = V_k[col] (col = lane % 16) from LDS; element
// v of the accumulator is D[lane / 16 + 4 v][lane % 16].
//
// The four waves of a workgroup share one item: wave v takes the steps of 64
// points starting at ka + (4 j + v) 64.  Points are sorted, so the anchors a
// wave meets only increase: it keeps one tile for its current anchor and adds
// it into its own cell sums in LDS when the anchor changes.  At the end the
// four waves' cell sums are added in a fixed order, so the result does not
// depend on timing.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

// 16-column tiles of the channel columns (re, im of 8 channels each): one
// to four, channel counts up to kMfmaMaxChannels
template <int NCH>
constexpr int kSpreadTiles = (2 * NCH + 15) / 16;

template <int NCH, int ANCH = kSpreadAnchors>
struct SpreadMfma {
    static constexpr int NCT = kSpreadTiles<NCH>;
    static constexpr int NC = 16 * NCT;            // real columns of the tiles (re, im of 8 NCT channels)
    static constexpr int VS = 2 * NCH + 1;         // LDS stride of a point's 2 NCH columns (odd: conflict-free writes)
    static constexpr int GC = ANCH + 15;           // cells an item's anchor tiles reach
    // points per step: 64, 32 with two column tiles, 16 with three or four,
    // so that the wider point records still fit (three workgroups per compute
    // unit at two tiles, two at four)
    static constexpr int WPTS = NCT > 2 ? 16 : NCT > 1 ? 32 : 64;
    // a point: its columns, its s and its anchor
    static constexpr size_t point_bytes = (VS + 1) * sizeof(double) + sizeof(int32_t);
    static constexpr size_t fold_bytes = (size_t)GC * NC * sizeof(double);   // the wave's cell sums
    static constexpr size_t wave_bytes = ((size_t)WPTS * point_bytes + 15) / 16 * 16 + fold_bytes;
    static constexpr size_t lds_bytes = 4 * wave_bytes;   // the workgroup's four waves
};

// Orders the LDS accesses of the wave's lanes around it (the region is
// written and read by different lanes of the same wave).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Points g_lo .. g_hi-1 of the step (g_lo a multiple of 8) into the tile of
// anchor a, two groups of four points per iteration (two independent kernel
// evaluations).  Lanes past np take B = 0; with MASK, points of other anchors
// take A = 0.
template <int NCH, bool MASK>
__device__ __forceinline__ void spread_mfma_run(v4d (&acc)[kSpreadTiles<NCH>], const double* s_v,
                                                const double* s_s, const int32_t* s_d,
                                                const double (&cf)[kEsDeg + 1], int g_lo, int g_hi, int np,
                                                int col, int kq, int a)
{
    constexpr int NCT = SpreadMfma<NCH>::NCT, VS = SpreadMfma<NCH>::VS;
    for (int g = g_lo; g < g_hi; g += 8) {
        const int i0 = g + kq, i1 = g + 4 + kq;
        const bool v0 = i0 < np, v1 = i1 < np;
        const int j0 = v0 ? i0 : g, j1 = v1 ? i1 : g;
        double b0[NCT], b1[NCT];
        #pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const bool on = ct * 16 + 16 <= 2 * NCH || ct * 16 + col < 2 * NCH;   // columns past 2 NCH are zero
            b0[ct] = (v0 && on) ? s_v[j0 * VS + ct * 16 + col] : 0.0;
            b1[ct] = (v1 && on) ? s_v[j1 * VS + ct * 16 + col] : 0.0;
        }
        const double s0 = s_s[j0], s1 = s_s[j1];
        double p0 = cf[kEsDeg], p1 = cf[kEsDeg];
        #pragma unroll
        for (int q = kEsDeg - 1; q >= 0; --q) {
            p0 = __builtin_fma(p0, s0, cf[q]);
            p1 = __builtin_fma(p1, s1, cf[q]);
        }
        if (MASK) {
            if (s_d[j0] != a) p0 = 0.0;
            if (s_d[j1] != a) p1 = 0.0;
        }
        #pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(p0, b0[ct], acc[ct], 0, 0, 0);
            acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(p1, b1[ct], acc[ct], 0, 0, 0);
        }
    }
}

// A full step of one anchor: all WPTS points valid and none masked, the same
// products in the same order as spread_mfma_run.  The loop is unrolled, so
// every LDS offset is a constant and no point needs a validity test.
template <int NCH>
__device__ __forceinline__ void spread_mfma_run_full(v4d (&acc)[kSpreadTiles<NCH>], const double* s_v,
                                                     const double* s_s, const double (&cf)[kEsDeg + 1], int col,
                                                     int kq)
{
    constexpr int NCT = SpreadMfma<NCH>::NCT, VS = SpreadMfma<NCH>::VS, WPTS = SpreadMfma<NCH>::WPTS;
    const double* v = s_v + kq * VS + col;
    const double* sp = s_s + kq;
    #pragma unroll
    for (int g = 0; g < WPTS; g += 8) {
        double b0[NCT], b1[NCT];
        #pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const bool on = ct * 16 + 16 <= 2 * NCH || ct * 16 + col < 2 * NCH;   // columns past 2 NCH are zero
            b0[ct] = on ? v[g * VS + ct * 16] : 0.0;
            b1[ct] = on ? v[(g + 4) * VS + ct * 16] : 0.0;
        }
        const double s0 = sp[g], s1 = sp[g + 4];
        double p0 = cf[kEsDeg], p1 = cf[kEsDeg];
        #pragma unroll
        for (int q = kEsDeg - 1; q >= 0; --q) {
            p0 = __builtin_fma(p0, s0, cf[q]);
            p1 = __builtin_fma(p1, s1, cf[q]);
        }
        #pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(p0, b0[ct], acc[ct], 0, 0, 0);
            acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(p1, b1[ct], acc[ct], 0, 0, 0);
        }
    }
}

// Adds the finished tile of anchor a into the wave's cell sums (row t of the
// tile to cell a + t) and clears it.
template <int NCH>
__device__ __forceinline__ void spread_mfma_flush(v4d (&acc)[kSpreadTiles<NCH>], double* s_g, int col, int kq, int a)
{
    constexpr int NCT = SpreadMfma<NCH>::NCT, NC = SpreadMfma<NCH>::NC;
    #pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
        #pragma unroll
        for (int v = 0; v < 4; ++v) s_g[(a + kq + 4 * v) * NC + ct * 16 + col] += acc[ct][v];
        acc[ct] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    wave_sync();   // the next anchor's cells overlap this one's in other lanes
}

// Item alist[slot] of the plan, with LDS for anchors up to ANCH.
template <int NCH, int ANCH>
__device__ __forceinline__ void spread_mfma_item(const PlanDev& P, int slot, double4* spread_lds)
{
    const double* __restrict__ cs = P.cs;
    const double* __restrict__ es_poly = P.es_poly;
    double2* __restrict__ part = P.part;
    using SM = SpreadMfma<NCH, ANCH>;
    constexpr int NCT = SM::NCT, NC = SM::NC, VS = SM::VS, WPTS = SM::WPTS, GC = SM::GC;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    char* base = reinterpret_cast<char*>(spread_lds) + wave * SM::wave_bytes;
    double* s_v = reinterpret_cast<double*>(base);
    double* s_s = s_v + WPTS * VS;
    int32_t* s_d = reinterpret_cast<int32_t*>(s_s + WPTS);
    double* s_g = reinterpret_cast<double*>(base + SM::wave_bytes - SM::fold_bytes);
    const Item I = P.aitems[P.alist[slot]];
    const ABlock B = P.ab[I.blk];
    const int col = lane & 15, kq = lane >> 4;
    const int w = P.w;
    const double hw = 0.5 * w;
    const double inv_h = 1.0 / B.h;      // exact: h is a power of two
    // polynomial piece of tap `col` (row col of A); rows at or beyond w are zero
    double cf[kEsDeg + 1];
    #pragma unroll
    for (int d = 0; d <= kEsDeg; ++d) cf[d] = col < w ? es_poly[col * (kEsDeg + 1) + d] : 0.0;
    for (int e = lane; e < GC * NC; e += 64) s_g[e] = 0.0;
    v4d acc[NCT];
    #pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[ct] = v4d{0.0, 0.0, 0.0, 0.0};
    int cur = -1;                              // anchor of the tile in acc
    // the next step's point and weight are loaded while the current one is
    // multiplied
    int k0 = I.ka + wave * WPTS;
    double r_nx = 0.0, c_nx = 0.0;
    if (k0 + lane < I.kb) { r_nx = P.rs[k0 + lane]; c_nx = cs[k0 + lane]; }
    for (; k0 < I.kb; k0 += 4 * WPTS) {
        const int np = (I.kb - k0) < WPTS ? (I.kb - k0) : WPTS;
        const double r = r_nx, c = c_nx;
        const int kn = k0 + 4 * WPTS + lane;
        if (kn < I.kb) { r_nx = P.rs[kn]; c_nx = cs[kn]; }
        wave_sync();                              // the previous step's reads of the region are done
        int dm = 0;
        if (lane < np) {
            const PointEval e = eval_point(B, r, c, inv_h, hw);
            dm = e.l0 - I.sub_lo;
            s_d[lane] = dm;
            s_s[lane] = e.s;
            double vr = e.wr, vi = e.wi;
            double* v = s_v + lane * VS;
            #pragma unroll
            for (int p = 0; p < NCH; ++p) {
                v[2 * p] = vr;
                v[2 * p + 1] = vi;
                vr *= e.q;
                vi *= e.q;
            }
        }
        wave_sync();
        // the step's anchors run from its first point's to its last point's
        const int a_lo = __builtin_amdgcn_readfirstlane(dm);
        const int a_hi = __builtin_amdgcn_readlane(dm, np - 1);
        if (a_lo == a_hi) {
            if (a_lo != cur) {
                if (cur >= 0) spread_mfma_flush<NCH>(acc, s_g, col, kq, cur);
                cur = a_lo;
            }
            if (np == WPTS) spread_mfma_run_full<NCH>(acc, s_v, s_s, cf, col, kq);
            else spread_mfma_run<NCH, false>(acc, s_v, s_s, s_d, cf, 0, np, np, col, kq, cur);
        } else {
            // the points of anchor a are consecutive lanes (points are sorted):
            // only the groups of eight that hold them are multiplied
            for (int a = a_lo; a <= a_hi; ++a) {
                const uint64_t mine = __ballot(lane < np && dm == a);
                if (mine == 0) continue;
                if (a != cur) {
                    if (cur >= 0) spread_mfma_flush<NCH>(acc, s_g, col, kq, cur);
                    cur = a;
                }
                const int first = __builtin_ctzll(mine), last = 63 - __builtin_clzll(mine);
                spread_mfma_run<NCH, true>(acc, s_v, s_s, s_d, cf, first & ~7, last + 1, np, col, kq, a);
            }
        }
    }
    if (cur >= 0) spread_mfma_flush<NCH>(acc, s_g, col, kq, cur);
    __syncthreads();
    // item partial [cell][channel] (re, im): waves summed in order
    const double* g0 = reinterpret_cast<const double*>(reinterpret_cast<char*>(spread_lds) + SM::wave_bytes -
                                                       SM::fold_bytes);
    constexpr size_t wstride = SM::wave_bytes / sizeof(double);
    double* out = reinterpret_cast<double*>(part + I.off);
    constexpr int row_len = 2 * NCH;
    for (int e = tid; e < I.sub_n * row_len; e += 256) {
        const int cell = e / row_len, c = e - cell * row_len;
        const int k = cell * NC + c;
        out[e] = ((g0[k] + g0[wstride + k]) + g0[2 * wstride + k]) + g0[3 * wstride + k];
    }
}

// Up to 8 channels (one column tile) the dense kernel fits four waves per
// SIMD, with two tiles three.  ANCH = kSpreadAnchors: the dense items, from
// slot 0 of the item list; kSpreadAnchorsMed: the medium ones, after them.
template <int NCH, int ANCH>
__global__ __launch_bounds__(256) void k_spread_mfma(PlanDev P)
{
    __shared__ double4 lds[SpreadMfma<NCH, ANCH>::lds_bytes / sizeof(double4)];
    const int first = ANCH == kSpreadAnchors ? 0 : P.n_adense;
    spread_mfma_item<NCH, ANCH>(P, first + blockIdx.x, lds);
}

template <int NCH, int ANCH>
__global__ __launch_bounds__(256) void k_spread_mfma_many(const PlanDev* __restrict__ plans,
                                                          const WorkSeg* __restrict__ segs, int nseg)
{
    __shared__ double4 lds[SpreadMfma<NCH, ANCH>::lds_bytes / sizeof(double4)];
    const WorkSeg w = find_seg(segs, nseg);
    const PlanDev& P = plan_of(plans, w.t);
    const int first = ANCH == kSpreadAnchors ? 0 : P.n_adense;
    spread_mfma_item<NCH, ANCH>(P, first + w.g0, lds);
}

// ---------------------------------------------------------------------------
// Grid assembly: each grid slot sums the item partials that cover it, in item
// order, and multiplies channel p by its factor beta_p (the Hankel coefficient
// with the sign and the factor i the combination step gives it), so that the
// row pass only sums the channels weighted by powers of 1/(om r0).
// Direct-sum-path grids are stored cell-major [cell][channel].  FFT
// path: mode l of the spread grid is divided by the inner kernel's transform
// psi^(l) = alpha2 ES^(|l| alpha2), alpha2 = w pi / N2 (the deconvolution of the
// type-2 step) and placed at FFT index l mod N2, channel-major [channel][N2];
// all other FFT inputs are zero.
// ---------------------------------------------------------------------------
// Partial i as double2: PT is double2, or float2 in the FP32-spreading mode
// (widened here, so the grids are assembled in FP64).
template <typename PT>
__device__ __forceinline__ double2 load_partial(const double2* __restrict__ part, int64_t i)
{
    PT v = reinterpret_cast<const PT*>(part)[i];
    return make_double2((double)v.x, (double)v.y);
}

template <typename PT>
__device__ __forceinline__ void spread_reduce_body(const PlanDev& P, int bid)
{
    const double2* __restrict__ part = P.part;
    double2* __restrict__ grids = P.grids;
    int64_t t = (int64_t)bid * blockDim.x + threadIdx.x;
    const int nch = P.nch;
    const int64_t total = P.grid_cells * nch;
    // Block owning a slot: the last block b with gslot[b] <= slot.  The wave
    // searches once for the slot of its first lane (uniform, through the scalar
    // unit); a wave spans at most 64 slots, so each lane then steps forward
    // over the few blocks that start inside that span.
    int64_t t0 = (int64_t)bid * blockDim.x + (threadIdx.x & ~63);
    int64_t slot0 = __builtin_amdgcn_readfirstlane((int32_t)((t0 < total ? t0 : total - 1) / nch));
    int32_t lo = 0, hi = P.n_a - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (P.gslot[mid] <= slot0) lo = mid; else hi = mid - 1;
    }
    // the wave's last slot: when it lies in the same block as the first, the
    // block's fields are read once through the scalar unit
    const int64_t tl = t0 + 63 < total ? t0 + 63 : total - 1;
    const int64_t slot_last = __builtin_amdgcn_readfirstlane((int32_t)(tl / nch));
    const bool one_block = P.gslot[lo + 1] > slot_last;
    if (t >= total) return;
    int64_t slot = t / nch;
    int p = (int)(t % nch);
    while (P.gslot[lo + 1] <= slot) ++lo;
    const ABlock B = one_block ? P.ab[__builtin_amdgcn_readfirstlane(lo)] : P.ab[lo];
    int64_t local = slot - P.gslot[lo];
    int32_t l;
    if (B.fft) l = local < B.N2 / 2 ? (int32_t)local : (int32_t)(local - B.N2);
    else l = B.llo + (int32_t)local;
    double sr = 0.0, si = 0.0;
    if (l >= B.llo && l < B.llo + B.N1) {
        // Items covering cell l: both ends of the items' cell ranges increase
        // with the item index, so they form one run [a, b): a is the first item
        // ending after l, b the first starting after l.  With the run known the
        // partials are loaded several at a time and still added in item order.
        const int32_t i0 = B.item0, i1 = B.item0 + B.nitems;
        int32_t a = i0, hi = i1;
        while (a < hi) {
            int32_t mid = (a + hi) >> 1;
            const Item& I = P.aitems[mid];
            if (I.sub_lo + I.sub_n <= l) a = mid + 1; else hi = mid;
        }
        // b: up to four steps forward from a (where points are spread out a
        // cell lies in the subgrids of one or two items), then a binary
        // search over the rest (where a block's points crowd a few cells,
        // dozens of items cover each)
        int32_t b = a;
        for (int k = 0; k < 4 && b < i1 && P.aitems[b].sub_lo <= l; ++k) ++b;
        if (b < i1 && P.aitems[b].sub_lo <= l) {
            hi = i1;
            ++b;
            while (b < hi) {
                int32_t mid = (b + hi) >> 1;
                if (P.aitems[mid].sub_lo <= l) b = mid + 1; else hi = mid;
            }
        }
        int32_t it = a;
        for (; it + 16 <= b; it += 16) {
            double2 v[16];
            #pragma unroll
            for (int q = 0; q < 16; ++q) {
                const Item& I = P.aitems[it + q];
                v[q] = load_partial<PT>(part, I.off + (int64_t)(l - I.sub_lo) * nch + p);
            }
            #pragma unroll
            for (int q = 0; q < 16; ++q) { sr += v[q].x; si += v[q].y; }
        }
        for (; it + 4 <= b; it += 4) {
            double2 v[4];
            #pragma unroll
            for (int q = 0; q < 4; ++q) {
                const Item& I = P.aitems[it + q];
                v[q] = load_partial<PT>(part, I.off + (int64_t)(l - I.sub_lo) * nch + p);
            }
            #pragma unroll
            for (int q = 0; q < 4; ++q) { sr += v[q].x; si += v[q].y; }
        }
        for (; it < b; ++it) {
            const Item& I = P.aitems[it];
            double2 v = load_partial<PT>(part, I.off + (int64_t)(l - I.sub_lo) * nch + p);
            sr += v.x;
            si += v.y;
        }
    }
    // channel factor: real for even p, i times real for odd p
    double f = P.chan[p];
    double2 v = (p & 1) ? make_double2(-si * f, sr * f) : make_double2(sr * f, si * f);
    if (B.fft) {
        double a2 = P.w * kPi / B.N2;
        double s = 1.0 / (a2 * eshat(P, fabs((double)l) * a2));
        grids[B.grid_off + (int64_t)p * B.N2 + local] = make_double2(v.x * s, v.y * s);
    } else {
        grids[B.grid_off + local * nch + p] = v;
    }
}

template <typename PT>
__global__ void k_spread_reduce(PlanDev P)
{
    spread_reduce_body<PT>(P, blockIdx.x);
}

template <typename PT>
__global__ void k_spread_reduce_many(const PlanDev* __restrict__ plans, const WorkSeg* __restrict__ segs, int nseg)
{
    const WorkSeg w = find_seg(segs, nseg);
    spread_reduce_body<PT>(plan_of(plans, w.t), w.g0);
}

// Transforms of N <= 4096 points, every size class of the transform in one
// launch (P.small).
__device__ __forceinline__ void fft_small_body(const PlanDev& P, int g)
{
    extern __shared__ double2 sm[];
    const SmallFfts& F = P.small;
    double2* __restrict__ grids = P.grids;
    int c = 0;
    while (c + 1 < F.n && g >= F.wg0[c + 1]) ++c;
    const int logN = F.log2n[c], N = 1 << logN;
    const int nch = P.nch;
    const int loc = g - F.wg0[c];
    const int slot = loc / nch, ch = loc % nch;
    const ABlock B = P.ab[P.fft_list[F.first[c] + slot]];
    double2* x = grids + B.grid_off + (int64_t)ch * N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) sm[i] = x[i];
    __syncthreads();
    lds_fft(sm, N, logN, 1, 0, 1);
    for (int i = threadIdx.x; i < N; i += blockDim.x) x[i] = sm[i];
}

__global__ __launch_bounds__(256) void k_fft_small(PlanDev P) { fft_small_body(P, blockIdx.x); }

__global__ __launch_bounds__(256) void k_fft_small_many(const PlanDev* __restrict__ plans,
                                                        const WorkSeg* __restrict__ segs, int nseg)
{
    const WorkSeg w = find_seg(segs, nseg);
    fft_small_body(plan_of(plans, w.t), w.g0);
}

// Transforms of N = 2^13 .. 2^24 points run as two or three passes, each a
// batch of transforms of length L <= 256 done in LDS.  A workgroup holds a
// tile of `lines` batches side by side (lines * L <= kFftTilePts), chosen so
// that every global read and write moves runs of `lines` consecutive elements
// (128 B or more) even where the transform itself is strided.
//
// With n = n1 + N1 n2 and k = k2 + N2 k1 (N = N1 N2),
//   X[k2 + N2 k1] = sum_n1 w_N1^(n1 k1) w_N^(n1 k2) sum_n2 x[n1 + N1 n2] w_N2^(n2 k2),
// w_M = e^(2 pi i / M).  The inner transform over n2 is a column pass (batches
// n1 at unit stride, the transform at stride N1) that also applies
// w_N^(n1 k2); the outer one is a row pass (the transform contiguous, output
// written at stride N2).  When N2 = Na Nb is longer than 256 it is split the
// same way (n2 = na + Na nb, k2 = kb + Nb ka) into two column passes: over nb
// with w_N2^(na kb), in place, then over na, which applies w_N^(n1 k2) and
// writes n1 + N1 k2.  Column passes read the grid and the second writes the
// scratch buffer; the row pass reads the scratch buffer and writes the grid.
constexpr int kFftTilePts = 2048;
constexpr int kFftMaxLines = 16;

// Twiddles, kept per device: entries 0..4095 hold e^(2 pi i j / 4096) and
// entries 4096..8191 hold e^(2 pi i j / 2^24), so that
// w_N^e = T[E >> 12] T[4096 + (E & 4095)] with E = (e mod N) 2^(24 - log2 N).
__device__ __forceinline__ double2 fft_twiddle(const double2* __restrict__ T, int64_t e, int logN)
{
    int64_t E = (e & ((int64_t(1) << logN) - 1)) << (kMaxFftLog2 - logN);
    return cmul(T[E >> 12], T[4096 + (E & 4095)]);
}

// In-LDS transforms of the tile's lines, Stockham radix 4 (one radix-2 stage
// first when log2 L is odd); element (line, n) at sm[line * ls + n].  tw holds
// w_L^j for j < L.
__device__ void lds_fft_lines(double2* sm, int logL, int lines, int ls, const double2* tw)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int L = 1 << logL;
    int Ns = 1, logNs = 0;
    if (logL & 1) {
        const int half = L >> 1, nb = lines * half;
        double2 v[kFftTilePts / 2 / 256][2];
        #pragma unroll
        for (int c = 0; c < kFftTilePts / 2 / 256; ++c) {
            int b = tid + c * nt;
            if (b < nb) {
                int line = b >> (logL - 1), j = b & (half - 1);
                v[c][0] = sm[line * ls + j];
                v[c][1] = sm[line * ls + j + half];
            }
        }
        __syncthreads();
        #pragma unroll
        for (int c = 0; c < kFftTilePts / 2 / 256; ++c) {
            int b = tid + c * nt;
            if (b < nb) {
                int line = b >> (logL - 1), j = b & (half - 1);
                double2 a = v[c][0], d = v[c][1];
                sm[line * ls + 2 * j] = make_double2(a.x + d.x, a.y + d.y);
                sm[line * ls + 2 * j + 1] = make_double2(a.x - d.x, a.y - d.y);
            }
        }
        __syncthreads();
        Ns = 2; logNs = 1;
    }
    const int q4 = L >> 2, nb = lines * q4;
    while (Ns < L) {
        double2 v[kFftTilePts / 4 / 256][4];
        #pragma unroll
        for (int c = 0; c < kFftTilePts / 4 / 256; ++c) {
            int b = tid + c * nt;
            if (b < nb) {
                int line = b >> (logL - 2), j = b & (q4 - 1);
                #pragma unroll
                for (int r = 0; r < 4; ++r) v[c][r] = sm[line * ls + j + r * q4];
            }
        }
        __syncthreads();
        #pragma unroll
        for (int c = 0; c < kFftTilePts / 4 / 256; ++c) {
            int b = tid + c * nt;
            if (b < nb) {
                int line = b >> (logL - 2), j = b & (q4 - 1);
                int k = j & (Ns - 1);
                int ti = k << (logL - 2 - logNs);          // w1 = e^(2 pi i k / (4 Ns)) = w_L^ti
                double2 w1 = tw[ti], w2 = tw[2 * ti], w3 = tw[3 * ti];
                double2 x0 = v[c][0];
                double2 x1 = cmul(v[c][1], w1);
                double2 x2 = cmul(v[c][2], w2);
                double2 x3 = cmul(v[c][3], w3);
                double2 a0 = make_double2(x0.x + x2.x, x0.y + x2.y);
                double2 a1 = make_double2(x0.x - x2.x, x0.y - x2.y);
                double2 a2 = make_double2(x1.x + x3.x, x1.y + x3.y);
                double2 a3 = make_double2(-(x1.y - x3.y), x1.x - x3.x);   // i (x1 - x3)
                int d0 = (j - k) * 4 + k;
                sm[line * ls + d0] = make_double2(a0.x + a2.x, a0.y + a2.y);
                sm[line * ls + d0 + Ns] = make_double2(a1.x + a3.x, a1.y + a3.y);
                sm[line * ls + d0 + 2 * Ns] = make_double2(a0.x - a2.x, a0.y - a2.y);
                sm[line * ls + d0 + 3 * Ns] = make_double2(a1.x - a3.x, a1.y - a3.y);
            }
        }
        __syncthreads();
        Ns <<= 2; logNs += 2;
    }
}

// A column pass.  Batch (b_lo, b_hi), b_lo < blo at unit stride; input element
// t at b_lo + b_hi in_hs + t in_es, output element k at
// b_lo + b_hi out_hs + k out_es, multiplied by w_N^e,
// e = (b_lo & lo_mask) (b_hi + kmul k).
struct FftCol {
    int32_t logL, logLines, logBlo, to_scratch;
    int64_t in_es, in_hs, out_es, out_hs, lo_mask, kmul;
};

// One pass over one size class of a transform: the class's first FFT-list
// slot, log2 of its FFT size, its offset in the scratch buffer, and the pass
// (for the row pass only C.logL = log2 N1 and C.logLines are used).
struct FftPass {
    int32_t first, logN;
    int64_t scratch_off;
    FftCol C;
};

// A transform's share of a batched FFT pass launch.
struct FftSeg {
    int32_t t, g0;
    FftPass F;
};

__device__ __forceinline__ void fft_stage_twiddles(double2* tw, const double2* __restrict__ T, int logL)
{
    for (int j = threadIdx.x; j < (1 << logL); j += blockDim.x) tw[j] = T[j << (12 - logL)];
}

__device__ __forceinline__ void fft_col_body(const PlanDev& P, int bid, const FftPass& F)
{
    double2* __restrict__ grids = P.grids;
    double2* __restrict__ scratch = P.scratch;
    const double2* __restrict__ T = P.fft_tw;
    const int first = F.first, logN = F.logN;
    const int64_t scratch_off = F.scratch_off;
    const FftCol& C = F.C;
    extern __shared__ double2 sm[];
    const int L = 1 << C.logL, lines = 1 << C.logLines, ls = L + 1;
    double2* tw = sm + lines * ls;
    const int tile = lines << C.logL;
    const int64_t N = int64_t(1) << logN;
    const int groups = (int)(N >> (C.logL + C.logLines));
    const int nch = P.nch;
    int tr = bid / groups, grp = bid - tr * groups;
    int slot = tr / nch, ch = tr - slot * nch;
    const ABlock B = P.ab[P.fft_list[first + slot]];
    const double2* x = grids + B.grid_off + (int64_t)ch * N;
    double2* y = C.to_scratch ? scratch + scratch_off + (int64_t)tr * N : grids + B.grid_off + (int64_t)ch * N;
    const int64_t bb = (int64_t)grp << C.logLines;
    const int64_t blo0 = bb & ((int64_t(1) << C.logBlo) - 1), bhi = bb >> C.logBlo;
    const double2* xs = x + blo0 + bhi * C.in_hs;
    constexpr int kPer = kFftTilePts / 256;
    double2 v[kPer];
    #pragma unroll
    for (int u = 0; u < kPer; ++u) {
        int e = threadIdx.x + u * 256;
        if (e < tile) v[u] = xs[(int64_t)(e >> C.logLines) * C.in_es + (e & (lines - 1))];
    }
    fft_stage_twiddles(tw, T, C.logL);
    #pragma unroll
    for (int u = 0; u < kPer; ++u) {
        int e = threadIdx.x + u * 256;
        if (e < tile) sm[(e & (lines - 1)) * ls + (e >> C.logLines)] = v[u];
    }
    __syncthreads();
    lds_fft_lines(sm, C.logL, lines, ls, tw);
    double2* ys = y + blo0 + bhi * C.out_hs;
    #pragma unroll
    for (int u = 0; u < kPer; ++u) {
        int e = threadIdx.x + u * 256;
        if (e < tile) {
            int k = e >> C.logLines, li = e & (lines - 1);
            double2 w = fft_twiddle(T, ((blo0 + li) & C.lo_mask) * (bhi + C.kmul * k), logN);
            ys[(int64_t)k * C.out_es + li] = cmul(sm[li * ls + k], w);
        }
    }
}

__global__ __launch_bounds__(256) void k_fft_col(PlanDev P, FftPass F) { fft_col_body(P, blockIdx.x, F); }

__global__ __launch_bounds__(256) void k_fft_col_many(const PlanDev* __restrict__ plans,
                                                      const FftSeg* __restrict__ segs, int nseg)
{
    const int s = find_seg_index(segs, nseg);
    fft_col_body(plan_of(plans, segs[s].t), (int)blockIdx.x - segs[s].g0, segs[s].F);
}

// The row pass: batch k2 < N2 of length L = N1 read contiguously at k2 N1 from
// the scratch buffer; output k1 written to the grid at k2 + N2 k1.
__device__ __forceinline__ void fft_row_body(const PlanDev& P, int bid, const FftPass& F)
{
    double2* __restrict__ grids = P.grids;
    const double2* __restrict__ scratch = P.scratch;
    const double2* __restrict__ T = P.fft_tw;
    const int first = F.first, logN = F.logN, logL = F.C.logL, logLines = F.C.logLines;
    const int64_t scratch_off = F.scratch_off;
    extern __shared__ double2 sm[];
    const int L = 1 << logL, lines = 1 << logLines, ls = L + 1;
    double2* tw = sm + lines * ls;
    const int tile = lines << logL;
    const int64_t N = int64_t(1) << logN, N2 = N >> logL;
    const int groups = (int)(N2 >> logLines);
    const int nch = P.nch;
    int tr = bid / groups, grp = bid - tr * groups;
    int slot = tr / nch, ch = tr - slot * nch;
    const ABlock B = P.ab[P.fft_list[first + slot]];
    const int64_t k20 = (int64_t)grp << logLines;
    const double2* xs = scratch + scratch_off + (int64_t)tr * N + (k20 << logL);
    double2* ys = grids + B.grid_off + (int64_t)ch * N + k20;
    constexpr int kPer = kFftTilePts / 256;
    double2 v[kPer];
    #pragma unroll
    for (int u = 0; u < kPer; ++u) {
        int e = threadIdx.x + u * 256;
        if (e < tile) v[u] = xs[e];
    }
    fft_stage_twiddles(tw, T, logL);
    #pragma unroll
    for (int u = 0; u < kPer; ++u) {
        int e = threadIdx.x + u * 256;
        if (e < tile) sm[(e >> logL) * ls + (e & (L - 1))] = v[u];
    }
    __syncthreads();
    lds_fft_lines(sm, logL, lines, ls, tw);
    #pragma unroll
    for (int u = 0; u < kPer; ++u) {
        int e = threadIdx.x + u * 256;
        if (e < tile) {
            int k1 = e >> logLines, li = e & (lines - 1);
            ys[(int64_t)k1 * N2 + li] = sm[li * ls + k1];
        }
    }
}

__global__ __launch_bounds__(256) void k_fft_row(PlanDev P, FftPass F) { fft_row_body(P, blockIdx.x, F); }

__global__ __launch_bounds__(256) void k_fft_row_many(const PlanDev* __restrict__ plans,
                                                      const FftSeg* __restrict__ segs, int nseg)
{
    const int s = find_seg_index(segs, nseg);
    fft_row_body(plan_of(plans, segs[s].t), (int)blockIdx.x - segs[s].g0, segs[s].F);
}

// ---------------------------------------------------------------------------
// Row side.
// ---------------------------------------------------------------------------

// Local block contribution at frequency om:  sum_{l=0}^{L} C_l(om R) t_l with
//   C_l(x) = delta_l J_{nu/2+l}(x/2) J_{nu/2-l}(x/2)        (nu even, reading x/2)
//   C_l(x) = 2 J_{(nu+1)/2+l}(x/2) J_{(nu-1)/2-l}(x/2)       (nu odd)
// J_k(y), y = om R / 2, comes from Miller's backward recurrence, started at N
// and normalised at the end by J_0^2 + 2 sum_k J_k^2 = 1.  Written with
// J_{-i} = (-1)^i J_i, the sum pairs index i with i + nu (the terms l > a,
// a = floor(nu/2), sign (-1)^i) and with nu - i (the terms l <= a).
//   MODE 0 (nu = 0): the products are J_i^2;
//   MODE 1 (nu = 1): J_i J_{i+1}, i.e. the current and the previous value;
//   MODE 2 (any nu): the partner nu steps back from a second copy of the
//   recurrence running behind the first; the floor(nu/2) + 1 partners of the
//   l <= a terms from LDS.
// In every mode the recurrence first runs alone down to the highest index a
// product needs, then continues with the products.
__device__ __forceinline__ void miller_rescale(double& yk, double& yk1, double& S2, double& dot)
{
    if (fabs(yk) > 1e100) { yk *= 1e-100; yk1 *= 1e-100; S2 *= 1e-200; dot *= 1e-200; }
}

// Once per four steps, for waves whose arguments are all >= kMillerGroupY: a
// step multiplies the values by at most 2N / y + 1 < 4.2e6 (start N <= 2048,
// the largest local rank allowed plus one), four steps by less than 3.1e26,
// so the values stay below 3.1e126 and their squares and sums finite.
constexpr double kMillerGroupY = 1e-3;
__device__ __forceinline__ void miller_rescale_group(double& yk, double& yk1, double& S2, double& dot)
{
    if (fmax(fabs(yk), fabs(yk1)) > 1e100) { yk *= 1e-100; yk1 *= 1e-100; S2 *= 1e-200; dot *= 1e-200; }
}

// Four consecutive local moments (8-byte aligned, read as one block).
struct Moments4 {
    double v[4];
};

template <int MODE>
__device__ double local_eval(const PlanDev& P, int lblk, double om, const double* __restrict__ lmom,
                             double* __restrict__ ring, int stride)
{
    const LBlock B = P.lb[lblk];
    double y = 0.5 * (om * B.R);
    const double* t = lmom + (int64_t)lblk * (P.L + 1);
    const int nu = MODE == 0 ? 0 : (MODE == 1 ? 1 : P.nu), L = P.L;
    if (y < 1e-30) return nu == 0 ? t[0] : 0.0;
    // the pairing reads J_{nu-i} for i <= nu/2, so the recurrence must have
    // produced every index up to nu; it also starts above every index a
    // product needs, so that the product phase runs over the same indices in
    // every lane (its index, and with it the moment loads, stay wave-uniform;
    // a higher start only makes the recurrence more accurate)
    int N = miller_start(y);
    if (N < nu + 1) N = nu + 1;
    {
        const int a_ = (MODE == 2 && (nu & 1)) ? (nu - 1) >> 1 : nu >> 1;
        const int top_ = MODE == 2 ? ((L - a_) > a_ ? (L - a_) : a_) : L;
        if (N < top_ + 1) N = top_ + 1;
    }
    const double rec = 2.0 / y;
    double yk1 = 0.0, yk = 1e-100, S2 = 0.0, dot = 0.0;
    if (MODE == 0) {
        // J_0^2 t_0 + sum_{i=1}^{L} 2 (-1)^i t_i J_i^2
        int i = N;
        // above L: the recurrence alone, with one rescale test per four
        // steps where the wave's arguments allow it (as in the grouped
        // steps below)
        auto lead = [&](int k) {
            S2 = __builtin_fma(2.0 * yk, yk, S2);
            double ykm1 = __builtin_fma((double)k * rec, yk, -yk1);
            yk1 = yk; yk = ykm1;
        };
        if (__all(y >= kMillerGroupY)) {
            for (; i - 3 > L; i -= 4) {
                lead(i); lead(i - 1); lead(i - 2); lead(i - 3);
                miller_rescale_group(yk, yk1, S2, dot);
            }
        }
        for (; i > L; --i) {
            lead(i);
            miller_rescale(yk, yk1, S2, dot);
        }
        i = L;   // where every lane left the loop (N > L): the index is now wave-uniform
        // i = L .. 1 in every lane (the start is above L): L mod 4 single
        // steps, then groups of four whose moments u[i-3 .. i] are read
        // together (u_i = 2 (-1)^i t_i)
        auto step = [&](int k, double uk, bool check) {
            double q = yk * yk;
            S2 = __builtin_fma(2.0, q, S2);
            dot = __builtin_fma(uk, q, dot);
            double ykm1 = __builtin_fma((double)k * rec, yk, -yk1);
            yk1 = yk; yk = ykm1;
            if (check) miller_rescale(yk, yk1, S2, dot);
        };
        for (int u = L & 3; u > 0; --u, --i) step(i, t[i], true);
        if (__all(y >= kMillerGroupY)) {
            // four steps grow the values by less than 1e27: one rescale test
            // per group, and the next group's moments in flight
            Moments4 nx;
            if (i >= 4) __builtin_memcpy(&nx, t + i - 3, sizeof nx);
            for (; i >= 4; i -= 4) {
                const Moments4 q = nx;
                if (i >= 8) __builtin_memcpy(&nx, t + i - 7, sizeof nx);
                step(i, q.v[3], false); step(i - 1, q.v[2], false);
                step(i - 2, q.v[1], false); step(i - 3, q.v[0], false);
                miller_rescale_group(yk, yk1, S2, dot);
            }
        } else {
            for (; i >= 4; i -= 4) {
                Moments4 q;
                __builtin_memcpy(&q, t + i - 3, sizeof q);
                step(i, q.v[3], true); step(i - 1, q.v[2], true); step(i - 2, q.v[1], true); step(i - 3, q.v[0], true);
            }
        }
        S2 = __builtin_fma(yk, yk, S2);
        dot = __builtin_fma(t[0] * yk, yk, dot);
        return dot / S2;
    } else if (MODE == 1) {
        // 2 t_0 J_0 J_1 + sum_{i=1}^{L} 2 (-1)^i t_i J_i J_{i+1}; yk1 = J_{i+1}
        int i = N;
        // above L: the recurrence alone, with one rescale test per four
        // steps where the wave's arguments allow it (as in the grouped
        // steps below)
        auto lead = [&](int k) {
            S2 = __builtin_fma(2.0 * yk, yk, S2);
            double ykm1 = __builtin_fma((double)k * rec, yk, -yk1);
            yk1 = yk; yk = ykm1;
        };
        if (__all(y >= kMillerGroupY)) {
            for (; i - 3 > L; i -= 4) {
                lead(i); lead(i - 1); lead(i - 2); lead(i - 3);
                miller_rescale_group(yk, yk1, S2, dot);
            }
        }
        for (; i > L; --i) {
            lead(i);
            miller_rescale(yk, yk1, S2, dot);
        }
        i = L;   // where every lane left the loop (N > L): the index is now wave-uniform
        auto step = [&](int k, double uk, bool check) {
            S2 = __builtin_fma(2.0 * yk, yk, S2);
            dot = __builtin_fma(uk * yk, yk1, dot);
            double ykm1 = __builtin_fma((double)k * rec, yk, -yk1);
            yk1 = yk; yk = ykm1;
            if (check) miller_rescale(yk, yk1, S2, dot);
        };
        for (int u = L & 3; u > 0; --u, --i) step(i, t[i], true);
        if (__all(y >= kMillerGroupY)) {
            Moments4 nx;
            if (i >= 4) __builtin_memcpy(&nx, t + i - 3, sizeof nx);
            for (; i >= 4; i -= 4) {
                const Moments4 q = nx;
                if (i >= 8) __builtin_memcpy(&nx, t + i - 7, sizeof nx);
                step(i, q.v[3], false); step(i - 1, q.v[2], false);
                step(i - 2, q.v[1], false); step(i - 3, q.v[0], false);
                miller_rescale_group(yk, yk1, S2, dot);
            }
        } else {
            for (; i >= 4; i -= 4) {
                Moments4 q;
                __builtin_memcpy(&q, t + i - 3, sizeof q);
                step(i, q.v[3], true); step(i - 1, q.v[2], true); step(i - 2, q.v[1], true); step(i - 3, q.v[0], true);
            }
        }
        S2 = __builtin_fma(yk, yk, S2);
        dot = __builtin_fma(2.0 * t[0] * yk, yk1, dot);
        return dot / S2;
    } else {
        // Part one pairs i with i + nu (1 <= i <= L - a, weight 2 (-1)^i t_{a+i});
        // part two pairs i with nu - i (0 <= i <= a, weight t_{a-i}, doubled
        // except the l = 0 term of an even order).  J_{i+nu} comes from a second
        // copy of the recurrence run nu steps behind the first: the same
        // operations on the same state give the same values, so the lagging
        // copy is started from the leading copy's state at s0 = min(N, L-a+nu)
        // and the two run as independent chains.  Part two's partners
        // J_{a2..nu} (a2 = nu - a) are kept per thread in LDS as the leading
        // copy passes them.  Both copies rescale by exact powers of two; the
        // leading copy's rescales since the lagging copy's state (d) set the
        // factor 2^(-332 d) between the two scales.
        const int odd = nu & 1;
        const int a = nu >> 1;
        const int a2 = nu - a;
        const double sa = (a & 1) ? -1.0 : 1.0;
        const int hi1 = L - a;
        const int top = hi1 > nu ? hi1 : nu;
        const int s0 = N < hi1 + nu ? N : hi1 + nu;
        const int act = s0 - nu;
        const double up = 0x1p332, down = 0x1p-332, down2 = 0x1p-664;
        // Here S2 holds half the normalising sum (J_0^2 / 2 + sum_{i>=1} J_i^2),
        // one FMA per step; the lagging copy starts (i == act) at one or two
        // steps of a wave, so that test is a wave vote first.
        double syk = yk, syk1 = 0.0;          // leading copy's state at s0
        double lyk = 0.0, lyk1 = 0.0, lsc = sa;   // lsc: (-1)^a 2^(-332 d)
        int d = 0;
        int i = N;
        auto lead = [&](int k) {
            if (k == s0) { syk = yk; syk1 = yk1; d = 0; lsc = sa; }
            S2 = __builtin_fma(yk, yk, S2);
            double ykm1 = __builtin_fma((double)k * rec, yk, -yk1);
            yk1 = yk; yk = ykm1;
        };
        auto lead_rescale = [&](bool group) {
            if ((group ? fmax(fabs(yk), fabs(yk1)) : fabs(yk)) > up) {
                yk *= down; yk1 *= down; S2 *= down2; dot *= down2;
                ++d; lsc = __builtin_amdgcn_ldexp(sa, -332 * d);
            }
        };
        if (__all(y >= kMillerGroupY)) {
            // one rescale test per four steps, as in the grouped steps below
            for (; i - 3 > top; i -= 4) {
                lead(i); lead(i - 1); lead(i - 2); lead(i - 3);
                lead_rescale(true);
            }
        }
        for (; i > top; --i) {
            lead(i);
            lead_rescale(false);
        }
        i = top;   // where every lane left the loop (N > top): the index is now wave-uniform
        // i = top .. 0 in every lane.  stepB takes the products at index i and
        // (i > 0) moves both copies one index down; rescaleB follows a step
        // whose last products were at index il (stored partners: indices il .. nu).
        auto stepB = [&](int i) {
            if (__any(i == act)) {
                if (i == act) { lyk = syk; lyk1 = syk1; }
            }
            S2 = __builtin_fma(i == 0 ? 0.5 * yk : yk, yk, S2);
            if (i >= a2 && i <= nu) ring[(i - a2) * stride] = yk;
            if (i >= 1 && i <= hi1) {
                // 2 (-1)^i t_{a+i} = (-1)^a u_{a+i}
                dot = __builtin_fma(t[a + i] * yk, lyk * lsc, dot);
            }
            if (i <= a && a - i <= L) {
                int l2 = a - i;
                double pv = ring[(nu - i - a2) * stride];
                // 2 t_l2 = (-1)^l2 u_l2 (l2 >= 1); t_0 = u_0
                double coef = l2 == 0 ? (odd ? 2.0 * t[0] : t[0]) : ((l2 & 1) ? -t[l2] : t[l2]);
                dot = __builtin_fma(coef * yk, pv, dot);
            }
            if (i > 0) {
                double ykm1 = __builtin_fma((double)i * rec, yk, -yk1);
                yk1 = yk; yk = ykm1;
                double lykm1 = __builtin_fma((double)(i + nu) * rec, lyk, -lyk1);
                lyk1 = lyk; lyk = lykm1;
            }
        };
        auto rescaleB = [&](int il, bool group) {
            const double ml = group ? fmax(fabs(yk), fabs(yk1)) : fabs(yk);
            if (ml > up) {
                yk *= down; yk1 *= down; S2 *= down2; dot *= down2;
                ++d; lsc = __builtin_amdgcn_ldexp(sa, -332 * d);
                for (int q = (il > a2 ? il : a2) - a2; q <= nu - a2; ++q) ring[q * stride] *= down;
            }
            const double mg = group ? fmax(fabs(lyk), fabs(lyk1)) : fabs(lyk);
            if (mg > up) {
                lyk *= down; lyk1 *= down;
                --d; lsc = __builtin_amdgcn_ldexp(sa, -332 * d);
            }
        };
        // Above nu (i = top .. nu + 1, present when hi1 > nu) a step has no
        // partner to store or read: only part one's product and the two
        // recurrences, so these steps skip stepB's index tests, and their
        // moments t[a + i] (contiguous, wave-uniform) come four at a time.
        auto stepA = [&](int i, double ti) {
            if (__any(i == act)) {
                if (i == act) { lyk = syk; lyk1 = syk1; }
            }
            S2 = __builtin_fma(yk, yk, S2);
            dot = __builtin_fma(ti * yk, lyk * lsc, dot);
            double ykm1 = __builtin_fma((double)i * rec, yk, -yk1);
            yk1 = yk; yk = ykm1;
            double lykm1 = __builtin_fma((double)(i + nu) * rec, lyk, -lyk1);
            lyk1 = lyk; lyk = lykm1;
        };
        const bool group = __all(y >= kMillerGroupY);
        if (group) {
            // one rescale test per four steps (growth below 3.1e26 per group);
            // the copies may rescale at different indices, d counts both
            Moments4 nx;
            if (i - 3 > nu) __builtin_memcpy(&nx, t + a + i - 3, sizeof nx);
            for (; i - 3 > nu; i -= 4) {
                const Moments4 q = nx;
                if (i - 7 > nu) __builtin_memcpy(&nx, t + a + i - 7, sizeof nx);
                stepA(i, q.v[3]); stepA(i - 1, q.v[2]); stepA(i - 2, q.v[1]); stepA(i - 3, q.v[0]);
                rescaleB(i - 3, true);
            }
        }
        for (; i > nu; --i) {
            stepA(i, t[a + i]);
            rescaleB(i, false);
        }
        if (group) {
            for (; i >= 4; i -= 4) {
                stepB(i); stepB(i - 1); stepB(i - 2); stepB(i - 3);
                rescaleB(i - 3, true);
            }
        }
        for (; i >= 0; --i) {
            stepB(i);
            if (i == 0) break;
            rescaleB(i, false);
        }
        return dot / (2.0 * S2);
    }
}

// Local block contribution at a half-integer order nu = n + 1/2, x = om R in
// [0, z]: from J_{n+1/2}(x y) = sqrt(y) sqrt(2x/pi) sum_l beta_{e+2l}(x) T_{e+2l}(y),
//   sqrt(2x/pi) sum_{l=0}^{L} beta_{e+2l}(x) t_l,   t_l = sum_k c_k sqrt(y_k) T_{e+2l}(y_k),
// with beta from the plan's table: panel p = floor(x / h), Horner's rule in the
// panel variable tau = 2 (x / h - p) - 1 for each l; the leading panels
// (below x = n + 10) hold beta / x^n, accurate relative to beta itself there.
__device__ double local_eval_half(const PlanDev& P, int lblk, double om, const double* __restrict__ lmom)
{
    const LBlock B = P.lb[lblk];
    const double x = om * B.R;
    const double* t = lmom + (int64_t)lblk * (P.L + 1);
    const double u = x * P.half_inv_h;
    int pn = (int)u;
    if (pn > P.half_np - 1) pn = P.half_np - 1;
    const double tau = 2.0 * (u - pn) - 1.0;
    const double* tab = P.half_tab + (int64_t)pn * (P.L + 1) * (kHalfDeg + 1);
    double acc = 0.0;
    for (int l = 0; l <= P.L; ++l) {
        const double* cf = tab + l * (kHalfDeg + 1);
        double b = cf[kHalfDeg];
        #pragma unroll
        for (int d = kHalfDeg - 1; d >= 0; --d) b = __builtin_fma(b, tau, cf[d]);
        acc = __builtin_fma(b, t[l], acc);
    }
    if (pn < P.half_ns && P.nu > 0) acc *= pow(x, (double)P.nu);
    return sqrt(2.0 * x / kPi) * acc;
}

// Asymptotic block contribution at frequency om (Sec. 3.2):
//   sqrt(2/pi) Re( e^{i phi} sum_p beta_p om^(-p-1/2) y_p ),
//   beta_{2l} = (-1)^l a_{2l},  beta_{2l+1} = i (-1)^l a_{2l+1},
// where y_p = sum_k x_k^(p) e^{i om r_k} is the type-3 sum of channel p.  With
// s' = om - D and theta = s' h:  y_p = e^{i om C} h F_p(theta) / phi^(s'),
// F_p(theta) = sum_l b_l^(p) e^{i l theta} evaluated directly over the cells
// (direct-sum path) or from the FFT by ES interpolation (FFT path).  The grids
// already hold beta_p b_l^(p), so with gamma = 1/(om r0) each cell (or tap)
// needs the single value sum_p gamma^p beta_p b_l^(p): two multiply-adds per
// channel.  On the direct-sum path the powers gamma^p are kept in registers
// (the grid value, when it comes through the scalar unit, is then a
// multiplicand and needs no copy into vector registers); on the FFT path the
// sum is Horner's rule in gamma.  One complex product per cell or tap.
// Called with a wave-uniform block index whenever every active lane of the
// wave is in the same block (the usual case, frequencies being sorted); the
// block's fields and its direct-sum grid are then read through the scalar
// unit and broadcast to all lanes.
// One Horner step of a direct-sum cell sum with the cell's channel-0 value
// (g0r, g0i) in scalar registers:
//   (ar, ai) <- (ar, ai) e^{i theta} + (g0r, g0i)
// in four FMAs, the scalar values as addends and ar, ai updated in place.
// The compiler would copy the two scalar values into vector registers first
// and move the results back into ar, ai (six more instructions per cell);
// the step is written out so that it does not.  Callers pass values that are
// the same in every lane.
__device__ __forceinline__ void rotate_add_uniform(double& ar, double& ai, double er, double ei, double g0r, double g0i)
{
    double t;
    asm("v_fma_f64 %2, %0, %4, %6\n\t"     // t  = ar ei + g0i
        "v_fma_f64 %0, %0, %3, %5\n\t"     // ar = ar er + g0r
        "v_fma_f64 %0, -%1, %4, %0\n\t"    // ar -= ai ei
        "v_fma_f64 %1, %1, %3, %2"           // ai = ai er + t
        : "+v"(ar), "+v"(ai), "=&v"(t)
        : "v"(er), "v"(ei), "s"(g0r), "s"(g0i));
}

// UNI: the block index, and so the block's fields and grid, is the same in
// every lane of the wave.
template <int NCH, bool UNI>
__device__ double asym_eval(const PlanDev& P, int ablk, double om, const double2* __restrict__ grids)
{
    const ABlock B = P.ab[ablk];
    const int w = P.w;
    // gamma = 1/(om r0) and its square root (om r0 > z > 0 on an asymptotic block)
    const double rs = rsqrt_refined(om * B.r0);
    const double gam = rs * rs;
    double gpow[NCH];
    gpow[0] = 1.0;
    #pragma unroll
    for (int p = 1; p < NCH; ++p) gpow[p] = gpow[p - 1] * gam;
    dd sp = two_sum(om, -B.D);
    double ar = 0.0, ai = 0.0;
    // final phase om C + phi (+ llo theta on the direct-sum path), double-double
    dd pc = two_prod(om, B.C);
    dd ph = two_sum(pc.hi, P.phi_hi);
    double ph_lo = ph.lo + pc.lo + P.phi_lo;
    if (!B.fft) {
        const double2* G = grids + B.grid_off;
        double th = sp.hi * B.h, tl = sp.lo * B.h;
        // the cell sum starts at l = llo: its factor e^{i llo theta} joins the
        // final phase, and the rotation starts at 1
        dd a0 = two_prod((double)B.llo, th);
        dd q = two_sum(ph.hi, a0.hi);
        ph.hi = q.hi;
        ph_lo += q.lo + __builtin_fma((double)B.llo, tl, a0.lo);
        double s1, c1;
        sincos_small(th, &s1, &c1);
        const double er = c1 - tl * s1, ei = s1 + tl * c1;
        // Horner's rule in e^{i theta} from the last cell down
        for (int cix = B.N1 - 1; cix >= 0; --cix) {
            // the channel sum with the powers of gamma as multiplicands (where
            // the block is uniform across the wave the grid values come in
            // scalar registers, and a scalar operand fits an FMA's
            // multiplicand with no copy)
            const double2* gp = G + (int64_t)cix * NCH;
            double2 gv[NCH];
            #pragma unroll
            for (int p = 0; p < NCH; ++p) gv[p] = gp[p];
            if constexpr (UNI) {
                // the rotation first, channel 0 its addend, then the other
                // channels straight into ar, ai
                rotate_add_uniform(ar, ai, er, ei, gv[0].x, gv[0].y);
                #pragma unroll
                for (int p = 1; p < NCH; ++p) {
                    ar = __builtin_fma(gv[p].x, gpow[p], ar);
                    ai = __builtin_fma(gv[p].y, gpow[p], ai);
                }
            } else {
                double br = gv[0].x, bi = gv[0].y;
                #pragma unroll
                for (int p = 1; p < NCH; ++p) {
                    br = __builtin_fma(gv[p].x, gpow[p], br);
                    bi = __builtin_fma(gv[p].y, gpow[p], bi);
                }
                const double tr = __builtin_fma(ar, er, __builtin_fma(-ai, ei, br));
                ai = __builtin_fma(ar, ei, __builtin_fma(ai, er, bi));
                ar = tr;
            }
        }
    } else {
        const double2* Aq = grids + B.grid_off;
        dd v = two_prod(sp.hi, B.Khi);
        double vl = v.lo + (sp.lo * B.Khi + sp.hi * B.Klo);
        int q0 = (int)ceil(v.hi - 0.5 * w);
        const int mask = B.N2 - 1;
        // Tap t sits at offset t + f0 - w/2 from the target, f0 in [0, 1).  Its
        // kernel value is piece t of the ES kernel at f0 (the pieces the
        // spreading uses, w x (kEsDeg + 1) monomial coefficients in 2 f - 1,
        // the same for every lane: each enters its FMA as the scalar addend).
        // Against exp and sqrt per tap this is a third of the instructions and
        // fewer registers.
        const double* __restrict__ es_poly = P.es_poly;
        const double sf = 2.0 * ((((double)q0 - v.hi) - vl) + 0.5 * w) - 1.0;
        for (int tap = 0; tap < w; ++tap) {
            int q = q0 + tap;
            int qi = q & mask;
            // the tap's channel values first, all loads in flight while the
            // kernel value is computed
            double2 gv[NCH];
            #pragma unroll
            for (int p = 0; p < NCH; ++p) gv[p] = Aq[(int64_t)p * B.N2 + qi];
            const double* cf = es_poly + tap * (kEsDeg + 1);
            double psi = cf[kEsDeg];
            #pragma unroll
            for (int d = kEsDeg - 1; d >= 0; --d) psi = fma_uniform_addend(psi, sf, cf[d]);
            // Horner's rule in gamma from the highest channel: the loaded values
            // (vector registers here) are the addends
            double br = gv[NCH - 1].x, bi = gv[NCH - 1].y;
            #pragma unroll
            for (int p = NCH - 2; p >= 0; --p) {
                br = __builtin_fma(br, gam, gv[p].x);
                bi = __builtin_fma(bi, gam, gv[p].y);
            }
            ar = __builtin_fma(psi, br, ar);
            ai = __builtin_fma(psi, bi, ai);
        }
        double sc = 2.0 * kPi / B.N2;
        ar *= sc;
        ai *= sc;
    }
    double kap = fabs(sp.hi) * B.alpha;
    double scale = B.h * rcp_refined(B.alpha * eshat(P, kap));
    double cr, ci;
    cis_dd(ph.hi, ph_lo, cr, ci);
    double amp = rs * scale;
    return kSqrt2OverPi * amp * __builtin_fma(cr, ar, -ci * ai);
}

// ---------------------------------------------------------------------------
// J_nu for the direct blocks.  Their entries lie along the curve omega r = z
// (every direct block straddles it at the finest subdivision level), so the
// plan carries a table of J_nu on panels of width kJtabWidth around z (built
// on the host in extended precision): per panel the degree-15 Chebyshev
// interpolant at the 16 Chebyshev points, stored as monomial coefficients in
// the panel coordinate u in [-1, 1].  Arguments outside the table take
// besselj_full.
// ---------------------------------------------------------------------------
// J_nu(xh + xl) from the table where it covers xh, else besselj_full.
__device__ __forceinline__ double besselj_direct(const PlanDev& P, double xh, double xl)
{
    const double t = (xh - P.jtab_x0) * (1.0 / kJtabWidth);
    if (t >= 0.0 && t < (double)P.jtab_np) {
        const int p = (int)t;
        // the panel's left end (exact), and xh - xs exactly (xs = 0 or xs <= xh <= 2 xs)
        const double xs = __builtin_fma((double)p, kJtabWidth, P.jtab_x0);
        const double u = ((xh - xs) - 1.0) + xl;
        const double2* __restrict__ c = (const double2*)(P.jtab + (int64_t)p * kJtabCoef);
        double2 a[kJtabCoef / 2];
        #pragma unroll
        for (int q = 0; q < kJtabCoef / 2; ++q) a[q] = c[q];
        double v = a[kJtabCoef / 2 - 1].y;
        #pragma unroll
        for (int q = kJtabCoef / 2 - 1; q >= 0; --q) {
            if (q < kJtabCoef / 2 - 1) v = __builtin_fma(v, u, a[q].y);
            v = __builtin_fma(v, u, a[q].x);
        }
        return v;
    }
    return besselj_full(P, xh, xl);
}

// Two entries' table values at once (both arguments on the table): the two
// panels' loads issue together and the two Horner chains interleave.
__device__ __forceinline__ bool on_jtab(const PlanDev& P, double xh)
{
    const double t = (xh - P.jtab_x0) * (1.0 / kJtabWidth);
    return t >= 0.0 && t < (double)P.jtab_np;
}

// The table's panels as (kJtabCoef / 2) double2 records, read from `tab`
// with a stride of STRIDE double2 per panel (global memory, or the LDS copy
// whose padded stride spreads consecutive panels over the banks).
template <int STRIDE, typename Tab>
__device__ __forceinline__ void besselj_table2(const PlanDev& P, Tab tab, double xh1, double xl1, double xh2,
                                               double xl2, double& j1, double& j2)
{
    const int p1 = (int)((xh1 - P.jtab_x0) * (1.0 / kJtabWidth));
    const int p2 = (int)((xh2 - P.jtab_x0) * (1.0 / kJtabWidth));
    const double u1 = ((xh1 - __builtin_fma((double)p1, kJtabWidth, P.jtab_x0)) - 1.0) + xl1;
    const double u2 = ((xh2 - __builtin_fma((double)p2, kJtabWidth, P.jtab_x0)) - 1.0) + xl2;
    const auto c1 = tab + p1 * STRIDE;
    const auto c2 = tab + p2 * STRIDE;
    double2 a[kJtabCoef / 2], b[kJtabCoef / 2];
    #pragma unroll
    for (int q = 0; q < kJtabCoef / 2; ++q) { a[q] = c1[q]; b[q] = c2[q]; }
    double v = a[kJtabCoef / 2 - 1].y, w = b[kJtabCoef / 2 - 1].y;
    #pragma unroll
    for (int q = kJtabCoef / 2 - 1; q >= 0; --q) {
        if (q < kJtabCoef / 2 - 1) {
            v = __builtin_fma(v, u1, a[q].y);
            w = __builtin_fma(w, u2, b[q].y);
        }
        v = __builtin_fma(v, u1, a[q].x);
        w = __builtin_fma(w, u2, b[q].x);
    }
    j1 = v;
    j2 = w;
}

// Direct blocks (entry by entry, J_nu to full precision).  One workgroup of
// kDirectThreads lanes per block: each row of the block is given G lanes (G a
// power of two up to 64, as many as fit), the lanes of a row sum strided
// entries and combine by shuffles.  A
// row lies in at most one direct block (the last block of its path down the
// subdivision tree), so the per-row sums are stored, not accumulated.
constexpr int kDirectThreads = 256;
// Tables of up to kJtabLdsPanels panels (z up to about 240 with the
// default range) are copied into LDS by each workgroup and read from there:
// shorter latency than the cache hierarchy for the eight 16-byte loads per
// entry.  A panel takes kJtabLdsStride double2 (one more than its
// coefficients), so that lanes on neighbouring panels read different banks.
constexpr int kJtabLdsPanels = 64;
constexpr int kJtabLdsStride = kJtabCoef / 2 + 1;

template <bool LDS>
__device__ __forceinline__ void direct_rows(const PlanDev& P, const DBlock& D, const double2* s_tab)
{
    const double* __restrict__ cs = P.cs;
    double* __restrict__ gd = P.gd;
    const int mb = D.j1 - D.j0 + 1, nb = D.k1 - D.k0 + 1;
    int G = 1;
    while (G < 64 && 2 * G * mb <= kDirectThreads) G <<= 1;
    const int rows_per_pass = kDirectThreads / G;
    const int lane = threadIdx.x;
    const int grp = lane / G, gl = lane & (G - 1);
    for (int r0 = 0; r0 < mb; r0 += rows_per_pass) {
        int i = r0 + grp;
        double acc = 0.0;
        if (i < mb) {
            double om = P.ws[D.j0 + i];
            // two entries per step (the lane's next two, in order): when both
            // arguments are on the table their evaluations interleave
            for (int k = gl; k < nb; k += 2 * G) {
                const bool two = k + G < nb;
                const int k2 = two ? k + G : k;
                const dd x1 = two_prod(om, P.rs[D.k0 + k]), x2 = two_prod(om, P.rs[D.k0 + k2]);
                const double c1 = cs[D.k0 + k], c2 = two ? cs[D.k0 + k2] : 0.0;
                double j1, j2;
                if (on_jtab(P, x1.hi) && on_jtab(P, x2.hi)) {
                    if constexpr (LDS)
                        besselj_table2<kJtabLdsStride>(P, s_tab, x1.hi, x1.lo, x2.hi, x2.lo, j1, j2);
                    else
                        besselj_table2<kJtabCoef / 2>(P, (const double2*)P.jtab, x1.hi, x1.lo, x2.hi, x2.lo, j1, j2);
                } else {
                    j1 = besselj_direct(P, x1.hi, x1.lo);
                    j2 = two ? besselj_direct(P, x2.hi, x2.lo) : 0.0;
                }
                acc = __builtin_fma(c1, j1, acc);
                acc = __builtin_fma(c2, j2, acc);
            }
        }
        for (int o = G >> 1; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
        if (i < mb && gl == 0) gd[D.j0 + i] = acc;
    }
}

__device__ __forceinline__ void direct_body(const PlanDev& P, int bid)
{
    __shared__ double2 s_tab[kJtabLdsPanels * kJtabLdsStride];
    const DBlock D = P.db[bid];
    if (P.jtab_np > 0 && P.jtab_np <= kJtabLdsPanels) {
        const double2* __restrict__ g = (const double2*)P.jtab;
        constexpr int per = kJtabCoef / 2;
        for (int e = threadIdx.x; e < P.jtab_np * per; e += kDirectThreads) {
            const int pn = e / per;
            s_tab[pn * kJtabLdsStride + (e - pn * per)] = g[e];
        }
        __syncthreads();
        direct_rows<true>(P, D, s_tab);
    } else {
        direct_rows<false>(P, D, nullptr);
    }
}

__global__ __launch_bounds__(kDirectThreads) void k_direct_blocks(PlanDev P) { direct_body(P, blockIdx.x); }

__global__ __launch_bounds__(kDirectThreads) void k_direct_blocks_many(const PlanDev* __restrict__ plans,
                                                                       const WorkSeg* __restrict__ segs, int nseg)
{
    const WorkSeg w = find_seg(segs, nseg);
    direct_body(plan_of(plans, w.t), w.g0);
}

__global__ void k_fill_zero(double* __restrict__ x, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

// Row pass, two kernels; each has one thread per sorted frequency and walks
// the block tree from the root.  At a node the row lies either in the local
// side (rows j0..js) -- local block, then the upper-right child -- or in the
// asymptotic side -- asymptotic block, then the lower-left child; a direct
// child ends the walk.  k_rows_asy adds the row's asymptotic blocks (no LDS,
// so it runs at the occupancy its registers allow) into ga; k_rows_local adds
// the local blocks, the direct-block sum from k_direct_blocks and ga, and
// writes g once in the caller's order.
template <int NCH>
__device__ __forceinline__ void rows_asy_body(const PlanDev& P, int bid)
{
    const double2* __restrict__ grids = P.grids;
    int j = bid * blockDim.x + threadIdx.x;
    if (j >= P.m) return;
    double om = P.ws[j];
    double acc = 0.0;
    int node = P.n_nodes > 0 ? 0 : -1;
    while (node >= 0) {
        const Node nd = P.nodes[node];
        int child;
        if (j <= nd.js) {
            child = nd.ur;
        } else {
            if (nd.ablk >= 0) {
                int ab = nd.ablk;
                int abu = __builtin_amdgcn_readfirstlane(ab);
                if (__all(ab == abu)) acc += asym_eval<NCH, true>(P, abu, om, grids);
                else acc += asym_eval<NCH, false>(P, ab, om, grids);
            }
            child = nd.ll;
        }
        node = child;
    }
    P.ga[j] = acc;
}

template <int NCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_rows_asy(PlanDev P)
{
    rows_asy_body<NCH>(P, blockIdx.x);
}

template <int NCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_rows_asy_many(
    const PlanDev* __restrict__ plans, const WorkSeg* __restrict__ segs, int nseg)
{
    const WorkSeg w = find_seg(segs, nseg);
    rows_asy_body<NCH>(plan_of(plans, w.t), w.g0);
}

template <int MODE>
__device__ __forceinline__ void rows_local_body(const PlanDev& P, int bid, double* g)
{
    const double* __restrict__ gd = P.gd;
    const double* __restrict__ ga = P.ga;
    const double* __restrict__ lmom = P.lmom;
    extern __shared__ double ring_all[];
    int j = bid * blockDim.x + threadIdx.x;
    if (j >= P.m) return;
    double* ring = ring_all + threadIdx.x;
    const int stride = blockDim.x;
    double om = P.ws[j];
    double acc = 0.0;
    int node = P.n_nodes > 0 ? 0 : -1;
    while (node >= 0) {
        const Node nd = P.nodes[node];
        int child;
        if (j <= nd.js) {
            if (nd.lblk >= 0) {
                int lb = nd.lblk;
                int lbu = __builtin_amdgcn_readfirstlane(lb);
                if constexpr (MODE == 3) {
                    if (__all(lb == lbu)) acc += local_eval_half(P, lbu, om, lmom);
                    else acc += local_eval_half(P, lb, om, lmom);
                } else {
                    if (__all(lb == lbu)) acc += local_eval<MODE>(P, lbu, om, lmom, ring, stride);
                    else acc += local_eval<MODE>(P, lb, om, lmom, ring, stride);
                }
            }
            child = nd.ur;
        } else {
            child = nd.ll;
        }
        if (child <= -2) {
            acc += gd[j];
            break;
        }
        node = child;
    }
    g[P.perm_w[j]] = P.sign * (acc + ga[j]);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_rows_local(PlanDev P, double* g, double* const* g_slot)
{
    rows_local_body<MODE>(P, blockIdx.x, g_slot ? *g_slot : g);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_rows_local_many(const PlanDev* __restrict__ plans,
                                                         const WorkSeg* __restrict__ segs, int nseg,
                                                         double* const* g_table)
{
    const WorkSeg w = find_seg(segs, nseg);
    rows_local_body<MODE>(plan_of(plans, w.t), w.g0, g_table[w.t]);
}

// Brute-force reference: one thread per frequency, all points.
__global__ void k_direct_all(PlanDev P, const double* __restrict__ r, const double* __restrict__ c, int32_t n,
                             const double* __restrict__ w, int32_t m, double* __restrict__ g)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double om = w[j];
    double acc = 0.0;
    for (int k = 0; k < n; ++k) {
        dd x = two_prod(om, r[k]);
        acc = __builtin_fma(c[k], besselj_full(P, x.hi, x.lo), acc);
    }
    g[j] = P.sign * acc;
}

// ---------------------------------------------------------------------------
static inline int cdiv64(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

template <int NCH>
static void launch_spread(const PlanDev& P, const Summary& S, hipStream_t s)
{
    const int32_t n_dense = S.n_adense, n_med = S.n_amed, n_rest = S.n_aitems - S.n_adense - S.n_amed;
    if constexpr (NCH <= kMfmaMaxChannels) {
        if (n_dense > 0)
            hipLaunchKernelGGL((k_spread_mfma<NCH, kSpreadAnchors>), dim3(n_dense), dim3(256), 0, s, P);
    }
    if constexpr (NCH <= kMfmaMedMaxChannels) {
        if (n_med > 0)
            hipLaunchKernelGGL((k_spread_mfma<NCH, kSpreadAnchorsMed>), dim3(n_med), dim3(256), 0, s, P);
    }
    if (n_rest > 0) {
        if (P.fp32)
            hipLaunchKernelGGL((k_spread<NCH, float>), dim3(n_rest), dim3(256), spread_lds_bytes<float>(P.w), s, P);
        else
            hipLaunchKernelGGL((k_spread<NCH, double>), dim3(n_rest), dim3(256), spread_lds_bytes<double>(P.w), s, P);
    }
}

template <int NCH>
static void launch_rows_asy(const PlanDev& P, hipStream_t s)
{
    hipLaunchKernelGGL(k_rows_asy<NCH>, dim3(cdiv64(P.m, 256)), dim3(256), 0, s, P);
}

// local_eval keeps J_{nu-a .. nu}, a = floor(nu/2), per thread in LDS: the
// block size and LDS bytes of the local-row kernel of order nu (MODE 2).
static int rows_local_block(int nu)
{
    const int slots = (nu >> 1) + 1;
    return slots * 256 * 8 <= 65536 ? 256 : 64;
}

static size_t rows_local_lds(int nu, int bs)
{
    return nu <= 1 ? 0 : (size_t)((nu >> 1) + 1) * bs * sizeof(double);
}

static void launch_rows_local(const PlanDev& P, const IoArgs& io, hipStream_t s)
{
    if (P.half) {      // half-integer orders: coefficients from the table
        hipLaunchKernelGGL(k_rows_local<3>, dim3(cdiv64(P.m, 256)), dim3(256), 0, s, P, io.g, io.g_slot);
        return;
    }
    if (P.nu <= 1) {   // no ring of earlier values needed
        auto k = P.nu == 0 ? k_rows_local<0> : k_rows_local<1>;
        hipLaunchKernelGGL(k, dim3(cdiv64(P.m, 256)), dim3(256), 0, s, P, io.g, io.g_slot);
        return;
    }
    const int bs = rows_local_block(P.nu);
    hipLaunchKernelGGL(k_rows_local<2>, dim3(cdiv64(P.m, bs)), dim3(bs), rows_local_lds(P.nu, bs), s, P, io.g,
                       io.g_slot);
}

// Calls f with std::integral_constant<int, nch>; nch is one of the instantiated
// channel counts (every even count up to 16, multiples of 4 up to 40).
template <class F>
static void dispatch_channels(int nch, F&& f)
{
    switch (nch) {
    case 2: f(std::integral_constant<int, 2>()); break;
    case 4: f(std::integral_constant<int, 4>()); break;
    case 6: f(std::integral_constant<int, 6>()); break;
    case 8: f(std::integral_constant<int, 8>()); break;
    case 10: f(std::integral_constant<int, 10>()); break;
    case 12: f(std::integral_constant<int, 12>()); break;
    case 14: f(std::integral_constant<int, 14>()); break;
    case 16: f(std::integral_constant<int, 16>()); break;
    case 20: f(std::integral_constant<int, 20>()); break;
    case 24: f(std::integral_constant<int, 24>()); break;
    case 28: f(std::integral_constant<int, 28>()); break;
    case 32: f(std::integral_constant<int, 32>()); break;
    case 36: f(std::integral_constant<int, 36>()); break;
    default: f(std::integral_constant<int, 40>()); break;
    }
}

static inline void mark(hipEvent_t* marks, int i, hipStream_t s)
{
    if (marks && marks[i]) (void)hipEventRecord(marks[i], s);
}

hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_value, dim3(cdiv64(n, 256)), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}

hipError_t launch_set_pointers(void** table, const void* const* ptrs, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (count > 224) return hipErrorInvalidValue;
    PtrArgs a;
    for (int i = 0; i < count; ++i) a.p[i] = const_cast<void*>(ptrs[i]);
    hipLaunchKernelGGL(k_set_pointers, dim3(1), dim3(256), 0, s, table, a, count);
    return hipGetLastError();
}

// Lines per tile for transforms of length 2^logL.
static int fft_log_lines(int logL)
{
    int l = 0;
    while ((1 << (l + 1)) <= kFftMaxLines && (1 << (l + 1 + logL)) <= kFftTilePts) ++l;
    return l;
}

static size_t fft_lds_bytes(int logL, int logLines)
{
    return sizeof(double2) * ((size_t)((1 << logL) + 1) * (1 << logLines) + (1 << logL));
}

// Two passes for N <= 2^16 (N1 = 2^floor(logN/2)), three beyond; every pass
// length is at most 2^8 and at least 2^6 for the sizes that reach here.
// pass 0: the inner column pass over nb (three-pass sizes only), 1: the
// column pass over na, 2: the row pass.  Returns false when the size class
// has no such pass; else its arguments, workgroups and LDS bytes.
static bool fft_pass(const FftClass& K, int nch, int pass, FftPass& F, int& blocks, size_t& lds)
{
    const int logN = K.log2n;
    const int ntr = K.count * nch;
    int logN1, logNa, logNb;
    if (logN <= 16) {
        logN1 = logN / 2; logNa = logN - logN1; logNb = 0;
    } else {
        logN1 = logN / 3; logNa = (logN - logN1) / 2; logNb = logN - logN1 - logNa;
    }
    const int64_t N1 = int64_t(1) << logN1, Na = int64_t(1) << logNa, Nb = int64_t(1) << logNb;
    F = FftPass{};
    F.first = K.first;
    F.logN = logN;
    F.scratch_off = K.scratch_off;
    FftCol& c = F.C;
    if (pass == 0) {
        if (logNb == 0) return false;
        c.logL = logNb; c.logLines = fft_log_lines(logNb); c.logBlo = logN1 + logNa; c.to_scratch = 0;
        c.in_es = N1 * Na; c.in_hs = 0; c.out_es = N1 * Na; c.out_hs = 0;
        c.lo_mask = ~(N1 - 1); c.kmul = 1;
    } else if (pass == 1) {
        c.logL = logNa; c.logLines = fft_log_lines(logNa); c.logBlo = logN1; c.to_scratch = 1;
        c.in_es = N1; c.in_hs = N1 * Na; c.out_es = N1 * Nb; c.out_hs = N1;
        c.lo_mask = ~int64_t(0); c.kmul = Nb;
    } else {
        c.logL = logN1; c.logLines = fft_log_lines(logN1);
        blocks = ntr * (int)((int64_t(1) << (logN - logN1)) >> c.logLines);
        lds = fft_lds_bytes(c.logL, c.logLines);
        return true;
    }
    blocks = ntr * (int)((int64_t(1) << logN) >> (c.logL + c.logLines));
    lds = fft_lds_bytes(c.logL, c.logLines);
    return true;
}

static void launch_fft_large(const PlanDev& P, const FftClass& K, hipStream_t s)
{
    for (int pass = 0; pass < 3; ++pass) {
        FftPass F;
        int blocks = 0;
        size_t lds = 0;
        if (!fft_pass(K, P.nch, pass, F, blocks, lds)) continue;
        if (pass < 2) hipLaunchKernelGGL(k_fft_col, dim3(blocks), dim3(256), lds, s, P, F);
        else hipLaunchKernelGGL(k_fft_row, dim3(blocks), dim3(256), lds, s, P, F);
    }
}

hipError_t launch_execute(const PlanDev& P, const Summary& S, const ExecBuffers& B, const FftClass* cls, int ncls,
                          const IoArgs& io, hipStream_t s, hipEvent_t* marks, const ExecFork* fork)
{
    if (P.m == 0) return hipSuccess;
    if (P.n == 0) {   // a fill kernel, not a memset node, so the call can be captured in a graph
        hipLaunchKernelGGL(k_zero_output, dim3(cdiv64(P.m, 256)), dim3(256), 0, s, io.g, io.g_slot, (int64_t)P.m);
        return hipGetLastError();
    }
    mark(marks, 0, s);
    hipLaunchKernelGGL(k_gather, dim3(cdiv64(P.n, 256)), dim3(256), 0, s, P, io.c, io.c_slot,
                       io.scale_by_points ? 1 : 0);
    mark(marks, 1, s);
    // the local moments and direct blocks read only the gathered weights
    const bool forked = fork && fork->side && (S.n_litems > 0 || P.n_d > 0);
    const hipStream_t ls = forked ? fork->side : s;
    if (forked) {
        hipError_t e = hipEventRecord(fork->ev_fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(ls, fork->ev_fork, 0);
        if (e != hipSuccess) return e;
    }
    if (S.n_litems > 0) {
        if (lmom_width(P.L) == 32) hipLaunchKernelGGL(k_lmom<32>, dim3(S.n_litems), dim3(64), 0, ls, P);
        else hipLaunchKernelGGL(k_lmom<64>, dim3(S.n_litems), dim3(64), 0, ls, P);
        hipLaunchKernelGGL(k_lmom_reduce, dim3(cdiv64((int64_t)S.n_l * (P.L + 1), 256)), dim3(256), 0, ls, P);
    }
    auto launch_direct = [&](hipStream_t st) {
        if (P.n_d > 0) {
            hipLaunchKernelGGL(k_fill_zero, dim3(cdiv64(P.m, 256)), dim3(256), 0, st, P.gd, (int64_t)P.m);
            hipLaunchKernelGGL(k_direct_blocks, dim3(P.n_d), dim3(kDirectThreads), 0, st, P);
        }
    };
    if (forked) {
        launch_direct(ls);
        const hipError_t e = hipEventRecord(fork->ev_join, ls);
        if (e != hipSuccess) return e;
    }
    mark(marks, 2, s);
    dispatch_channels(P.nch, [&](auto k) { launch_spread<decltype(k)::value>(P, S, s); });
    mark(marks, 3, s);
    if (P.grid_cells > 0) {
        if (P.fp32)
            hipLaunchKernelGGL(k_spread_reduce<float2>, dim3(cdiv64(P.grid_cells * P.nch, 256)), dim3(256), 0, s, P);
        else
            hipLaunchKernelGGL(k_spread_reduce<double2>, dim3(cdiv64(P.grid_cells * P.nch, 256)), dim3(256), 0, s, P);
    }
    mark(marks, 4, s);
    if (P.small.n > 0 && P.small.wg0[P.small.n] > 0)
        hipLaunchKernelGGL(k_fft_small, dim3(P.small.wg0[P.small.n]), dim3(256),
                           sizeof(double2) << P.small.max_log2n, s, P);
    for (int q = 0; q < ncls; ++q)
        if (cls[q].log2n > 12) launch_fft_large(P, cls[q], s);
    mark(marks, 5, s);
    if (!forked) launch_direct(s);
    mark(marks, 6, s);
    dispatch_channels(P.nch, [&](auto k) { launch_rows_asy<decltype(k)::value>(P, s); });
    mark(marks, 7, s);
    if (forked) {
        const hipError_t e = hipStreamWaitEvent(s, fork->ev_join, 0);
        if (e != hipSuccess) return e;
    }
    launch_rows_local(P, io, s);
    mark(marks, 8, s);
    return hipGetLastError();
}

void small_fft_table(PlanDev& P, const FftClass* cls, int ncls)
{
    SmallFfts& F = P.small;
    F = SmallFfts{};
    int wg = 0;
    for (int q = 0; q < ncls; ++q) {
        const FftClass& C = cls[q];
        if (C.log2n > 12 || F.n == 8) continue;
        F.log2n[F.n] = C.log2n;
        F.first[F.n] = C.first;
        F.wg0[F.n] = wg;
        wg += C.count * P.nch;
        F.max_log2n = C.log2n > F.max_log2n ? C.log2n : F.max_log2n;
        ++F.n;
    }
    F.wg0[F.n] = wg;
}

// ---------------------------------------------------------------------------
// Batches: the launch list.  Kinds in execution order; a launch's variant is
// its channel count (spreading, grid rows) or local-row mode.
// ---------------------------------------------------------------------------
enum BatchKind : int32_t {
    kZeroOut, kGather, kLmom, kLmomReduce, kSpreadMfma, kSpreadMfmaMed, kSpreadVec, kSpreadReduce, kFftSmall,
    kFftPass0, kFftPass1, kFftPass2, kZeroGd, kDirect, kRowsAsy, kRowsLocal
};

void build_batch_schedule(const BatchTransform* tr, int count, const int* order, BatchSchedule& out)
{
    out = BatchSchedule{};
    std::vector<WorkSeg> segs;
    std::vector<FftSeg> fsegs;
    // one launch of `kind` over the transforms accepted by `take`, which gives
    // a transform's workgroups (0: none) and may raise the launch's LDS bytes
    auto add = [&](int32_t kind, int32_t variant, int32_t fp32, int32_t threads, auto&& take) {
        BatchLaunch L{};
        L.kind = kind; L.variant = variant; L.fp32 = fp32; L.threads = threads;
        L.seg0 = (int32_t)segs.size();
        int64_t g = 0;
        for (int q = 0; q < count; ++q) {
            const int t = order[q];
            size_t lds = 0;
            const int64_t wg = take(tr[t], lds);
            if (wg <= 0) continue;
            segs.push_back(WorkSeg{t, (int32_t)g});
            g += wg;
            if (lds > L.lds) L.lds = lds;
        }
        L.nseg = (int32_t)segs.size() - L.seg0;
        L.blocks = (int32_t)g;
        if (L.nseg > 0) out.launches.push_back(L);
    };
    auto live = [](const PlanDev& P) { return P.n > 0 && P.m > 0; };
    add(kZeroOut, 0, 0, 256, [&](const BatchTransform& T, size_t&) -> int64_t {
        return (T.P->n == 0 && T.P->m > 0) ? cdiv64(T.P->m, 256) : 0;
    });
    add(kGather, 0, 0, 256, [&](const BatchTransform& T, size_t&) -> int64_t {
        return live(*T.P) ? cdiv64(T.P->n, 256) : 0;
    });
    for (const int width : {32, 64})
        add(kLmom, width, 0, 64, [&](const BatchTransform& T, size_t&) -> int64_t {
            return live(*T.P) && lmom_width(T.P->L) == width ? T.S->n_litems : 0;
        });
    add(kLmomReduce, 0, 0, 256, [&](const BatchTransform& T, size_t&) -> int64_t {
        return live(*T.P) && T.S->n_litems > 0 ? cdiv64((int64_t)T.S->n_l * (T.P->L + 1), 256) : 0;
    });
    // the channel counts and precisions present
    std::vector<std::pair<int, int>> variants;
    for (int t = 0; t < count; ++t) {
        const std::pair<int, int> v{tr[t].P->nch, tr[t].P->fp32};
        if (live(*tr[t].P) && std::find(variants.begin(), variants.end(), v) == variants.end()) variants.push_back(v);
    }
    std::sort(variants.begin(), variants.end());
    for (const auto& v : variants) {
        const int nch = v.first, fp32 = v.second;
        auto same = [&](const PlanDev& P) { return live(P) && P.nch == nch && P.fp32 == fp32; };
        if (nch <= kMfmaMaxChannels)   // static LDS: no launch bytes
            add(kSpreadMfma, nch, fp32, 256, [&](const BatchTransform& T, size_t&) -> int64_t {
                return same(*T.P) ? T.S->n_adense : 0;
            });
        if (nch <= kMfmaMedMaxChannels)
            add(kSpreadMfmaMed, nch, fp32, 256, [&](const BatchTransform& T, size_t&) -> int64_t {
                return same(*T.P) ? T.S->n_amed : 0;
            });
        add(kSpreadVec, nch, fp32, 256, [&](const BatchTransform& T, size_t& lds) -> int64_t {
            if (!same(*T.P)) return 0;
            lds = fp32 ? spread_lds_bytes<float>(T.P->w) : spread_lds_bytes<double>(T.P->w);
            return T.S->n_aitems - T.S->n_adense - T.S->n_amed;
        });
    }
    for (int fp32 = 0; fp32 <= 1; ++fp32)
        add(kSpreadReduce, 0, fp32, 256, [&](const BatchTransform& T, size_t&) -> int64_t {
            return live(*T.P) && T.P->fp32 == fp32 ? cdiv64(T.P->grid_cells * T.P->nch, 256) : 0;
        });
    add(kFftSmall, 0, 0, 256, [&](const BatchTransform& T, size_t& lds) -> int64_t {
        const SmallFfts& F = T.P->small;
        if (!live(*T.P) || F.n == 0) return 0;
        lds = sizeof(double2) << F.max_log2n;
        return F.wg0[F.n];
    });
    for (int pass = 0; pass < 3; ++pass) {
        BatchLaunch L{};
        L.kind = kFftPass0 + pass;
        L.threads = 256;
        L.seg0 = (int32_t)fsegs.size();
        int64_t g = 0;
        for (int q = 0; q < count; ++q) {
            const int t = order[q];
            if (!live(*tr[t].P)) continue;
            for (int c = 0; c < tr[t].ncls; ++c) {
                const FftClass& K = tr[t].cls[c];
                if (K.log2n <= 12) continue;
                FftSeg f{};
                int blocks = 0;
                size_t lds = 0;
                if (!fft_pass(K, tr[t].P->nch, pass, f.F, blocks, lds) || blocks <= 0) continue;
                f.t = t;
                f.g0 = (int32_t)g;
                fsegs.push_back(f);
                g += blocks;
                if (lds > L.lds) L.lds = lds;
            }
        }
        L.nseg = (int32_t)fsegs.size() - L.seg0;
        L.blocks = (int32_t)g;
        if (L.nseg > 0) out.launches.push_back(L);
    }
    add(kZeroGd, 0, 0, 256, [&](const BatchTransform& T, size_t&) -> int64_t {
        return live(*T.P) && T.P->n_d > 0 ? cdiv64(T.P->m, 256) : 0;
    });
    add(kDirect, 0, 0, kDirectThreads, [&](const BatchTransform& T, size_t&) -> int64_t {
        return live(*T.P) ? T.P->n_d : 0;
    });
    std::vector<int> chans;
    for (const auto& v : variants)
        if (std::find(chans.begin(), chans.end(), v.first) == chans.end()) chans.push_back(v.first);
    for (int nch : chans)
        add(kRowsAsy, nch, 0, 256, [&](const BatchTransform& T, size_t&) -> int64_t {
            return live(*T.P) && T.P->nch == nch ? cdiv64(T.P->m, 256) : 0;
        });
    // local rows: orders 0 and 1, the general mode at 256 and at 64 lanes,
    // half-integer orders
    for (int mode = 0; mode < 5; ++mode) {
        const int bs = mode == 3 ? 64 : 256;
        const int variant = mode < 2 ? mode : (mode == 4 ? 3 : 2);
        add(kRowsLocal, variant, 0, bs, [&](const BatchTransform& T, size_t& lds) -> int64_t {
            const int nu = T.P->nu;
            if (!live(*T.P) || (T.P->half != 0) != (mode == 4)) return 0;
            if (mode < 2 ? nu != mode : (mode < 4 && (nu <= 1 || rows_local_block(nu) != bs))) return 0;
            lds = mode == 4 ? 0 : rows_local_lds(nu, bs);
            return cdiv64(T.P->m, bs);
        });
    }
    // the device tables: PlanDev[count], WorkSeg[], FftSeg[] (each 256-byte aligned)
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    out.segs_off = align(sizeof(PlanDev) * (size_t)count);
    out.fsegs_off = out.segs_off + align(sizeof(WorkSeg) * segs.size());
    out.table.assign(out.fsegs_off + sizeof(FftSeg) * fsegs.size(), 0);
    for (int t = 0; t < count; ++t) std::memcpy(out.table.data() + sizeof(PlanDev) * t, tr[t].P, sizeof(PlanDev));
    if (!segs.empty()) std::memcpy(out.table.data() + out.segs_off, segs.data(), sizeof(WorkSeg) * segs.size());
    if (!fsegs.empty()) std::memcpy(out.table.data() + out.fsegs_off, fsegs.data(), sizeof(FftSeg) * fsegs.size());
}

hipError_t launch_execute_many(const BatchSchedule& S, const void* table_dev, void* const* c_table,
                               void* const* g_table, hipStream_t s, const ExecFork* fork)
{
    const char* base = (const char*)table_dev;
    const PlanDev* plans = (const PlanDev*)base;
    const WorkSeg* segs = (const WorkSeg*)(base + S.segs_off);
    const FftSeg* fsegs = (const FftSeg*)(base + S.fsegs_off);
    const double* const* cin = (const double* const*)c_table;
    double* const* gout = (double* const*)g_table;
    // with `fork`: the local moments and direct blocks on its side stream,
    // forked at the first of them (after the gather) and joined before the
    // local rows (or at the end)
    bool forked = false, joined = false;
    auto join = [&]() -> hipError_t {
        hipError_t e = hipEventRecord(fork->ev_join, fork->side);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, fork->ev_join, 0);
        joined = true;
        return e;
    };
    for (const BatchLaunch& L : S.launches) {
        const dim3 grid(L.blocks), block(L.threads);
        const bool side_kind = L.kind == kLmom || L.kind == kLmomReduce || L.kind == kZeroGd || L.kind == kDirect;
        hipStream_t st = s;
        if (fork && side_kind && !joined) {
            if (!forked) {
                hipError_t e = hipEventRecord(fork->ev_fork, s);
                if (e == hipSuccess) e = hipStreamWaitEvent(fork->side, fork->ev_fork, 0);
                if (e != hipSuccess) return e;
                forked = true;
            }
            st = fork->side;
        }
        if (forked && !joined && L.kind == kRowsLocal) {
            const hipError_t e = join();
            if (e != hipSuccess) return e;
        }
        const WorkSeg* sg = segs + L.seg0;
        const FftSeg* fs = fsegs + L.seg0;
        switch (L.kind) {
        case kZeroOut: hipLaunchKernelGGL(k_zero_output_many, grid, block, 0, s, plans, sg, L.nseg, gout); break;
        case kGather: hipLaunchKernelGGL(k_gather_many, grid, block, 0, s, plans, sg, L.nseg, cin); break;
        case kLmom:
            if (L.variant == 32) hipLaunchKernelGGL(k_lmom_many<32>, grid, block, 0, st, plans, sg, L.nseg);
            else hipLaunchKernelGGL(k_lmom_many<64>, grid, block, 0, st, plans, sg, L.nseg);
            break;
        case kLmomReduce: hipLaunchKernelGGL(k_lmom_reduce_many, grid, block, 0, st, plans, sg, L.nseg); break;
        case kSpreadMfma:
        case kSpreadMfmaMed:
            dispatch_channels(L.variant, [&](auto k) {
                constexpr int NCH = decltype(k)::value;
                if constexpr (NCH <= kMfmaMaxChannels) {
                    if (L.kind == kSpreadMfma)
                        hipLaunchKernelGGL((k_spread_mfma_many<NCH, kSpreadAnchors>), grid, block, 0, s, plans, sg,
                                           L.nseg);
                }
                if constexpr (NCH <= kMfmaMedMaxChannels) {
                    if (L.kind == kSpreadMfmaMed)
                        hipLaunchKernelGGL((k_spread_mfma_many<NCH, kSpreadAnchorsMed>), grid, block, 0, s, plans,
                                           sg, L.nseg);
                }
            });
            break;
        case kSpreadVec:
            dispatch_channels(L.variant, [&](auto k) {
                constexpr int NCH = decltype(k)::value;
                if (L.fp32) hipLaunchKernelGGL((k_spread_many<NCH, float>), grid, block, L.lds, s, plans, sg, L.nseg);
                else hipLaunchKernelGGL((k_spread_many<NCH, double>), grid, block, L.lds, s, plans, sg, L.nseg);
            });
            break;
        case kSpreadReduce:
            if (L.fp32) hipLaunchKernelGGL(k_spread_reduce_many<float2>, grid, block, 0, s, plans, sg, L.nseg);
            else hipLaunchKernelGGL(k_spread_reduce_many<double2>, grid, block, 0, s, plans, sg, L.nseg);
            break;
        case kFftSmall: hipLaunchKernelGGL(k_fft_small_many, grid, block, L.lds, s, plans, sg, L.nseg); break;
        case kFftPass0:
        case kFftPass1: hipLaunchKernelGGL(k_fft_col_many, grid, block, L.lds, s, plans, fs, L.nseg); break;
        case kFftPass2: hipLaunchKernelGGL(k_fft_row_many, grid, block, L.lds, s, plans, fs, L.nseg); break;
        case kZeroGd: hipLaunchKernelGGL(k_zero_gd_many, grid, block, 0, st, plans, sg, L.nseg); break;
        case kDirect: hipLaunchKernelGGL(k_direct_blocks_many, grid, block, 0, st, plans, sg, L.nseg); break;
        case kRowsAsy:
            dispatch_channels(L.variant, [&](auto k) {
                hipLaunchKernelGGL((k_rows_asy_many<decltype(k)::value>), grid, block, 0, s, plans, sg, L.nseg);
            });
            break;
        case kRowsLocal:
            if (L.variant == 0) hipLaunchKernelGGL(k_rows_local_many<0>, grid, block, L.lds, s, plans, sg, L.nseg, gout);
            else if (L.variant == 1)
                hipLaunchKernelGGL(k_rows_local_many<1>, grid, block, L.lds, s, plans, sg, L.nseg, gout);
            else if (L.variant == 3)
                hipLaunchKernelGGL(k_rows_local_many<3>, grid, block, L.lds, s, plans, sg, L.nseg, gout);
            else hipLaunchKernelGGL(k_rows_local_many<2>, grid, block, L.lds, s, plans, sg, L.nseg, gout);
            break;
        default: return hipErrorInvalidValue;
        }
    }
    if (forked && !joined) {
        const hipError_t e = join();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_half_difference(const double* w, const double* a, const double* b, double* out, int32_t n,
                                  hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_half_difference, dim3(cdiv64(n, 256)), dim3(256), 0, s, w, a, b, out, n);
    return hipGetLastError();
}

hipError_t launch_direct(const PlanDev& P, const double* r, const double* c, int32_t n, const double* w, int32_t m,
                         double* g, hipStream_t s)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_direct_all, dim3(cdiv64(m, 128)), dim3(128), 0, s, P, r, c, n, w, m, g);
    return hipGetLastError();
}

}  // namespace nuht
