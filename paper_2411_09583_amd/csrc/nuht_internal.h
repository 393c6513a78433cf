// nuht_internal.h -- data structures shared by the host code and the HIP kernels.
//
// Index conventions follow the paper (Sec. 4.1): rows j index the frequencies
// omega (sorted ascending), columns k index the points r (sorted ascending).
// A block is the inclusive index rectangle rows j0..j1, columns k0..k1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nuht {

constexpr int kMaxChannels = 40;       // 2M with M <= 20 (eq. num-asy-terms caps M at 20)
constexpr int kMaxFftLog2 = 24;        // largest FFT of an asymptotic block: 2^24 = 4096^2 points (two passes)
constexpr int kLocalChunk = 4096;      // columns per local-moment work item
constexpr int kSpreadChunk = 1024;     // default points per spreading work item (a plan option)
// Default direct-block threshold of Alg. 1 for an n x m transform.  The
// paper leaves min_size to numerical experiments (its example: 1024).  On
// MI355X, with the direct entries read from a J_nu table, the fastest
// threshold grows with the matrix: 1024 for n m below about 5e5, 2048 near
// 1e6, 8192 from about 1e7 on (uniform, radial, exponential, Fourier-Bessel
// and batched workloads).  The rule takes the power of two at or below
// n m / 256, within [1024, 8192].
constexpr int64_t kMinSizeLo = 1024;
constexpr int64_t kMinSizeHi = 8192;
inline int64_t default_min_size(int64_t n, int64_t m) {
    const double a = (double)n * (double)m / 256.0;
    int64_t s = kMinSizeLo;
    while (s < kMinSizeHi && (double)(2 * s) <= a) s *= 2;
    return s;
}
constexpr int kMaxEsWidth = 18;        // largest ES kernel width
constexpr int kEshatTerms = 16;        // terms of the polynomial for the ES kernel's Fourier transform
constexpr int kEsDeg = 13;             // degree of the per-cell polynomial pieces of the ES kernel
constexpr int kSpreadAnchors = 6;      // first cells (anchors) of a dense matrix-core spreading item
constexpr int kSpreadAnchorsMed = 40;  // first cells of a medium one (its own launch, larger LDS cell sums)
constexpr int kMfmaMaxChannels = 32;   // channel counts whose dense items go to the matrix cores
constexpr int kMfmaMedMaxChannels = 16; // ... and whose medium items (their LDS cell sums grow with the channels)
constexpr int kMaxLevels = 4096;       // subdivision depth limit
constexpr int kHalfDeg = 20;           // degree of the half-integer local coefficients on a panel
constexpr double kHalfWidth = 4.0;     // panel width (in omega R) of those coefficients
constexpr int kJtabCoef = 16;          // coefficients per panel of the direct-block J_nu table (degree 15)
constexpr double kJtabWidth = 2.0;     // panel width (in x = omega r) of that table

// A mixed block of Alg. 1 and the split chosen for it.  Rows j0..js and
// columns k0..ks are the local (upper-left) side.  A wholly local block is
// stored with (js, ks) = (j1, k1), a wholly asymptotic one with
// (js, ks) = (j0-1, k0-1).
struct Node {
    int32_t j0, j1, k0, k1;
    int32_t js, ks;
    int32_t lblk, ablk;   // local / asymptotic child block index, -1 if empty
    int32_t ur, ll;       // upper-right / lower-left child: >= 0 mixed node,
                          // <= -2 direct block (-2 - index), -1 empty
    int32_t level, pad;
};

__host__ __device__ inline int32_t encode_direct(int32_t d) { return -2 - d; }
__host__ __device__ inline int32_t decode_direct(int32_t c) { return -2 - c; }

struct LBlock {
    int32_t j0, j1, k0, k1;
    double R;             // expansion radius: r_{k1}, or z / omega_{j1} when r_{k1} = 0
    int32_t item0, nitems;
    int32_t level, pad;
};

struct ABlock {
    int32_t j0, j1, k0, k1;
    double C, D;          // centres of the point and frequency ranges
    double h;             // spread-grid spacing (a power of two)
    double r0;            // smallest point of the block (weights are normalised by it)
    double alpha;         // ES kernel half-width w h / 2
    double Khi, Klo;      // h N2 / (2 pi) as a double-double (FFT path)
    int32_t llo, N1;      // spread-grid cells llo .. llo + N1 - 1
    int32_t N2, fft;      // FFT size and 1 for the FFT path; 0 for the direct-sum path
    int64_t grid_off;     // offset of the block's grid (complex elements)
    int32_t item0, nitems;
    int64_t part_off;     // first partial-subgrid element of its items (complex)
    int32_t level, fft_slot;  // fft_slot: position in the FFT size-class list
};

struct DBlock {
    int32_t j0, j1, k0, k1;
};

// Work item of the column-side kernels: a chunk of one block's columns.
struct Item {
    int32_t blk;
    int32_t ka, kb;       // columns ka .. kb-1
    int32_t sub_lo, sub_n;  // spread items: subgrid cells sub_lo .. sub_lo + sub_n - 1
    int32_t dense;        // spread items on the matrix cores: 1 (dense) if its points' first cells
                          // lie in sub_lo .. sub_lo + kSpreadAnchors - 1, 2 (medium) if within
                          // kSpreadAnchorsMed of sub_lo; else 0 (vector spreading)
    int64_t off;          // spread items: partial-subgrid offset (complex elements)
};

// Written by the planning kernels, read once by the host.
struct Summary {
    int32_t n_nodes, n_l, n_a, n_d;
    int32_t levels, overflow;
    int32_t n_litems, n_aitems;
    int32_t n_fft, max_nch;
    int32_t n_adense, n_amed;  // dense and medium spread items (the first n_adense, then n_amed, of the item list)
    int64_t l_row, l_col, a_row, a_col, d_ent;
    int64_t grid_cells;     // sum N1 (all asymptotic blocks)
    int64_t dft_cells;      // sum N1 over direct-sum-path blocks
    int64_t fft_points;     // sum N2 over FFT-path blocks
    int64_t part_cells;     // sum of item subgrid sizes
    int64_t dft_row_cells;  // sum of rows x N1 over direct-sum-path blocks
    int64_t fft_rows;       // sum of rows over FFT-path blocks
    int32_t fft_count[kMaxFftLog2 + 1];   // FFT-path blocks per log2(N2)
    int32_t fft_first[kMaxFftLog2 + 1];   // start of each size class in the FFT list
    int32_t domain_error;
    int32_t grid_error;     // an asymptotic block needs an FFT larger than 2^kMaxFftLog2
};

// FFT-path grids of at most 4096 points, every size class in one launch:
// workgroup g belongs to class c when wg0[c] <= g < wg0[c + 1], and within it
// to the FFT-list slot (g - wg0[c]) / nch of the class and channel
// (g - wg0[c]) % nch.
struct SmallFfts {
    int32_t n;                 // classes
    int32_t log2n[8], first[8];
    int32_t wg0[9];            // wg0[n]: workgroups of the launch
    int32_t max_log2n;         // largest class (its transform sets the launch's LDS)
};

// Everything the execution kernels need for one transform (passed by value to
// the kernels of a single transform; kept in a device array for a batch).
struct PlanDev {
    int32_t n, m, nu, M, L, w;       // sizes, |order| (its integer part when half), terms, local rank, ES width
    int32_t half, half_np;           // half = 1: the order is nu + 1/2; panels of the local coefficient table
    int32_t half_ns, pad0;           // leading panels holding the coefficients divided by x^nu
    int32_t nch, sign;               // channels (2M padded to a kernel instance); (-1)^nu for negative orders, else 1
    int32_t fp32;                    // FP32 spreading (weights, kernel values and channel sums in float)
    int32_t mfma;                    // dense spreading items go to the matrix cores (FP64, w <= 16, nch <= 32)
    double z, beta, eps;
    double phi_hi, phi_lo;           // -(2nu+1) pi/4 reduced to [0, 2pi), double-double
    double hank[2 * 20 + 2];         // a_p(nu), p = 0 .. 2M+1 (Hankel coefficients)
    double chan[kMaxChannels];       // channel factors (-1)^(p/2) a_p(nu) for p < 2M (odd p carry a factor i), 0 above
    double eshat[kEshatTerms];       // ES^ on [0, kappa_max]: monomial coefficients in s = 2 (kappa / kappa_max)^2 - 1
    int32_t spread_chunk, pad3;      // points per spreading work item
    double kappa_max, eshat_s;       // eshat_s = 2 / kappa_max^2
    const double* rs;                // sorted points (n)
    const double* ws;                // sorted frequencies (m)
    const int32_t* perm_r;           // sorted position -> caller index (points)
    const int32_t* perm_w;           // sorted position -> caller index (frequencies)
    const Node* nodes;
    const LBlock* lb;
    const ABlock* ab;
    const DBlock* db;
    const Item* litems;
    const Item* aitems;
    const int32_t* alist;            // spreading order: dense items from the front, the others from the back
    const int32_t* fft_list;         // FFT-path blocks grouped by size class
    const int64_t* gslot;            // first grid slot of each asymptotic block; gslot[n_a] = all slots
    const double* es_poly;           // ES kernel pieces, w x (kEsDeg + 1) monomial coefficients
    const double* half_tab;          // half-integer orders: [panel][l][degree] local coefficients
    double half_inv_h;               // 1 / panel width
    const double* jtab;              // J_nu on [jtab_x0, jtab_x0 + jtab_np kJtabWidth): per panel the
                                     // monomial coefficients in u in [-1, 1] of its Chebyshev interpolant
    double jtab_x0;
    int32_t jtab_np, pad2;
    int32_t n_nodes, n_l, n_a, n_d, n_litems, n_aitems, n_adense, n_amed;
    // execution buffers of the partition
    double* cs;                      // weights gathered into sorted point order (n)
    double* lpart;                   // local-moment partial sums (items x (L + 1))
    double* lmom;                    // local moments (local blocks x (L + 1))
    double2* part;                   // spread partial subgrids
    double2* grids;                  // spread grids (direct-sum path) and FFT buffers (FFT path)
    double2* scratch;                // second buffer of the multi-pass FFTs
    double* gd;                      // per-row direct-block sums (m)
    double* ga;                      // per-row asymptotic sums (m)
    const double2* fft_tw;           // FFT twiddles (8192 entries)
    int64_t grid_cells;              // grid slots (without the channel factor)
    SmallFfts small;                 // the FFT size classes up to 4096 points
};

// One transform's share of a batched launch: workgroups g0 .. (next g0) - 1
// of the launch work on transform t, as its workgroups 0, 1, ...
struct WorkSeg {
    int32_t t, g0;
};

}  // namespace nuht
