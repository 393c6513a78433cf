/*
 * nuht.h -- C ABI of libnuht, a nonuniform fast Hankel transform for AMD MI355X.
 *
 * The transform (Beckman & O'Neil, "A Nonuniform Fast Hankel Transform",
 * Sec. 1, eq. DHT; matrix form in Sec. 2):
 *
 *     g_j = sum_{k=0}^{n-1} c_k J_nu(omega_j r_k),    j = 0 .. m-1,
 *
 * from n points r_k >= 0 with weights c_k to m frequencies omega_j >= 0, for
 * integer order nu, to a requested tolerance eps.  The method is Alg. 2 of the
 * paper: the expansion orders (M, z, L) come from eps (Sec. 3.3); the matrix
 * J_nu(omega_j r_k) is split along omega r = z by Alg. 1 (Sec. 4.1); local
 * blocks are applied with the Wimp expansion (Sec. 3.1), asymptotic blocks with
 * 2M type-3 NUFFTs of Hankel's expansion (Sec. 3.2), and a few small direct
 * blocks entry by entry.
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers (HIP global memory) of FP64
 *    values; the caller owns them.  Pointers without _dev are host pointers.
 *  - Arrays are dense and contiguous; element i of r pairs with element i of c.
 *    Inputs may be in any order; outputs follow the order of the caller's
 *    frequencies (forward) or points (adjoint).
 *  - `stream` is a hipStream_t passed as void* (0 = the null stream).  Work is
 *    enqueued on it.  Only nuht_plan and nuht_plan_info synchronise it.
 *  - Return value: 0 on success, a negative NUHT_E* code on failure.  On
 *    failure the output arguments are left unspecified and no plan is leaked.
 */
#ifndef NUHT_H
#define NUHT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define NUHT_OK           0
#define NUHT_EINVAL      -1   /* bad size, null pointer with nonzero size, nu or eps out of range */
#define NUHT_EDOMAIN     -2   /* some r or omega is negative, NaN or infinite */
#define NUHT_EPRECISION  -3   /* FP32 spreading requested with eps < 1e-7 */
#define NUHT_ENOMEM      -4   /* device allocation failed */
#define NUHT_EHIP        -5   /* a HIP runtime call failed */
#define NUHT_ECAPACITY   -6   /* the partition exceeds an internal table limit */
#define NUHT_ENOTREADY   -7   /* nuht_gradient_noalloc: a partition it needs is not built yet */

/* Precision of the NUFFT spreading and interpolation. */
#define NUHT_FP64        0
#define NUHT_FP32_SPREAD 1    /* FP32 spreading; eps >= 1e-7 (see nuht_opts) */

typedef struct nuht_plan_s *nuht_plan_t;

/*
 * Options; pass NULL for the defaults.
 *   min_size          direct-block threshold of Alg. 1: an off-diagonal child
 *                     of area <= min_size is applied directly (0 -> the
 *                     power of two at or below n m / 256, within [1024,
 *                     8192]; the paper, Alg. 2, leaves it to numerical
 *                     experiments with 1024 as its example, and this rule
 *                     follows what measured fastest here).
 *   M_override        number of asymptotic terms M (0 -> eq. num-asy-terms).
 *   split_candidates  equispaced candidate rows in SplitIndices (0 -> 16);
 *                     -1: every row of a block (the exact optimum of the
 *                     split objective, Sec. 4.1; O(rows) per split on one lane).
 *   precision         NUHT_FP64, or NUHT_FP32_SPREAD: the ES spreading of
 *                     the asymptotic blocks (step one of the type-3 NUFFTs,
 *                     Sec. 3.2) keeps its weights, kernel values and channel
 *                     sums in FP32 and uses a kernel one point narrower;
 *                     positions and phases stay double-double, grids are
 *                     assembled in FP64 and every other step is FP64.  Allowed
 *                     for eps >= 1e-7 (else NUHT_EPRECISION).
 *   dft_max           asymptotic blocks whose spread grid has at most this
 *                     many cells are evaluated by a direct sum over the grid
 *                     instead of an FFT and interpolation (0 -> built-in default,
 *                     negative -> always use the FFT path).
 *   spread_chunk      points per spreading work item, 64 .. 16384 (0 -> 1024).
 *   tune              nonzero: nuht_plan_many picks min_size, dft_max,
 *                     spread_chunk and split_candidates per size class with
 *                     nuht_tune (the fields above are then starting values).
 *   vector_spread     nonzero: every spreading work item runs on the vector
 *                     units.  By default, in FP64 with an ES width of at most
 *                     16 and at most 16 channels, items whose points reach the
 *                     grid from at most 6 first cells (many points per cell)
 *                     are spread on the matrix cores; the two give the same
 *                     sums up to rounding order.
 *   local_rank        0: the local rank L of Lemma 3.1 (Sec. 3.3); -1: the
 *                     smallest L whose dropped Wimp terms sum below eps / 2
 *                     at 512 points of (0, z] (tighter for large nu: 205
 *                     instead of 270 at nu = 100, eps = 1e-8); 1 .. 2000: that
 *                     L (the caller answers for the accuracy).
 *   margin            0 or 1: the expansion orders (M, z, L) and the ES width
 *                     are chosen for eps itself, as the paper prescribes
 *                     (Sec. 3.3), which bounds every matrix entry's error by
 *                     eps; summed over the many entries near the crossover
 *                     the output's normwise maximum error can exceed eps
 *                     (measured up to 6.6 eps at order 42, n = 5.5e5).
 *                     margin > 1 (at most 1000): they are chosen for
 *                     eps / margin.  Measured over 256 transforms of orders
 *                     0 .. 63 with n, m up to 1e6 at eps = 1e-12, the worst
 *                     normwise maximum error is 2.4 eps with margin 2,
 *                     0.98 eps with 4 and 0.54 eps with 8.  eps / margin must
 *                     stay >= 1e-15 (>= 1e-7 with FP32 spreading).
 *   tune_cache        NULL, or the path of a tuning cache file (JSON, one
 *                     entry per tuned key: size class floor(log10(n + m)),
 *                     channel count, local rank, ES width, precision, exact
 *                     split).  nuht_tune and the tuning of nuht_plan_many read
 *                     a key's options from it instead of timing candidates,
 *                     and write the options they time; the file is created
 *                     when missing and rewritten through a temporary file
 *                     (path + ".tmp") and a rename.  The string is read during
 *                     the call only (the plan keeps its own copy).
 */
typedef struct {
    int64_t min_size;
    int32_t M_override;
    int32_t split_candidates;
    int32_t precision;
    int32_t dft_max;
    int32_t spread_chunk;
    int32_t tune;
    int32_t vector_spread;
    int32_t local_rank;
    double  margin;
    const char *tune_cache;
} nuht_opts;

/*
 * Plan statistics and parameters (filled by nuht_plan_info).
 */
typedef struct {
    int32_t nu, M, L, es_width;       /* order, asymptotic terms, local rank, ES kernel width */
    double  eps, z, es_beta;          /* tolerance, crossover, ES kernel shape */
    int32_t levels;                   /* depth of the subdivision */
    int32_t n_nodes, n_local, n_asy, n_direct;
    int32_t n_fft_blocks;             /* asymptotic blocks using the FFT path */
    int64_t local_row_members, local_col_members;
    int64_t asy_row_members, asy_col_members;
    int64_t direct_entries;
    int64_t grid_cells;               /* sum of spread-grid sizes N1 over asymptotic blocks */
    int64_t fft_points;               /* sum of FFT sizes N2 over FFT-path blocks */
    int64_t dft_row_cells;            /* sum of rows x N1 over direct-sum-path blocks */
    int64_t fft_row_members;          /* sum of rows over FFT-path blocks */
    int64_t workspace_bytes;          /* device memory held by the plan */
    int64_t min_size;                 /* options in use (after defaults and tuning) */
    int32_t dft_max, spread_chunk;
    int32_t spread_items;             /* spreading work items of the asymptotic blocks */
    int32_t dense_items;              /* of which spread on the matrix cores */
    int32_t split_candidates;         /* candidate rows of SplitIndices in use (-1: exact) */
    int32_t half_order;               /* 1: the order is nu + 1/2 (nuht_plan_half) */
} nuht_info;

/*
 * nuht_plan -- prepare the transform r (n points) -> omega (m frequencies).
 *
 * Sorts r and omega on the device, computes (M, z, L) for (nu, eps) (Sec. 3.3),
 * and subdivides the matrix (Alg. 1).  Copies r and omega into plan-owned
 * storage, so the caller may free or change them afterwards.  The planning
 * runs on a stream of the library's, ordered after the work already queued
 * on `stream` (which may produce r and omega); the call waits once for that
 * planning work alone (to size the plan's workspace), not for the rest of
 * `stream`, so a plan made on a side stream overlaps the GPU's other work.
 * Later execute / adjoint calls may use any stream; a plan's buffers are
 * released only after the last of them.  Every argument is validated:
 * n, m >= 0; r_dev / omega_dev non-null when n / m > 0; |nu| <= 100;
 * 1e-15 <= eps <= 1e-2; all r, omega finite and >= 0 (else NUHT_EDOMAIN).
 * n == 0 or m == 0 is valid (the transform then writes zeros).  An
 * asymptotic block whose spread grid would need an FFT of more than 2^24
 * points per channel (half its point range times half its frequency range
 * above about 1.6e6 to 3.3e6, the grid spacing being a power of two) makes
 * the call fail with NUHT_ECAPACITY.
 */
int nuht_plan(nuht_plan_t *plan, int nu, double eps,
              int64_t n, const double *r_dev, int64_t m, const double *omega_dev,
              const nuht_opts *opts, void *stream);

/*
 * nuht_plan_half -- nuht_plan for integer or half-integer orders, the order
 * given twice: nu = nu2 / 2.  Even nu2 (|nu2| <= 200) is the integer order
 * nu2 / 2, exactly as nuht_plan.  Odd nu2 with 1 <= nu2 <= 199 is the
 * half-integer order nu = n + 1/2, n = (nu2 - 1) / 2 (the radial Fourier
 * transform in odd dimension d has nu = d/2 - 1).  The paper treats integer
 * orders (Sec. 3); at half-integers the same method runs with:
 *  - Hankel's expansion (Sec. 3.2), which ends at a_n (a_l = 0 for l > n):
 *    M is eq. num-asy-terms capped at ceil((n + 1) / 2); when the M terms
 *    are the whole expansion the crossover z is the smallest z >= 1 where
 *    the terms' magnitudes sum_k |a_k| z^-k are at most 10, else Newton's
 *    root of the bound of eq. asy-error (at least 1);
 *  - the local form J_{n+1/2}(omega r) = sqrt(r/R) sqrt(2x/pi)
 *    sum_l beta_{e+2l}(x) T_{e+2l}(r/R), x = omega R, e = n mod 2, the
 *    Chebyshev series of the spherical Bessel function j_n(x y) in y, with L
 *    from the Siegel bound of Lemma 3.1 applied to its coefficients
 *    (opts->local_rank = -1 is the same as 0 here);
 *  - J_{n+1/2} to full precision in the direct blocks.
 * Negative half-integer orders (the Y functions, singular at 0) are not
 * supported (NUHT_EINVAL).  nuht_gradient's dr and domega need nu >= 3/2
 * (orders nu -+ 1 are half-integers too).  All other entry points act on a
 * half-integer plan as on an integer one; nuht_plan_set_order and the
 * batches (nuht_plan_many) take integer orders.
 */
int nuht_plan_half(nuht_plan_t *plan, int nu2, double eps,
                   int64_t n, const double *r_dev, int64_t m, const double *omega_dev,
                   const nuht_opts *opts, void *stream);

/*
 * nuht_execute -- g = A c (forward transform, Alg. 2).
 *   c_dev: n weights in the caller's point order (as passed to nuht_plan).
 *   g_dev: m outputs in the caller's frequency order; overwritten.
 * Asynchronous on `stream`; allocates nothing.  The local moments and direct
 * blocks, which read only the gathered weights, run on a side stream the
 * library keeps per device and rejoin `stream` before the local rows, so the
 * call is ordered on `stream` as one sequence of kernels.  While `stream` is
 * being captured into a graph, or while the local-moment, direct or
 * local-row stages are timed (nuht_profile_stages), every stage runs on
 * `stream`.
 */
int nuht_execute(nuht_plan_t plan, const double *c_dev, double *g_dev, void *stream);

/*
 * nuht_adjoint -- cbar = A^T y, i.e. cbar_k = sum_j y_j J_nu(omega_j r_k).
 *   y_dev: m values in frequency order; cbar_dev: n outputs in point order
 *   (overwritten).  J_nu(omega r) is symmetric in its two factors, so this is
 *   the same method with the roles of points and frequencies exchanged; its
 *   partition is built on first use and kept in the plan.
 * Asynchronous on `stream` after its first call (the first call synchronises
 * once to size the transposed partition).
 */
int nuht_adjoint(nuht_plan_t plan, const double *y_dev, double *cbar_dev, void *stream);

/*
 * nuht_gradient -- derivatives of a loss L(g), g = A c, given gbar = dL/dg
 * (m values in frequency order), with respect to the weights, the points and
 * the frequencies:
 *   dc[k]     = sum_j gbar_j J_nu(omega_j r_k)                 (A^T gbar)
 *   dr[k]     = c_k sum_j gbar_j omega_j J_nu'(omega_j r_k)
 *   domega[j] = gbar_j sum_k c_k r_k J_nu'(omega_j r_k)
 * with J_nu' = (J_{nu-1} - J_{nu+1}) / 2 (J_{-1} = -J_1), so dr and domega
 * are two transposed and two forward transforms of orders nu -+ 1 on the
 * plan's sorted geometry (Sec. 3 applied at those orders).  Any of dc, dr,
 * domega may be NULL (not computed); c_dev may be NULL when neither dr nor
 * domega is asked for.  Outputs are in the caller's order and overwritten.
 * Orders nu -+ 1 need |nu| <= 100.  The partitions of the orders used are
 * built on the first call (one synchronisation each) and kept in the plan
 * (up to four orders), as are two n- and two m-sized temporaries; later calls
 * are asynchronous on `stream` and allocate nothing.
 */
int nuht_gradient(nuht_plan_t plan, const double *c_dev, const double *gbar_dev,
                  double *dc_dev, double *dr_dev, double *domega_dev, void *stream);

/*
 * nuht_gradient_noalloc -- nuht_gradient for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, outputs and ordering as
 * nuht_gradient (the same kernels in the same order, so the same values), but
 * the call allocates nothing and never builds a partition:
 *  - the four temporaries of dr and domega (two of n and two of m doubles)
 *    live in one library-wide device array of 64 MiB (8 388 608 doubles), one
 *    copy per device, held until the process ends, instead of in the plan;
 *    dr or domega requested with 2 (n + m) > 8 388 608 gives NUHT_ECAPACITY;
 *  - the partitions it runs (order nu transposed for dc; orders nu -+ 1,
 *    transposed for dr and forward for domega) must already be in the plan,
 *    built by an earlier nuht_gradient, nuht_adjoint or nuht_plan_set_order
 *    call, else NUHT_ENOTREADY and nothing is enqueued.
 * Every call on one device shares the array and overwrites it entirely before
 * reading it (nothing carries over from an earlier call); calls that overlap
 * on one device (different streams or threads without ordering) race on it.
 * The first call on a device looks up the array's address (no allocation).
 */
int nuht_gradient_noalloc(nuht_plan_t plan, const double *c_dev, const double *gbar_dev,
                          double *dc_dev, double *dr_dev, double *domega_dev, void *stream);

/*
 * nuht_plan_set_order -- switch the plan to order nu (same points, frequencies
 * and eps): (M, z, L) and the partition of that order are computed on the
 * sorted geometry (no new sort) the first time the order is used, which
 * synchronises `stream` once, and kept for later switches.
 */
int nuht_plan_set_order(nuht_plan_t plan, int nu, void *stream);

/* nuht_plan_info -- parameters and partition statistics of the current order. */
int nuht_plan_info(nuht_plan_t plan, nuht_info *info);

/*
 * nuht_plan_order -- the plan's sorted geometry.  The method works on points
 * and frequencies in increasing order (Thm. 4.1 and Alg. 1 assume it), so the
 * plan sorts both once; this copies, on `stream` (device pointers, each may be
 * NULL to skip it): r_sorted (n doubles, nondecreasing; -0.0 becomes +0.0),
 * perm_r (n int32: the caller's index of each sorted point, equal values in
 * the caller's order), and likewise omega_sorted and perm_omega (m each).
 * NUHT_EINVAL for a null plan.
 */
int nuht_plan_order(nuht_plan_t plan, double *r_sorted, int32_t *perm_r, double *omega_sorted,
                    int32_t *perm_omega, void *stream);

/*
 * nuht_tune -- pick the spreading work-item size, min_size, dft_max and (unless
 * the plan uses the exact split) split_candidates for this plan's geometry and
 * order: coordinate descent over a few candidates of each, every candidate
 * planned on the plan's sorted geometry and timed over `reps` executes
 * (0 -> 3) with HIP events on `stream` (c_dev: n weights, or NULL for all
 * ones; the timing does not depend on the values).  With a tuning cache (the
 * plan's opts.tune_cache) holding the plan's key, its options are taken
 * without timing; otherwise the timed result is added to the cache.  The best
 * options are written to *best (tune_cache NULL; their time per execute to
 * *best_ms, may be NULL) and adopted by the plan, whose partitions are
 * rebuilt.  Synchronises `stream` once per candidate.
 */
int nuht_tune(nuht_plan_t plan, const double *c_dev, int reps, nuht_opts *best, double *best_ms,
              void *stream);

/*
 * Batches of independent transforms (uneven n, m and order).
 *
 * nuht_plan_many -- plan `count` transforms: transform i maps n[i] points
 * r_dev[i] to m[i] frequencies omega_dev[i] at order nu[i], all with
 * tolerance eps and the options *opts (NULL: defaults).  Every argument is
 * validated as in nuht_plan.  Their sorts and subdivisions run on the batch's
 * own streams (four, default priority) after the work already queued on
 * `stream`, and the whole batch synchronises once (plus once more for any
 * transform whose tables had to grow).  With opts->tune set, the largest
 * transform of every size class (floor(log10(n + m))) is tuned first
 * (nuht_tune, timing with all-ones weights) and its options serve the class.
 *
 * nuht_execute_many -- g_dev[i] = A_i c_dev[i] for every transform (host arrays
 * of `count` device pointers; c_dev[i] in the caller's point order, g_dev[i]
 * overwritten in frequency order).  The first call captures every transform's
 * execution into one HIP graph: the transforms run concurrently on the
 * batch's streams (largest first, balanced by n + m) and read their input and
 * output addresses from a device table.  Each call writes the table with a
 * small kernel and replays the graph, ordered after the work already queued
 * on `stream` and before anything queued there later.  Asynchronous; it
 * allocates nothing after the first call.  Calls on one batch must not
 * overlap (they share the batch's buffers).
 *
 * nuht_batch_info -- nuht_plan_info of transform `index`.
 * nuht_batch_destroy -- synchronise the batch's streams and free it.
 */
typedef struct nuht_batch_s *nuht_batch_t;
int nuht_plan_many(nuht_batch_t *batch, int count, const int *nu, double eps,
                   const int64_t *n, const double *const *r_dev,
                   const int64_t *m, const double *const *omega_dev,
                   const nuht_opts *opts, void *stream);
int nuht_execute_many(nuht_batch_t batch, const double *const *c_dev, double *const *g_dev, void *stream);
int nuht_batch_info(nuht_batch_t batch, int index, nuht_info *info);
int nuht_batch_destroy(nuht_batch_t batch);

/*
 * Stage timing (diagnostics).  nuht_profile(plan, 1) clears and starts it:
 * every later nuht_execute / nuht_adjoint on the plan records HIP events on its
 * own stream between its NUHT_NSTAGES stages (0 gather of c, 1 local moments,
 * 2 ES spreading, 3 grid assembly, 4 FFTs, 5 direct blocks, 6 asymptotic rows,
 * 7 local rows and output).
 * nuht_profile(plan, 0)
 * stops it.  nuht_profile_stages(plan, mask) does the same for the stages
 * whose bits are set in mask (bit i: stage i; 0 stops), recording events only
 * at their boundaries, so that timing a few stages disturbs the execution
 * less; NUHT_EINVAL for bits beyond NUHT_NSTAGES.  nuht_profile_read
 * synchronises on the last recorded event and writes the per-stage totals in
 * milliseconds to stage_ms[NUHT_NSTAGES] (0 for stages not timed) and the
 * number of profiled calls to *calls (may be NULL).
 */
#define NUHT_NSTAGES 8
int nuht_profile(nuht_plan_t plan, int enable);
int nuht_profile_stages(nuht_plan_t plan, uint32_t mask);
int nuht_profile_read(nuht_plan_t plan, double *stage_ms, int64_t *calls);

/* nuht_destroy -- free the plan and its device memory (NULL is allowed). */
int nuht_destroy(nuht_plan_t plan);

/* nuht_strerror -- static description of an error code. */
const char *nuht_strerror(int code);

/*
 * nuht_direct -- brute-force O(nm) evaluation on the device of
 *   g_j = sum_k c_k J_nu(omega_j r_k)
 * with the library's own device J_nu (Hankel's M-term expansion above the
 * crossover z, Miller's recurrence below it; eps-accurate per entry).  A
 * reference for mid-sized checks, not a fast path.  Same argument conventions
 * as nuht_execute; asynchronous on `stream`.
 */
int nuht_direct(int nu, double eps, int64_t n, const double *r_dev, const double *c_dev,
                int64_t m, const double *omega_dev, double *g_dev, void *stream);

/*
 * Fourier-Bessel expansions on the unit disk and the Helmholtz solver on them
 * (Sec. 5.3).  A solver object holds the polar grid and the transforms of
 * orders 0 .. L between the radii and the zeros of J_l, planned once.
 *
 * nuht_fb_plan -- the grid: m radii r_dev in (0, 1] with radial weights wr_dev
 * (a quadrature rule for int_0^1 g(r) dr, e.g. Gauss-Legendre mapped to
 * [0, 1]) and t equispaced angles theta_s = 2 pi s / t (t a power of two,
 * 2 <= t <= 4096); orders l = -L .. L with 0 <= L <= 100 and 2L + 1 <= t; J
 * radial modes per order, zeros_dev holding (L + 1) x J values, row l being
 * j_{l,1} < ... < j_{l,J}, the first J positive zeros of J_l (the caller's;
 * the library does not compute them).  eps is the tolerance of every
 * transform.  method selects how the radial sums are taken:
 *   NUHT_FB_TRANSFORM (0): the transforms of this library, planned here for
 *     orders 0 .. L in both directions; cost O((L + 1)(m + J) log) per solve;
 *   NUHT_FB_DIRECT (1): the sums over m J terms per order, each J_l evaluated
 *     in place to full FP64 accuracy (eps is then unused but still checked);
 *     nothing is planned; cost O((L + 1) m J) Bessel evaluations per solve,
 *     the faster choice while m J is small (a few 10^5).
 * The arrays are copied; planning synchronises `stream`.
 *
 * nuht_fb_analysis -- the coefficients of eq. FB-coef with the grid's rules,
 * the angular integral taken as a mean (the eigenfunctions' squared norm being
 * pi J_{l+1}(j_{l,j})^2), so that f = sum alpha_jl J_l(j_{l,j} r) e^{i l theta}:
 *   alpha_jl = 2 / J_{l+1}(j_{l,j})^2 sum_k wr_k r_k J_l(j_{l,j} r_k)
 *              (1 / t) sum_s f(r_k, theta_s) e^{-i l theta_s}.
 *   f_dev: m x t real samples, row k = f(r_k, theta_0 .. theta_{t-1}).
 *   alpha_dev: (2L + 1) x J complex (re, im interleaved), row l + L.
 * nuht_fb_synthesis -- the expansion on the grid:
 *   u(r_k, theta_s) = Re sum_{l=-L..L} sum_j beta_jl J_l(j_{l,j} r_k) e^{i l theta_s},
 *   beta_dev as alpha_dev, u_dev as f_dev.
 * nuht_fb_helmholtz -- (Delta + kappa^2) u = f on the disk, u = 0 on the
 *   circle: analysis, beta_jl = alpha_jl / (kappa^2 - j_{l,j}^2) (the
 *   Dirichlet eigenvalues being -j_{l,j}^2), synthesis.  alpha_dev and
 *   beta_dev may be NULL (kept in the solver's own buffers); kappa^2 must not
 *   be an eigenvalue.
 * All three are asynchronous on `stream` and allocate nothing; calls on one
 * solver must not overlap.  nuht_fb_destroy synchronises and frees.
 */
typedef struct nuht_fb_s *nuht_fb_t;
#define NUHT_FB_TRANSFORM 0
#define NUHT_FB_DIRECT 1
int nuht_fb_plan(nuht_fb_t *fb, int32_t L, int64_t m, const double *r_dev, const double *wr_dev, int64_t t,
                 int64_t J, const double *zeros_dev, double eps, int32_t method, void *stream);
int nuht_fb_analysis(nuht_fb_t fb, const double *f_dev, double *alpha_dev, void *stream);
int nuht_fb_synthesis(nuht_fb_t fb, const double *beta_dev, double *u_dev, void *stream);
int nuht_fb_helmholtz(nuht_fb_t fb, double kappa, const double *f_dev, double *alpha_dev, double *beta_dev,
                      double *u_dev, void *stream);
int nuht_fb_destroy(nuht_fb_t fb);

#ifdef __cplusplus
}
#endif

#endif /* NUHT_H */
