// nuht_launch.h -- device tables of a partition and the host-side launchers.
#pragma once

#include <vector>

#include "nuht_internal.h"

namespace nuht {

struct Rect {
    int32_t j0, j1, k0, k1;
};

// Device tables of one partition, with their capacities.  The planning
// kernels write them; if any capacity is exceeded they report overflow in the
// Summary and the host retries with larger tables.
struct Arena {
    Node* nodes;
    LBlock* lb;
    ABlock* ab;
    DBlock* db;
    Rect* q0;
    Rect* q1;
    Item* litems;
    Item* aitems;
    int32_t* alist;      // spreading order of the asymptotic items (aitem_cap)
    int32_t* fft_list;
    int64_t* gslot;      // first grid slot of each asymptotic block, then the total (a_cap + 1)
    int32_t node_cap, l_cap, a_cap, d_cap, q_cap, litem_cap, aitem_cap, pad;
};

// planning (plan.hip)
// Keys (bit patterns) of r (na values) and w (nb values) sorted into (k0, v0)
// with their caller indices, (k1, v1) and hist (sort_hist_len ints) as
// scratch; errs[t] (sort_tiles entries) = 1 for each tile of the inputs that
// holds a negative, NaN or infinite value, else 0.
hipError_t launch_keys_and_sort(const double* r, int32_t na, const double* w, int32_t nb, uint64_t* k0, int32_t* v0,
                                uint64_t* k1, int32_t* v1, int32_t* hist, int32_t* errs, hipStream_t s);
int sort_tiles(int32_t na, int32_t nb);
int sort_hist_len(int32_t na, int32_t nb);
// *flag = 1 if any of errs[0 .. n-1] is set, else 0
hipError_t launch_reduce_errs(const int32_t* errs, int32_t n, int32_t* flag, hipStream_t s);
// Staircases, subdivision (Alg. 1), block parameters, work items and their
// offsets, all on the device; counts and totals are left in *sum.
// The summary is cleared first; its domain_error is set from the input
// check's tile flags (errs, n_errs entries).
hipError_t launch_planning(const PlanDev& P, const Arena& A, int32_t* K, int32_t* Jc, int32_t* a_cells,
                           int64_t min_size, int32_t ncand, int32_t dft_max, double sigma, Summary* sum,
                           const int32_t* errs, int32_t n_errs, hipStream_t s);

// execution (exec.hip)
struct ExecBuffers {
    double* cs;         // gathered weights (sorted point order)
    double* lpart;      // local-moment partial sums, n_litems x (L+1)
    double* lmom;       // local moments, n_l x (L+1)
    double2* part;      // spread partial subgrids
    double2* grids;     // spread grids (direct-sum path) and FFT buffers (FFT path)
    double2* scratch;   // second buffer of the two-pass FFTs
    double* gd;         // per-row direct-block sums (m)
    double* ga;         // per-row asymptotic sums (m)
    const double* es_poly;  // ES kernel pieces (w x (kEsDeg + 1)), shared by all plans on the device
    const double2* fft_tw;  // FFT twiddles (8192 entries), shared by all plans on the device
    int64_t grid_cells; // grid slots (without the channel factor)
};

struct FftClass {
    int32_t log2n, count, first;
    int64_t scratch_off;   // complex elements
};

// Execution stages, timed between consecutive events of `marks` (kStages + 1
// events, or null; a null entry records nothing).
constexpr int kStages = 8;   // gather, local moments, spread, grid assembly, FFT, direct, asymptotic rows, local rows
// Input and output of one transform.  When the slots are set, the kernels
// read the input and output pointers from those device locations at run time
// (so a captured graph serves any buffers); otherwise c and g are used.  With
// scale_by_points the input is multiplied by the geometry's sorted point
// coordinates as it is gathered (r c for the forward geometry, omega y for
// the transposed one).
struct IoArgs {
    const double* c = nullptr;
    double* g = nullptr;
    const double* const* c_slot = nullptr;
    double* const* g_slot = nullptr;
    bool scale_by_points = false;
};

// A second stream for the stages that depend only on the gathered weights
// (local moments, direct blocks): after the gather `s` records ev_fork, `side`
// waits for it and runs them, records ev_join, and `s` waits for ev_join before
// the local rows, the first stage to read their results.
struct ExecFork {
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

// One transform with the plan's partition: out = A in (or A^T in on the
// transposed geometry).  With `fork` the local moments and direct blocks run
// on its side stream, beside the spreading, grid assembly and FFT; without,
// every stage runs on `s` in order.
hipError_t launch_execute(const PlanDev& P, const Summary& S, const ExecBuffers& B, const FftClass* cls, int ncls,
                          const IoArgs& io, hipStream_t s, hipEvent_t* marks, const ExecFork* fork = nullptr);
// Fills P.small, the FFT size classes of at most 4096 points, from the
// partition's classes.
void small_fft_table(PlanDev& P, const FftClass* cls, int ncls);

// A batch of transforms executed stage by stage: every stage (and kernel
// variant: channel count, precision, local-row mode) is one launch over all
// transforms with work in it, each workgroup finding its transform in a table
// of segments.  Built once on the host; its device tables (the transforms'
// PlanDev array, the segments) are one block of bytes, `table`, that the
// caller copies to device memory and passes to launch_execute_many.
struct BatchTransform {
    const PlanDev* P;
    const Summary* S;
    const FftClass* cls;
    int ncls;
};
struct BatchLaunch {
    int32_t kind, variant, fp32;
    int32_t seg0, nseg;          // segments seg0 .. seg0 + nseg - 1 (WorkSeg or FFT segments by kind)
    int32_t blocks, threads;
    size_t lds;
};
struct BatchSchedule {
    std::vector<BatchLaunch> launches;
    std::vector<char> table;     // PlanDev[count], then the WorkSeg segments, then the FFT segments
    size_t segs_off = 0, fsegs_off = 0;
};
// `order`: the transforms in the order their workgroups are laid out in every
// launch (largest first).
void build_batch_schedule(const BatchTransform* tr, int count, const int* order, BatchSchedule& out);
hipError_t launch_execute_many(const BatchSchedule& S, const void* table_dev, void* const* c_table,
                               void* const* g_table, hipStream_t s,
                               const ExecFork* fork = nullptr);
// x[i] = v
hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s);
// -(2 nu + 1) pi / 4 modulo 2 pi as a double-double (the Hankel phase offset).
void phase_offset_dd(int nu, double* hi, double* lo);
// table[i] = ptrs[i] for i < count (count <= 224): fills a device pointer table
// from kernel arguments
hipError_t launch_set_pointers(void** table, const void* const* ptrs, int count, hipStream_t s);
// out[i] = w[i] (a[i] - b[i]) / 2
hipError_t launch_half_difference(const double* w, const double* a, const double* b, double* out, int32_t n,
                                  hipStream_t s);
hipError_t launch_direct(const PlanDev& P, const double* r, const double* c, int32_t n, const double* w, int32_t m,
                         double* g, hipStream_t s);

}  // namespace nuht
