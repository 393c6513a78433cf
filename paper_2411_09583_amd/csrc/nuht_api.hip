// nuht_api.hip -- host side of libnuht: expansion parameters (Sec. 3.3), ES
// kernel set-up, plan construction (sort, staircase, Alg. 1) and the C ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "nuht.h"
#include "nuht_launch.h"

namespace nuht {

// ===========================================================================
// Expansion parameters (Sec. 3.3).
// ===========================================================================

// M = min(floor(1 + nu/5 - log10(eps)/4), 20)   (eq. num-asy-terms)
static int num_asy_terms(int nu, double eps)
{
    int M = (int)std::floor(1.0 + std::fabs((double)nu) / 5.0 - std::log10(eps) / 4.0);
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
static double crossover(int nu, double eps, int M)
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

static void eshat_chebyshev(int w, double beta, double kappa_max, double* coef, int nc)
{
    std::vector<double> x, wt;
    gauss_legendre(240, x, wt);
    std::vector<double> f(nc);
    for (int j = 0; j < nc; ++j) {
        double t = std::cos(M_PI * (j + 0.5) / nc);
        double kappa = 0.5 * (t + 1.0) * kappa_max;
        long double s = 0.0L;
        for (size_t i = 0; i < x.size(); ++i) {
            double xx = x[i];
            double es = std::exp(beta * (std::sqrt(std::max(0.0, 1.0 - xx * xx)) - 1.0));
            s += (long double)wt[i] * es * std::cos(kappa * xx);
        }
        f[j] = (double)s;
    }
    for (int k = 0; k < nc; ++k) {
        long double s = 0.0L;
        for (int j = 0; j < nc; ++j) s += (long double)f[j] * std::cos(M_PI * k * (j + 0.5) / nc);
        coef[k] = (double)(2.0L * s / nc);
    }
    coef[0] *= 0.5;
    (void)w;
}

// The ES kernel as w polynomial pieces.  A point at grid coordinate u reaches
// the w cells l0 + t (t = 0 .. w-1), l0 = floor(u - w/2) + 1; with
// f = l0 - (u - w/2) in (0, 1], cell l0 + t sees ES((2 (t + f) - w) / w).
// Piece t is that function of s = 2 f - 1 on [-1, 1], interpolated at the
// kEsDeg + 1 Chebyshev points and rewritten in monomials of s, all in long
// double; coefficients are stored [t][d] (d = 0 .. kEsDeg).  Rounded to double
// and summed by Horner's rule they reproduce the kernel to ~6e-16 of its peak
// for w >= 15, and below the kernel's own truncation e^-beta for smaller w.
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

// -(2nu+1) pi/4 modulo 2 pi as a double-double in (0, 2 pi].
static void phase_offset(int nu, double& hi, double& lo)
{
    int k = 8 - ((2 * nu + 1) % 8);           // -(2nu+1) = k - 8(...)  (mod 8)
    const double q_hi = 0.78539816339744827900;   // pi/4 rounded
    const double q_lo = 3.0616169978683830e-17;   // pi/4 - q_hi
    double p = k * q_hi;                           // exact: k <= 8
    hi = p;
    lo = k * q_lo;
}

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

static int dev_alloc(DevBuf& b, size_t bytes, hipStream_t s)
{
    b = DevBuf{};
    if (bytes == 0) return NUHT_OK;
    void* p = nullptr;
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
    int nu_req = 0;
    double eps = 0.0;
    nuht_opts opts{};
    int64_t n = 0, m = 0;
    DevBuf b_geom;               // keys, values, sort scratch, summary, flag
    uint64_t* keys = nullptr;    // sorted points then sorted frequencies (bit patterns)
    int32_t* vals = nullptr;     // matching caller indices
    uint64_t* keys2 = nullptr;
    int32_t* vals2 = nullptr;
    int32_t* hist = nullptr;
    Summary* d_sum = nullptr;
    int32_t* d_flag = nullptr;   // domain error flag of the input check
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
    // stage timing (diagnostics): kStages + 1 events per profiled call
    bool prof = false;
    std::vector<hipEvent_t> prof_events;
    int64_t prof_calls = 0;
};

static void prof_clear(nuht_plan_t p)
{
    for (hipEvent_t e : p->prof_events) (void)hipEventDestroy(e);
    p->prof_events.clear();
    p->prof_calls = 0;
}

// Events for one profiled execute call, or null when profiling is off.
static hipEvent_t* prof_marks(nuht_plan_t p)
{
    if (!p->prof) return nullptr;
    size_t base = p->prof_events.size();
    for (int i = 0; i <= kStages; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
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

static void fill_params(PlanDev& P, int nu, double eps, const nuht_opts& o)
{
    int anu = std::abs(nu);
    P.nu = anu;
    P.sign = (nu < 0 && (anu & 1)) ? -1 : 1;
    P.eps = eps;
    int M = o.M_override > 0 ? std::min(o.M_override, 20) : num_asy_terms(anu, eps);
    P.M = M;
    P.nch = padded_channels(2 * M);
    P.z = crossover(anu, eps, M);
    P.L = local_rank(anu, eps, P.z);
    P.w = es_width(eps, o.precision);
    P.beta = es_beta(P.w);
    for (int p = 0; p < 2 * M + 2; ++p) P.hank[p] = hankel_coef(anu, p);
    for (int p = 0; p < kMaxChannels; ++p)
        P.chan[p] = p < 2 * M ? (((p >> 1) & 1) ? -P.hank[p] : P.hank[p]) : 0.0;
    phase_offset(anu, P.phi_hi, P.phi_lo);
    P.kappa_max = P.w * M_PI / 4.0 * (1.0 + 1e-9);
    P.n_eshat = 30;
    // the Chebyshev series depends only on the kernel width (beta follows w)
    static std::mutex mu;
    static double cache[32][32];
    static bool have[32] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (!have[P.w]) {
        eshat_chebyshev(P.w, P.beta, P.kappa_max, cache[P.w], P.n_eshat);
        have[P.w] = true;
    }
    for (int i = 0; i < P.n_eshat; ++i) P.eshat[i] = cache[P.w][i];
}

static int build_partition(nuht_plan_t pl, Partition& Pt, const Geometry& G, int nu, hipStream_t s)
{
    Pt.release();
    Pt.stream = s;
    const nuht_opts& o = pl->opts;
    PlanDev& P = Pt.P;
    P = PlanDev{};
    fill_params(P, nu, pl->eps, o);
    if (P.L < 0) return NUHT_EINVAL;
    P.n = G.n; P.m = G.m;
    P.rs = G.rs; P.ws = G.ws; P.perm_r = G.perm_r; P.perm_w = G.perm_w;
    Pt.sum = Summary{};
    if (G.n == 0 || G.m == 0) {
        std::unique_lock<std::mutex> lock;
        HostStage* h = host_stage(lock);
        if (!h) return NUHT_ENOMEM;
        HIP_TRY(hipMemcpyAsync(&h->flag, pl->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (h->flag) return NUHT_EDOMAIN;
        Pt.built = true;
        return NUHT_OK;
    }

    int64_t min_size = o.min_size > 0 ? o.min_size : 1024;
    int ncand = o.split_candidates > 1 ? o.split_candidates : 16;
    int dft_max = o.dft_max == 0 ? 48 : o.dft_max;
    const double sigma = 2.0;

    int64_t tot = (int64_t)G.n + G.m;
    int32_t cap = (int32_t)std::min<int64_t>(tot / 32 + 4096, 1 << 28);
    int32_t icap = (int32_t)std::min<int64_t>(64 * (tot / kSpreadChunk) + 2 * (int64_t)cap, 1 << 28);
    Summary& S = Pt.sum;
    for (int attempt = 0; attempt < 6; ++attempt) {
        Partition tmp;   // this attempt's tables; dropped on a retry
        tmp.stream = s;
        Arena A{};
        A.node_cap = cap; A.l_cap = cap; A.a_cap = cap; A.d_cap = 2 * cap; A.q_cap = cap;
        A.litem_cap = icap; A.aitem_cap = icap;
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
        slab.add(A.fft_list, (size_t)A.a_cap);
        slab.add(A.gslot, (size_t)A.a_cap + 1);
        NUHT_TRY(slab.commit(tmp));
        P.nodes = A.nodes; P.lb = A.lb; P.ab = A.ab; P.db = A.db;
        P.litems = A.litems; P.aitems = A.aitems; P.fft_list = A.fft_list; P.gslot = A.gslot;
        HIP_TRY(hipMemsetAsync(pl->d_sum, 0, sizeof(Summary), s));
        HIP_TRY(launch_planning(P, A, K, Jc, a_cells, min_size, ncand, dft_max, sigma, pl->d_sum, s));
        int32_t flag = 0;
        {
            std::unique_lock<std::mutex> lock;
            HostStage* h = host_stage(lock);
            if (!h) return NUHT_ENOMEM;
            HIP_TRY(hipMemcpyAsync(&h->sum, pl->d_sum, sizeof(Summary), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(&h->flag, pl->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            S = h->sum;
            flag = h->flag;
        }
        if (flag) return NUHT_EDOMAIN;
        if (S.overflow == 2) return NUHT_ECAPACITY;   // subdivision deeper than kMaxLevels
        if (S.grid_error) return NUHT_ECAPACITY;
        if (S.overflow) {
            int64_t need = std::max<int64_t>({(int64_t)S.n_nodes, (int64_t)S.n_l, (int64_t)S.n_a, (int64_t)S.n_d / 2});
            if (need >= cap) cap = (int32_t)std::min<int64_t>(2 * need + 1024, 1 << 29);
            int64_t ineed = std::max<int64_t>((int64_t)S.n_litems, (int64_t)S.n_aitems);
            if (ineed >= icap) icap = (int32_t)std::min<int64_t>(2 * ineed + 1024, 1 << 29);
            if (need < cap && ineed < icap) { cap *= 2; icap *= 2; }
            continue;
        }
        // keep this attempt's tables
        for (auto& b : tmp.bufs) Pt.bufs.push_back(b);
        Pt.bytes += tmp.bytes;
        tmp.bufs.clear();
        tmp.bytes = 0;
        Pt.A = A;
        break;
    }
    if (S.overflow) return NUHT_ECAPACITY;
    P.n_nodes = S.n_nodes; P.n_l = S.n_l; P.n_a = S.n_a; P.n_d = S.n_d;
    P.n_litems = S.n_litems; P.n_aitems = S.n_aitems;

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
    slab.add(B.es_poly, (size_t)P.w * (kEsDeg + 1));
    NUHT_TRY(slab.commit(Pt));
    HIP_TRY(hipMemcpyAsync(B.es_poly, es_pieces_cached(P.w, P.beta), sizeof(double) * P.w * (kEsDeg + 1),
                           hipMemcpyHostToDevice, s));
    P.es_poly = B.es_poly;
    Pt.built = true;
    return NUHT_OK;
}

static void free_plan(nuht_plan_t p)
{
    if (!p) return;
    prof_clear(p);
    p->orders.clear();
    dev_free(p->b_grad);
    dev_free(p->b_geom);
    delete p;
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
            if (p->orders[i]->nu != p->nu_req &&
                (victim == p->orders.size() || p->orders[i]->used < p->orders[victim]->used))
                victim = i;
        if (victim < p->orders.size()) p->orders.erase(p->orders.begin() + victim);
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
        int rc = build_partition(p, Pt, transposed ? p->adj : p->fwd, nu, s);
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
        if (o->nu == p->nu_req && o->f.built) return &o->f;
    return nullptr;
}

static int run(nuht_plan_t p, const Partition& Pt, const double* in, double* out, bool scale, hipStream_t s)
{
    HIP_TRY(launch_execute(Pt.P, Pt.sum, Pt.B, Pt.cls.data(), (int)Pt.cls.size(), in, out, scale, s,
                           prof_marks(p)));
    return NUHT_OK;
}

static bool valid_common(int nu, double eps)
{
    if (nu < -100 || nu > 100) return false;
    if (!(eps >= 1e-15 && eps <= 1e-2)) return false;
    return true;
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
        default: return "unknown error";
    }
}

int nuht_plan(nuht_plan_t* out, int nu, double eps, int64_t n, const double* r_dev, int64_t m,
              const double* omega_dev, const nuht_opts* opts, void* stream)
{
    if (!out) return NUHT_EINVAL;
    *out = nullptr;
    if (!valid_common(nu, eps)) return NUHT_EINVAL;
    if (n < 0 || m < 0 || n > INT32_MAX / 2 || m > INT32_MAX / 2) return NUHT_EINVAL;
    if ((n > 0 && !r_dev) || (m > 0 && !omega_dev)) return NUHT_EINVAL;
    nuht_opts o{};
    if (opts) o = *opts;
    if (o.precision != NUHT_FP64 && o.precision != NUHT_FP32_SPREAD) return NUHT_EINVAL;
    if (o.precision == NUHT_FP32_SPREAD) return NUHT_EPRECISION;   // FP64 path only in this build
    if (o.min_size < 0 || o.M_override < 0 || o.M_override > 20 || o.split_candidates < 0) return NUHT_EINVAL;
    hipStream_t s = (hipStream_t)stream;

    nuht_plan_s* p = new (std::nothrow) nuht_plan_s();
    if (!p) return NUHT_ENOMEM;
    p->nu_req = nu; p->eps = eps; p->opts = o; p->n = n; p->m = m;
    int64_t tot = n + m;
    auto fail = [&](int code) { free_plan(p); return code; };
    {
        Slab slab;
        slab.add(p->d_sum, 1);
        slab.add(p->d_flag, 1);
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
    if (hipMemsetAsync(p->d_flag, 0, sizeof(int32_t), s) != hipSuccess) return fail(NUHT_EHIP);
    if (launch_make_keys(r_dev, (int32_t)n, p->keys, p->vals, p->d_flag, s) != hipSuccess) return fail(NUHT_EHIP);
    if (launch_make_keys(omega_dev, (int32_t)m, p->keys + n, p->vals + n, p->d_flag, s) != hipSuccess)
        return fail(NUHT_EHIP);
    if (launch_sort_pairs(p->keys, p->vals, p->keys2, p->vals2, p->hist, (int32_t)n, (int32_t)m, s) != hipSuccess)
        return fail(NUHT_EHIP);
    p->fwd.n = (int32_t)n; p->fwd.m = (int32_t)m;
    p->fwd.rs = (const double*)p->keys;
    p->fwd.ws = (const double*)(p->keys + n);
    p->fwd.perm_r = p->vals;
    p->fwd.perm_w = p->vals + n;
    p->adj.n = (int32_t)m; p->adj.m = (int32_t)n;
    p->adj.rs = p->fwd.ws; p->adj.ws = p->fwd.rs;
    p->adj.perm_r = p->fwd.perm_w; p->adj.perm_w = p->fwd.perm_r;
    // the one synchronisation of the plan happens inside (it also reads the
    // input check's flag)
    p->nu_req = nu;
    Partition* Pt = nullptr;
    int rc = get_partition(p, nu, false, s, &Pt);
    if (rc != NUHT_OK) return fail(rc);
    *out = p;
    return NUHT_OK;
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
    int rc = get_partition(p, p->nu_req, true, s, &Pt);
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
    const int nu = p->nu_req;
    if ((want_r || want_w) && std::abs(nu) + 1 > 101) return NUHT_EINVAL;
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
        if ((rc = get_partition(p, nu - 1, true, s, &Pt)) != NUHT_OK) return rc;
        if ((rc = run(p, *Pt, gbar_dev, p->grad_t[0], true, s)) != NUHT_OK) return rc;
        if ((rc = get_partition(p, nu + 1, true, s, &Pt)) != NUHT_OK) return rc;
        if ((rc = run(p, *Pt, gbar_dev, p->grad_t[1], true, s)) != NUHT_OK) return rc;
        HIP_TRY(launch_half_difference(c_dev, p->grad_t[0], p->grad_t[1], dr_dev, (int32_t)p->n, s));
    }
    if (want_w && p->m > 0) {            // dL/domega = (gbar/2) (A_{nu-1} - A_{nu+1})(r c)
        if ((rc = get_partition(p, nu - 1, false, s, &Pt)) != NUHT_OK) return rc;
        if ((rc = run(p, *Pt, c_dev, p->grad_t[2], true, s)) != NUHT_OK) return rc;
        if ((rc = get_partition(p, nu + 1, false, s, &Pt)) != NUHT_OK) return rc;
        if ((rc = run(p, *Pt, c_dev, p->grad_t[3], true, s)) != NUHT_OK) return rc;
        HIP_TRY(launch_half_difference(gbar_dev, p->grad_t[2], p->grad_t[3], domega_dev, (int32_t)p->m, s));
    }
    return NUHT_OK;
}

int nuht_plan_set_order(nuht_plan_t p, int nu, void* stream)
{
    if (!p) return NUHT_EINVAL;
    if (!valid_common(nu, p->eps)) return NUHT_EINVAL;
    const int prev = p->nu_req;
    p->nu_req = nu;
    Partition* Pt = nullptr;
    int rc = get_partition(p, nu, false, (hipStream_t)stream, &Pt);
    if (rc != NUHT_OK) p->nu_req = prev;
    return rc;
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
    info->nu = p->nu_req; info->M = P.M; info->L = P.L; info->es_width = P.w;
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
    return NUHT_OK;
}

int nuht_profile(nuht_plan_t p, int enable)
{
    if (!p) return NUHT_EINVAL;
    prof_clear(p);
    p->prof = enable != 0;
    return NUHT_OK;
}

int nuht_profile_read(nuht_plan_t p, double* stage_ms, int64_t* calls)
{
    if (!p || !stage_ms) return NUHT_EINVAL;
    for (int i = 0; i < kStages; ++i) stage_ms[i] = 0.0;
    int64_t nc = (int64_t)p->prof_events.size() / (kStages + 1);
    if (nc > 0) HIP_TRY(hipEventSynchronize(p->prof_events.back()));
    for (int64_t c = 0; c < nc; ++c) {
        hipEvent_t* e = p->prof_events.data() + c * (kStages + 1);
        for (int i = 0; i < kStages; ++i) {
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
    fill_params(P, nu, eps, o);
    if (m == 0) return NUHT_OK;
    if (n == 0) { HIP_TRY(hipMemsetAsync(g_dev, 0, sizeof(double) * (size_t)m, s)); return NUHT_OK; }
    HIP_TRY(launch_direct(P, r_dev, c_dev, (int32_t)n, omega_dev, (int32_t)m, g_dev, s));
    return NUHT_OK;
}

}  // extern "C"
