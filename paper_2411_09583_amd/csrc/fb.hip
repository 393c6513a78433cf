// Fourier-Bessel expansions on the unit disk and the Helmholtz solver built on
// them (Sec. 5.3): the coefficients of a forcing f sampled on a polar grid
// (eq. FB-coef), the expansion's values on that grid, and the solution of
// (Delta + kappa^2) u = f, u(1, theta) = 0, by dividing the coefficients by
// the eigenvalues lambda_jl + kappa^2 = kappa^2 - j_{l,j}^2.
//
// Grid: m radii r_k in (0, 1] with radial weights wr_k (a rule for
// int_0^1 g(r) dr) and t = 2^q angles theta_s = 2 pi s / t.  Orders
// l = -L .. L (2L + 1 <= t, L <= 100), radial indices j = 1 .. J.
//
// Analysis, for every order l (eq. FB-coef with the angular integral taken as
// a mean, (1 / 2 pi) int d theta: int int |psi_jl|^2 r dr d theta =
// pi J_{l+1}(j_{l,j})^2, so the factor 2 / J_{l+1}^2 goes with the mean):
//   F_l(r_k)  = (1 / t) sum_s f(r_k, theta_s) e^{-i l theta_s}            (t-point FFT per radius)
//   a_jl      = sum_k wr_k r_k F_l(r_k) J_l(j_{l,j} r_k)                (a transform of order |l|,
//                                                                         points r, frequencies j_{|l|,.})
//   alpha_jl  = 2 a_jl / J_{l+1}(j_{l,j})^2
// with J_{-l} = (-1)^l J_l, so orders l and -l share the plan of |l|, and
// J_{l+1}(j_{l,j})^2 = J_{l-1}(j_{l,j})^2 (J_{l-1} + J_{l+1} = (2l/x) J_l
// vanishes at a zero of J_l), evaluated at order |l| - 1 (1 for l = 0).
// Synthesis, for every order l (the transposed transforms, points j_{|l|,.},
// frequencies r):
//   U_l(r_k)  = sum_j beta_jl J_l(j_{l,j} r_k)
//   u(r_k, theta_s) = Re sum_l U_l(r_k) e^{i l theta_s}                  (t-point FFT per radius)
// Real and imaginary parts of the complex weights are separate transforms,
// two per order |l| = a in each direction:
//  - f is real, so F_{-a} = conj(F_a) and a_{j,-a} = (-1)^a conj(a_{j,a}):
//    the analysis transforms (re, im) of F_a alone;
//  - only the real part of the synthesis is kept, and
//    Re(U_a e^{i a theta} + U_{-a} e^{-i a theta}) = Re(V_a e^{i a theta}) with
//    V_a = U_a + conj(U_{-a}) = sum_j (beta_{j,a} + (-1)^a conj(beta_{j,-a})) J_a(j_{a,j} r),
//    one complex sum of order a (V_0 = U_0).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "nuht.h"
#include "nuht_device.h"
#include "nuht_launch.h"

namespace nuht {

// One radius per workgroup: the t real samples f(r_k, .) in LDS, the FFT
// (e^{+}), then for 0 <= l <= L the weights wr_k r_k F_l(r_k),
// F_l = (1 / t) conj(X[l]) (f real), written as two weight vectors per order:
// C[(2 l + q) m + k], q = 0 (re), 1 (im).
__global__ __launch_bounds__(256) void k_fb_angular_fwd(const double* __restrict__ f, int64_t m, int logt, int L,
                                                        const double* __restrict__ r, const double* __restrict__ wr,
                                                        double* __restrict__ C)
{
    extern __shared__ double2 sm[];
    const int t = 1 << logt;
    const int64_t k = blockIdx.x;
    const double* fk = f + k * t;
    for (int s = threadIdx.x; s < t; s += blockDim.x) sm[s] = make_double2(fk[s], 0.0);
    __syncthreads();
    lds_fft(sm, t, logt, 1, 0, 1);
    __syncthreads();
    const double scale = wr[k] * r[k] / t;
    for (int l = threadIdx.x; l <= L; l += blockDim.x) {
        const double2 xp = sm[l];              // X[l]: F_l = scale conj(X[l])
        C[(2 * (int64_t)l + 0) * m + k] = scale * xp.x;
        C[(2 * (int64_t)l + 1) * m + k] = -scale * xp.y;
    }
}

// alpha[(l + L) J + j] (complex) from the transform outputs
// G[(2 |l| + q) J + j] and the factors nrm[|l| J + j] = 2 / J_{l+1}(j_{l,j})^2;
// order -l is (-1)^l times the conjugate of order l.
__global__ void k_fb_scale(const double* __restrict__ G, const double* __restrict__ nrm, int L, int64_t J,
                           double2* __restrict__ alpha)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)(2 * L + 1) * J;
    if (e >= total) return;
    const int li = (int)(e / J);
    const int64_t j = e - (int64_t)li * J;
    const int l = li - L, a = l < 0 ? -l : l;
    const double sg = (l < 0 && (a & 1)) ? -1.0 : 1.0;
    const double s = sg * nrm[(int64_t)a * J + j];
    const double im = G[(2 * (int64_t)a + 1) * J + j];
    alpha[e] = make_double2(s * G[2 * (int64_t)a * J + j], l < 0 ? -s * im : s * im);
}

// beta = alpha / (kappa^2 - j_{|l|,j}^2).
__global__ void k_fb_helmholtz(const double2* __restrict__ alpha, const double* __restrict__ zeros, int L,
                               int64_t J, double kappa, double2* __restrict__ beta)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)(2 * L + 1) * J;
    if (e >= total) return;
    const int li = (int)(e / J);
    const int64_t j = e - (int64_t)li * J;
    const int a = li >= L ? li - L : L - li;
    const double z = zeros[(int64_t)a * J + j];
    const double d = 1.0 / ((kappa - z) * (kappa + z));
    const double2 v = alpha[e];
    beta[e] = make_double2(v.x * d, v.y * d);
}

// The synthesis weights of order a = 0 .. L: B[(2 a + q) J + j] = (re, im) of
// beta_{j,a} + (-1)^a conj(beta_{j,-a}) (beta_{j,0} for a = 0), from
// beta[(l + L) J + j].
__global__ void k_fb_split(const double2* __restrict__ beta, int L, int64_t J, double* __restrict__ Bw)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)(L + 1) * J;
    if (e >= total) return;
    const int a = (int)(e / J);
    const int64_t j = e - (int64_t)a * J;
    double2 v = beta[(int64_t)(L + a) * J + j];
    if (a > 0) {
        const double2 w = beta[(int64_t)(L - a) * J + j];
        const double sg = (a & 1) ? -1.0 : 1.0;
        v.x += sg * w.x;
        v.y -= sg * w.y;
    }
    Bw[2 * (int64_t)a * J + j] = v.x;
    Bw[(2 * (int64_t)a + 1) * J + j] = v.y;
}

// One radius per workgroup: the spectrum S[a] = V_a(r_k) for 0 <= a <= L
// (zero elsewhere) from U[(2 a + q) m + k], the FFT (e^{+}), and
// u(r_k, theta_s) = Re X[s].
__global__ __launch_bounds__(256) void k_fb_angular_inv(const double* __restrict__ U, int64_t m, int logt, int L,
                                                        double* __restrict__ u)
{
    extern __shared__ double2 sm[];
    const int t = 1 << logt;
    const int64_t k = blockIdx.x;
    for (int s = threadIdx.x; s < t; s += blockDim.x) sm[s] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int l = threadIdx.x; l <= L; l += blockDim.x)
        sm[l] = make_double2(U[(2 * (int64_t)l + 0) * m + k], U[(2 * (int64_t)l + 1) * m + k]);
    __syncthreads();
    lds_fft(sm, t, logt, 1, 0, 1);
    __syncthreads();
    double* uk = u + k * t;
    for (int s = threadIdx.x; s < t; s += blockDim.x) uk[s] = sm[s].x;
}

// The direct method: the same radial sums with every J_l(j_{l,j} r_k)
// evaluated in place (full FP64 accuracy), shared by the two weight vectors
// of order l.  A workgroup of 16 waves owns 64 outputs of one order (one per
// lane); its waves take every 16th term of the sum, and the 16 partial sums
// are added in wave order.  Lanes past the end evaluate J at x = 0 and write
// nothing.
constexpr int kFbWaves = 16;

// Analysis: G[(2 l + q) J + j] = sum_k C[(2 l + q) m + k] J_l(z_{l,j} r_k).
__global__ __launch_bounds__(1024) void k_fb_direct_fwd(const double* __restrict__ C, const double* __restrict__ r,
                                                        int64_t m, const double* __restrict__ zeros, int64_t J,
                                                        const double* __restrict__ phi, double* __restrict__ G)
{
    __shared__ double red[kFbWaves][2][64];
    const int l = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + lane;
    const double z = j < J ? zeros[(int64_t)l * J + j] : 0.0;
    const double ph = phi[2 * l], pl = phi[2 * l + 1];
    const double* c0 = C + 2 * (int64_t)l * m;
    double a0 = 0.0, a1 = 0.0;
    for (int64_t k = w; k < m; k += kFbWaves) {
        const double rk = r[k];
        const double x = z * rk;
        const double v = besselj_core(l, ph, pl, x, __builtin_fma(z, rk, -x));
        a0 = __builtin_fma(c0[k], v, a0);
        a1 = __builtin_fma(c0[m + k], v, a1);
    }
    red[w][0][lane] = a0; red[w][1][lane] = a1;
    __syncthreads();
    if (threadIdx.x < 128) {
        const int q = threadIdx.x >> 6;
        double s = 0.0;
        #pragma unroll
        for (int v = 0; v < kFbWaves; ++v) s += red[v][q][lane];
        if (j < J) G[(2 * (int64_t)l + q) * J + j] = s;
    }
}

// Synthesis: U[(2 l + q) m + k] = sum_j B[(2 l + q) J + j] J_l(z_{l,j} r_k).
__global__ __launch_bounds__(1024) void k_fb_direct_inv(const double* __restrict__ B, const double* __restrict__ r,
                                                        int64_t m, const double* __restrict__ zeros, int64_t J,
                                                        const double* __restrict__ phi, double* __restrict__ U)
{
    __shared__ double red[kFbWaves][2][64];
    const int l = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t k = (int64_t)blockIdx.x * 64 + lane;
    const double rk = k < m ? r[k] : 0.0;
    const double ph = phi[2 * l], pl = phi[2 * l + 1];
    const double* b0 = B + 2 * (int64_t)l * J;
    const double* zl = zeros + (int64_t)l * J;
    double a0 = 0.0, a1 = 0.0;
    for (int64_t j = w; j < J; j += kFbWaves) {
        const double z = zl[j];
        const double x = z * rk;
        const double v = besselj_core(l, ph, pl, x, __builtin_fma(z, rk, -x));
        a0 = __builtin_fma(b0[j], v, a0);
        a1 = __builtin_fma(b0[J + j], v, a1);
    }
    red[w][0][lane] = a0; red[w][1][lane] = a1;
    __syncthreads();
    if (threadIdx.x < 128) {
        const int q = threadIdx.x >> 6;
        double s = 0.0;
        #pragma unroll
        for (int v = 0; v < kFbWaves; ++v) s += red[v][q][lane];
        if (k < m) U[(2 * (int64_t)l + q) * m + k] = s;
    }
}

// 2 / J^2 in place.
__global__ void k_fb_norm(double* __restrict__ v, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) {
        const double x = v[e];
        v[e] = 2.0 / (x * x);
    }
}

static inline int blocks_for(int64_t n) { return (int)((n + 255) / 256); }

}  // namespace nuht

using namespace nuht;

struct nuht_fb_s {
    int L = 0, logt = 0;
    int64_t m = 0, t = 0, J = 0;
    double* r = nullptr;        // m radii
    double* wr = nullptr;       // m radial weights
    double* zeros = nullptr;    // (L + 1) x J
    double* nrm = nullptr;      // (L + 1) x J: 2 / J_{l+1}(j_{l,j})^2
    double* C = nullptr;        // 2 (L + 1) x m analysis weights
    double* G = nullptr;        // 2 (L + 1) x J analysis outputs / synthesis weights
    double* U = nullptr;        // 2 (L + 1) x m synthesis outputs
    double2* A = nullptr;       // (2L + 1) x J coefficients (Helmholtz temporaries)
    double2* Bc = nullptr;      // (2L + 1) x J
    double* phi = nullptr;      // 2 (L + 1): phase offsets of orders 0 .. L (direct method)
    int method = NUHT_FB_TRANSFORM;
    nuht_batch_t fwd = nullptr; // orders 0 .. L: r -> zeros_l (transform method)
    nuht_batch_t inv = nullptr; // orders 0 .. L: zeros_l -> r
};

namespace {

void fb_free(nuht_fb_s* fb)
{
    if (!fb) return;
    if (fb->fwd) nuht_batch_destroy(fb->fwd);
    if (fb->inv) nuht_batch_destroy(fb->inv);
    for (void* p : {(void*)fb->r, (void*)fb->wr, (void*)fb->zeros, (void*)fb->nrm, (void*)fb->C, (void*)fb->G,
                    (void*)fb->U, (void*)fb->A, (void*)fb->Bc, (void*)fb->phi})
        if (p) (void)hipFree(p);
    delete fb;
}

template <class T>
bool fb_alloc(T*& p, int64_t count)
{
    if (hipMalloc((void**)&p, sizeof(T) * (size_t)(count > 0 ? count : 1)) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return false;
    }
    return true;
}

// Two executions of a batch (q = 0, 1: real and imaginary parts): input rows
// in[(2 l + q) nin], output rows out[(2 l + q) nout].
int fb_run(nuht_batch_t b, int L, const double* in, int64_t nin, double* out, int64_t nout, hipStream_t s)
{
    std::vector<const double*> cp(L + 1);
    std::vector<double*> gp(L + 1);
    for (int q = 0; q < 2; ++q) {
        for (int l = 0; l <= L; ++l) {
            cp[l] = in + (2 * (int64_t)l + q) * nin;
            gp[l] = out + (2 * (int64_t)l + q) * nout;
        }
        int rc = nuht_execute_many(b, cp.data(), gp.data(), s);
        if (rc != NUHT_OK) return rc;
    }
    return NUHT_OK;
}

int fb_analysis(nuht_fb_s* fb, const double* f, double2* alpha, hipStream_t s)
{
    hipLaunchKernelGGL(k_fb_angular_fwd, dim3((unsigned)fb->m), dim3(256), sizeof(double2) * fb->t, s, f, fb->m,
                       fb->logt, fb->L, fb->r, fb->wr, fb->C);
    if (hipGetLastError() != hipSuccess) return NUHT_EHIP;
    if (fb->method == NUHT_FB_DIRECT) {
        hipLaunchKernelGGL(k_fb_direct_fwd, dim3((unsigned)((fb->J + 63) / 64), (unsigned)(fb->L + 1)),
                           dim3(64 * kFbWaves), 0, s, fb->C, fb->r, fb->m, fb->zeros, fb->J, fb->phi, fb->G);
        if (hipGetLastError() != hipSuccess) return NUHT_EHIP;
    } else {
        int rc = fb_run(fb->fwd, fb->L, fb->C, fb->m, fb->G, fb->J, s);
        if (rc != NUHT_OK) return rc;
    }
    const int64_t total = (int64_t)(2 * fb->L + 1) * fb->J;
    hipLaunchKernelGGL(k_fb_scale, dim3(blocks_for(total)), dim3(256), 0, s, fb->G, fb->nrm, fb->L, fb->J, alpha);
    return hipGetLastError() == hipSuccess ? NUHT_OK : NUHT_EHIP;
}

int fb_synthesis(nuht_fb_s* fb, const double2* beta, double* u, hipStream_t s)
{
    const int64_t total = (int64_t)(fb->L + 1) * fb->J;
    hipLaunchKernelGGL(k_fb_split, dim3(blocks_for(total)), dim3(256), 0, s, beta, fb->L, fb->J, fb->G);
    if (hipGetLastError() != hipSuccess) return NUHT_EHIP;
    if (fb->method == NUHT_FB_DIRECT) {
        hipLaunchKernelGGL(k_fb_direct_inv, dim3((unsigned)((fb->m + 63) / 64), (unsigned)(fb->L + 1)),
                           dim3(64 * kFbWaves), 0, s, fb->G, fb->r, fb->m, fb->zeros, fb->J, fb->phi, fb->U);
        if (hipGetLastError() != hipSuccess) return NUHT_EHIP;
    } else {
        int rc = fb_run(fb->inv, fb->L, fb->G, fb->J, fb->U, fb->m, s);
        if (rc != NUHT_OK) return rc;
    }
    hipLaunchKernelGGL(k_fb_angular_inv, dim3((unsigned)fb->m), dim3(256), sizeof(double2) * fb->t, s, fb->U,
                       fb->m, fb->logt, fb->L, u);
    return hipGetLastError() == hipSuccess ? NUHT_OK : NUHT_EHIP;
}

}  // namespace

extern "C" {

int nuht_fb_plan(nuht_fb_t* out, int32_t L, int64_t m, const double* r_dev, const double* wr_dev, int64_t t,
                 int64_t J, const double* zeros_dev, double eps, int32_t method, void* stream)
{
    if (!out) return NUHT_EINVAL;
    *out = nullptr;
    if (L < 0 || L > 100 || m < 1 || m > INT32_MAX || J < 1 || J > INT32_MAX) return NUHT_EINVAL;
    if (t < 2 || t > 4096 || (t & (t - 1)) != 0 || 2 * (int64_t)L + 1 > t) return NUHT_EINVAL;
    if (!r_dev || !wr_dev || !zeros_dev) return NUHT_EINVAL;
    if (!(eps >= 1e-15 && eps <= 1e-2)) return NUHT_EINVAL;
    if (method != NUHT_FB_TRANSFORM && method != NUHT_FB_DIRECT) return NUHT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    nuht_fb_s* fb = new (std::nothrow) nuht_fb_s;
    if (!fb) return NUHT_ENOMEM;
    fb->L = L; fb->m = m; fb->t = t; fb->J = J; fb->method = method;
    while ((int64_t(1) << fb->logt) < t) ++fb->logt;
    const int64_t nl = L + 1, no = 2 * (int64_t)L + 1;
    if (!fb_alloc(fb->r, m) || !fb_alloc(fb->wr, m) || !fb_alloc(fb->zeros, nl * J) || !fb_alloc(fb->nrm, nl * J) ||
        !fb_alloc(fb->C, 2 * nl * m) || !fb_alloc(fb->G, 2 * nl * J) || !fb_alloc(fb->U, 2 * nl * m) ||
        !fb_alloc(fb->A, no * J) || !fb_alloc(fb->Bc, no * J) || !fb_alloc(fb->phi, 2 * nl)) {
        fb_free(fb);
        return NUHT_ENOMEM;
    }
    if (hipMemcpyAsync(fb->r, r_dev, sizeof(double) * m, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(fb->wr, wr_dev, sizeof(double) * m, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(fb->zeros, zeros_dev, sizeof(double) * nl * J, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        (void)hipGetLastError();
        fb_free(fb);
        return NUHT_EHIP;
    }
    std::vector<int> nu(nl);
    std::vector<int64_t> nn(nl), nm(nl);
    std::vector<const double*> pr(nl), pz(nl);
    std::vector<double> ph(2 * nl);
    for (int l = 0; l <= L; ++l) {
        nu[l] = l;
        nn[l] = m;
        nm[l] = J;
        pr[l] = fb->r;
        pz[l] = fb->zeros + (int64_t)l * J;
        phase_offset_dd(l, &ph[2 * l], &ph[2 * l + 1]);
    }
    int rc = NUHT_OK;
    if (hipMemcpyAsync(fb->phi, ph.data(), sizeof(double) * 2 * nl, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        rc = NUHT_EHIP;
    if (rc == NUHT_OK && method == NUHT_FB_TRANSFORM)
        rc = nuht_plan_many(&fb->fwd, (int)nl, nu.data(), eps, nn.data(), pr.data(), nm.data(), pz.data(), nullptr,
                            stream);
    if (rc == NUHT_OK && method == NUHT_FB_TRANSFORM)
        rc = nuht_plan_many(&fb->inv, (int)nl, nu.data(), eps, nm.data(), pz.data(), nn.data(), pr.data(), nullptr,
                            stream);
    // normalisation: J_{|l|-1} (J_1 for l = 0) at the zeros, by the direct sum
    // over one point r = 1 with weight 1 (the two constants are kept in the U
    // buffer, unused until the first synthesis)
    if (rc == NUHT_OK) {
        const double one[2] = {1.0, 1.0};
        if (hipMemcpyAsync(fb->U, one, sizeof one, hipMemcpyHostToDevice, s) != hipSuccess) rc = NUHT_EHIP;
        if (rc == NUHT_OK && hipStreamSynchronize(s) != hipSuccess) rc = NUHT_EHIP;
        for (int l = 0; l <= L && rc == NUHT_OK; ++l)
            rc = nuht_direct(l == 0 ? 1 : l - 1, eps, 1, fb->U, fb->U + 1, J, fb->zeros + (int64_t)l * J,
                             fb->nrm + (int64_t)l * J, stream);
        if (rc == NUHT_OK) {
            hipLaunchKernelGGL(k_fb_norm, dim3(blocks_for(nl * J)), dim3(256), 0, s, fb->nrm, nl * J);
            if (hipGetLastError() != hipSuccess) rc = NUHT_EHIP;
        }
        if (rc == NUHT_OK && hipStreamSynchronize(s) != hipSuccess) rc = NUHT_EHIP;
    }
    if (rc != NUHT_OK) {
        (void)hipGetLastError();
        fb_free(fb);
        return rc;
    }
    *out = fb;
    return NUHT_OK;
}

int nuht_fb_analysis(nuht_fb_t fb, const double* f_dev, double* alpha_dev, void* stream)
{
    if (!fb || !f_dev || !alpha_dev) return NUHT_EINVAL;
    return fb_analysis(fb, f_dev, reinterpret_cast<double2*>(alpha_dev), (hipStream_t)stream);
}

int nuht_fb_synthesis(nuht_fb_t fb, const double* beta_dev, double* u_dev, void* stream)
{
    if (!fb || !beta_dev || !u_dev) return NUHT_EINVAL;
    return fb_synthesis(fb, reinterpret_cast<const double2*>(beta_dev), u_dev, (hipStream_t)stream);
}

int nuht_fb_helmholtz(nuht_fb_t fb, double kappa, const double* f_dev, double* alpha_dev, double* beta_dev,
                      double* u_dev, void* stream)
{
    if (!fb || !f_dev || !u_dev || !std::isfinite(kappa)) return NUHT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double2* alpha = alpha_dev ? reinterpret_cast<double2*>(alpha_dev) : fb->A;
    double2* beta = beta_dev ? reinterpret_cast<double2*>(beta_dev) : fb->Bc;
    int rc = fb_analysis(fb, f_dev, alpha, s);
    if (rc != NUHT_OK) return rc;
    const int64_t total = (int64_t)(2 * fb->L + 1) * fb->J;
    hipLaunchKernelGGL(k_fb_helmholtz, dim3(blocks_for(total)), dim3(256), 0, s, alpha, fb->zeros, fb->L, fb->J,
                       kappa, beta);
    if (hipGetLastError() != hipSuccess) return NUHT_EHIP;
    return fb_synthesis(fb, beta, u_dev, s);
}

int nuht_fb_destroy(nuht_fb_t fb)
{
    if (fb) (void)hipDeviceSynchronize();
    fb_free(fb);
    return NUHT_OK;
}

}  // extern "C"
