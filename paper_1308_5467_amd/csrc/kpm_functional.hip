// Functionals of the approximate densities (Lin, Saad & Yang, section 2,
// eq. (errormetric_g)): <phi~, f> = int f(lambda) phi~(lambda) dlambda, and
// the heat capacity of section 4.3, C_v(T) = <phi~, g_T> with g_T of eq.
// (gfunc) in units where k_B = 1 and hbar c / k_B = 1:
//   g_T(lambda) = x^2 e^{-x} / (1 - e^{-x})^2 = (x / (2 sinh(x/2)))^2,
//   x = sqrt(lambda) / T (g_T = 1 at lambda <= 0: frequencies are >= 0).
//
// KPM density: in theta = arccos t the integral becomes
//   (1/pi) int_0^pi f(c + d cos theta) D(theta) dtheta,
//   D(theta) = sum_k (2 - [k = 0]) g_k mu_k cos(k theta),
// taken by Gauss-Chebyshev quadrature on Q nodes theta_q = (q + 1/2) pi / Q:
//   <phi~, f> ~ (1/Q) sum_q f(c + d cos theta_q) D(theta_q),
// exact when f is a polynomial of degree < 2Q - M and converging
// geometrically in Q for f analytic on [lb, ub].  D is evaluated at the
// nodes once; each functional is then one pass over the Q nodes.
//
// Lanczos density (section 4.3 replaces the Gaussian of eq. (landos) by
// g_T): (1/nvec) sum_l sum_k tau_k^2 g_T(theta_k).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "kpm_internal.h"

namespace kpm {
namespace {

__device__ __forceinline__ double heat_g(double lam, double T) {
    const double x = sqrt(fmax(lam, 0.0)) / T;
    if (x == 0.0) return 1.0;
    const double h = 0.5 * x;
    const double r = h / sinh(h);  // 0 once sinh overflows
    return r * r;
}

// D_q, one thread per node, by the Chebyshev recurrence in t_q = cos theta_q.
__global__ __launch_bounds__(256) void series_at_nodes_kernel(const double* __restrict__ mu,
                                                              const double* __restrict__ g, int M, int Q,
                                                              double* __restrict__ D) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= Q) return;
    const double t = cos((q + 0.5) * M_PI / Q);
    double tkm1 = 1.0, tk = t;
    double s = (g ? g[0] : 1.0) * mu[0];
    for (int k = 1; k <= M; ++k) {
        s = fma(2.0 * (g ? g[k] : 1.0) * mu[k], tk, s);
        const double tn = 2.0 * t * tk - tkm1;
        tkm1 = tk;
        tk = tn;
    }
    D[q] = s;
}

// Fixed-order block sum of 256 per-thread values (deterministic).
__device__ __forceinline__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    return sh[0];
}

// One workgroup per temperature: C_v(T_j) = (1/Q) sum_q g_T(x_q) D_q.
__global__ __launch_bounds__(256) void kpm_heat_capacity_kernel(const double* __restrict__ D, int Q, double c,
                                                                double d, const double* __restrict__ T,
                                                                double* __restrict__ out) {
    __shared__ double sh[256];
    const double Tj = T[blockIdx.x];
    double s = 0.0;
    for (int q = threadIdx.x; q < Q; q += 256) s = fma(heat_g(c + d * cos((q + 0.5) * M_PI / Q), Tj), D[q], s);
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = tot / Q;
}

// One workgroup: <phi~, f> = (1/Q) sum_q f_q D_q.
__global__ __launch_bounds__(256) void kpm_functional_kernel(const double* __restrict__ D,
                                                             const double* __restrict__ f, int Q,
                                                             double* __restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int q = threadIdx.x; q < Q; q += 256) s = fma(f[q], D[q], s);
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = tot / Q;
}

// One workgroup per temperature over all nodes of all probes.
__global__ __launch_bounds__(256) void slq_heat_capacity_kernel(const double* __restrict__ theta,
                                                                const double* __restrict__ tau2, int64_t nn,
                                                                int nvec, const double* __restrict__ T,
                                                                double* __restrict__ out) {
    __shared__ double sh[256];
    const double Tj = T[blockIdx.x];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < nn; k += 256) {
        const double w = tau2[k];
        if (w != 0.0) s = fma(w, heat_g(theta[k], Tj), s);
    }
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = tot / nvec;
}

}  // namespace
}  // namespace kpm

using namespace kpm;

static kpm_status upload_f(kpm_ctx* ctx, const char* role, const void* src, size_t bytes, void** dst) {
    kpm_status st = kpm_ws(ctx, role, bytes, dst);
    if (st != KPM_OK) return st;
    KPM_HIP(ctx, hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
    return KPM_OK;
}

// Uploads mu and g and evaluates D at the Q nodes.
static kpm_status series_nodes(kpm_ctx* ctx, const double* mu, const double* g, int M, int Q, double** D) {
    void *mud, *gd = nullptr, *dd;
    kpm_status st;
    if ((st = upload_f(ctx, "fn_mu", mu, (size_t)(M + 1) * 8, &mud)) != KPM_OK) return st;
    if (g && (st = upload_f(ctx, "fn_g", g, (size_t)(M + 1) * 8, &gd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "fn_D", (size_t)Q * 8, &dd)) != KPM_OK) return st;
    series_at_nodes_kernel<<<(Q + 255) / 256, 256, 0, ctx->stream>>>((const double*)mud, (const double*)gd, M, Q,
                                                                    (double*)dd);
    KPM_HIP(ctx, hipGetLastError());
    *D = (double*)dd;
    return KPM_OK;
}

static bool check_range(double lb, double ub) { return std::isfinite(lb) && std::isfinite(ub) && ub > lb; }

extern "C" kpm_status kpm_functional_nodes(int Q, double lb, double ub, double* x) {
    if (!x || Q < 1 || Q > (1 << 26) || !check_range(lb, ub)) return KPM_ERR_ARG;
    const double c = 0.5 * (lb + ub), d = 0.5 * (ub - lb);
    for (int q = 0; q < Q; ++q) x[q] = c + d * cos((q + 0.5) * M_PI / Q);
    return KPM_OK;
}

extern "C" kpm_status kpm_functional(kpm_ctx* ctx, const double* mu, const double* g, int M, double lb, double ub,
                                     const double* fvals, int Q, double* out) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!mu || !fvals || !out || M < 0 || M > (1 << 20) || Q < 1 || Q > (1 << 26))
        return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (!check_range(lb, ub)) return kpm_fail(ctx, KPM_ERR_ARG, "need finite lb < ub");
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    double* D;
    void *fd, *od;
    kpm_status st;
    if ((st = series_nodes(ctx, mu, g, M, Q, &D)) != KPM_OK) return st;
    if ((st = upload_f(ctx, "fn_f", fvals, (size_t)Q * 8, &fd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "fn_out", 8, &od)) != KPM_OK) return st;
    kpm_functional_kernel<<<1, 256, 0, ctx->stream>>>(D, (const double*)fd, Q, (double*)od);
    KPM_HIP(ctx, hipGetLastError());
    KPM_HIP(ctx, hipMemcpyAsync(out, od, 8, hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return KPM_OK;
}

extern "C" kpm_status kpm_heat_capacity(kpm_ctx* ctx, const double* mu, const double* g, int M, double lb,
                                        double ub, const double* T, int nT, int Q, double* cv) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!mu || !T || !cv || M < 0 || M > (1 << 20) || nT < 0 || Q < 0 || Q > (1 << 26))
        return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (!check_range(lb, ub)) return kpm_fail(ctx, KPM_ERR_ARG, "need finite lb < ub");
    for (int j = 0; j < nT; ++j)
        if (!(T[j] > 0.0) || !std::isfinite(T[j])) return kpm_fail(ctx, KPM_ERR_ARG, "temperatures must be > 0");
    if (nT == 0) return KPM_OK;
    if (Q == 0) Q = std::max(1024, 4 * (M + 1));
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    double* D;
    void *td, *od;
    kpm_status st;
    if ((st = series_nodes(ctx, mu, g, M, Q, &D)) != KPM_OK) return st;
    if ((st = upload_f(ctx, "fn_T", T, (size_t)nT * 8, &td)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "fn_cv", (size_t)nT * 8, &od)) != KPM_OK) return st;
    const double c = 0.5 * (lb + ub), d = 0.5 * (ub - lb);
    kpm_heat_capacity_kernel<<<nT, 256, 0, ctx->stream>>>(D, Q, c, d, (const double*)td, (double*)od);
    KPM_HIP(ctx, hipGetLastError());
    KPM_HIP(ctx, hipMemcpyAsync(cv, od, (size_t)nT * 8, hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return KPM_OK;
}

extern "C" kpm_status kpm_slq_heat_capacity(kpm_ctx* ctx, const double* theta, const double* tau2, int nvec,
                                            int M, const double* T, int nT, double* cv) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!theta || !tau2 || !T || !cv || nvec < 1 || M < 1 || nT < 0) return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    for (int j = 0; j < nT; ++j)
        if (!(T[j] > 0.0) || !std::isfinite(T[j])) return kpm_fail(ctx, KPM_ERR_ARG, "temperatures must be > 0");
    if (nT == 0) return KPM_OK;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    const size_t nn = (size_t)nvec * M;
    void *thd, *wd, *td, *od;
    kpm_status st;
    if ((st = upload_f(ctx, "slq_theta", theta, nn * 8, &thd)) != KPM_OK) return st;
    if ((st = upload_f(ctx, "slq_tau2", tau2, nn * 8, &wd)) != KPM_OK) return st;
    if ((st = upload_f(ctx, "fn_T", T, (size_t)nT * 8, &td)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "fn_cv", (size_t)nT * 8, &od)) != KPM_OK) return st;
    slq_heat_capacity_kernel<<<nT, 256, 0, ctx->stream>>>((const double*)thd, (const double*)wd, (int64_t)nn, nvec,
                                                          (const double*)td, (double*)od);
    KPM_HIP(ctx, hipGetLastError());
    KPM_HIP(ctx, hipMemcpyAsync(cv, od, (size_t)nT * 8, hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return KPM_OK;
}
