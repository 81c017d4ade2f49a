// Legendre expansions (Lin, Saad & Yang): KPM with Legendre polynomials
// (the variant named in Appendix A) and the Delta-Gauss-Legendre method
// (section 3.1.3, Algorithm DGL; coefficients from Appendix B).
//
// Both need the Legendre moments mu_k = tr L_k(B)/n.  The paper's Algorithm
// DGL runs the Legendre three-term recurrence, one sparse product per
// moment.  Here the moments come from the Chebyshev moments of the fused
// step instead: every Legendre polynomial is a combination of Chebyshev
// polynomials with non-negative weights,
//   L_n = sum_{k <= n/2} (2 - [n = 2k]) a_k a_{n-k} T_{n-2k},
//   a_m = (2m)! / (4^m (m!)^2) = prod_{j <= m} (2j - 1) / (2j),
// whose sum is L_n(1) = 1.  So v^T L_n(B) v is an average of v^T T_j(B) v:
// the product identity of Appendix A then gives M Legendre moments from
// ceil(M/2) sparse products, and the conversion cannot amplify the
// moments' rounding errors (a convex combination).  The paper's recurrence
// in the fused step is available too (KPM_FLAG_LEGENDRE_RECURRENCE).
//
// DGL: for each point t, gamma_k(t) = int_{-1}^{1} L_k(s) exp(-((s-t)/sigma)^2/2) ds
// by the recurrence of eq. (Leg3) from gamma_0 of eq. (gam0), stopped by
// eq. (StopRecur); the density is eq. (dglexpansion) with the stochastic
// moments.  KPM-Legendre: sum_k (k + 1/2) g_k mu_k L_k(t).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "kpm_internal.h"
#include "kpm_step.h"

namespace kpm {
namespace {

// zetaL[l][n] = sum_{k <= n/2} w a_k a_{n-k} zeta[l][n-2k], one workgroup per
// probe row, terms added from k = 0 (highest Chebyshev degree) up.
__global__ __launch_bounds__(256) void cheb_to_legendre_kernel(const double* __restrict__ zeta, int M,
                                                               const double* __restrict__ a,
                                                               double* __restrict__ out) {
    const int64_t row = (int64_t)blockIdx.x * (M + 1);
    for (int n = threadIdx.x; n <= M; n += 256) {
        double s = 0.0;
        for (int k = 0; 2 * k <= n; ++k) {
            const double w = (2 * k == n ? 1.0 : 2.0) * a[k] * a[n - k];
            s = fma(w, zeta[row + n - 2 * k], s);
        }
        out[row + n] = s;
    }
}

// One thread per point.  deg[i] = degree used; bad[i] = 1 if the
// recurrence diverged (|gamma_k| > gamma_0, impossible in exact arithmetic).
__global__ __launch_bounds__(256) void dgl_dos_kernel(const double* __restrict__ mu, int M, double c, double d,
                                                      double sig, double tol, const double* __restrict__ x,
                                                      int npts, double* __restrict__ phi, int* __restrict__ deg,
                                                      int* __restrict__ bad) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= npts) return;
    const double t = (x[i] - c) / d;
    const double r2s = sqrt(2.0) * sig;
    const double ea = (1.0 - t) / r2s, eb = (1.0 + t) / r2s;
    // erf(ea) + erf(eb), as a difference of erfc when one argument is
    // negative (centre outside [-1, 1]: the sum would cancel)
    const double S = ea < 0.0 ? erfc(-ea) - erfc(eb) : (eb < 0.0 ? erfc(-eb) - erfc(ea) : erf(ea) + erf(eb));
    const double g0 = sig * sqrt(M_PI / 2.0) * S;
    double acc = 0.5 * g0 * mu[0];
    int m = M, diverged = 0;
    if (M > 0) {
        const double e_hi = exp(-0.5 * ((1.0 - t) / sig) * ((1.0 - t) / sig));
        const double e_lo = exp(-0.5 * ((1.0 + t) / sig) * ((1.0 + t) / sig));
        const double s2 = sig * sig;
        double gkm1 = 0.0, gk = g0, pkm1 = 0.0, pk = 0.0;
        for (int k = 0; k < M; ++k) {
            const double zk = (k & 1) ? e_hi + e_lo : e_hi - e_lo;
            const double gn = (double)(2 * k + 1) / (double)(k + 1) * (s2 * (pk - zk) + t * gk) -
                              (double)k / (double)(k + 1) * gkm1;
            const double pn = (double)(2 * k + 1) * gk + pkm1;
            if (!(fabs(gn) <= g0)) {
                diverged = 1;
                m = k + 1;
                break;
            }
            acc = fma((double)k + 1.5, gn * mu[k + 1], acc);
            if (fabs(gk) + fabs(gn) <= (double)(k + 1) * tol) {
                m = k + 1;
                break;
            }
            gkm1 = gk;
            gk = gn;
            pkm1 = pk;
            pk = pn;
        }
    } else {
        m = 0;
    }
    phi[i] = acc / sqrt(2.0 * M_PI * sig * sig) / d;
    deg[i] = m;
    bad[i] = diverged;
}

// One thread per point: forward Legendre recurrence (stable on [-1, 1]).
__global__ __launch_bounds__(256) void legendre_dos_kernel(const double* __restrict__ mu,
                                                           const double* __restrict__ g, int M, double c, double d,
                                                           const double* __restrict__ x, int npts,
                                                           double* __restrict__ phi) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= npts) return;
    const double t = (x[i] - c) / d;
    if (!(fabs(t) <= 1.0)) {
        phi[i] = 0.0;
        return;
    }
    double lkm1 = 1.0, lk = t;  // L_0, L_1
    double acc = 0.5 * (g ? g[0] : 1.0) * mu[0];
    for (int k = 1; k <= M; ++k) {
        acc = fma((double)k + 0.5, (g ? g[k] : 1.0) * mu[k] * lk, acc);
        const double ln = ((double)(2 * k + 1) * t * lk - (double)k * lkm1) / (double)(k + 1);
        lkm1 = lk;
        lk = ln;
    }
    phi[i] = acc / d;
}

// One thread per (row, word): bit j of word w is set when entry `row` of
// probe vec0 + 32 w + j is -1, from the probes' generator itself (the same
// signs the block fill writes), so the block is not read back.
__global__ __launch_bounds__(256) void sign_bits_kernel(uint64_t seed, int64_t vec0, int ncols, int64_t n, int sw,
                                                        uint32_t* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * sw) return;
    const int64_t row = t / sw;
    const int w = (int)(t - row * sw);
    const int c0 = w * 32, c1 = std::min(ncols, c0 + 32);
    uint32_t bits = 0;
    for (int cidx = c0; cidx < c1; ++cidx)
        if (rademacher_sign(seed, (uint64_t)(vec0 + cidx), (uint64_t)row) < 0.0f) bits |= 1u << (cidx - c0);
    out[t] = bits;
}

__global__ __launch_bounds__(256) void legendre_assemble_kernel(const double* __restrict__ dots, int ld, int ncols,
                                                                int M, double n, int64_t vec0,
                                                                double* __restrict__ zeta) {
    const int j = blockIdx.y;
    for (int k = blockIdx.x * 256 + threadIdx.x; k <= M; k += gridDim.x * 256)
        zeta[(vec0 + j) * (M + 1) + k] = k == 0 ? 1.0 : dots[(int64_t)(k - 1) * 2 * ld + j] / n;
}

}  // namespace

hipError_t launch_sign_bits(hipStream_t s, uint64_t seed, int64_t vec0, int ncols, int64_t n, int sw,
                            uint32_t* out) {
    const int64_t tot = n * sw;
    if (tot == 0) return hipSuccess;
    sign_bits_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(seed, vec0, ncols, n, sw, out);
    return hipGetLastError();
}

hipError_t launch_legendre_assemble(hipStream_t s, const double* dots, int ld, int ncols, int M, double n,
                                    int64_t vec0, double* zeta) {
    const dim3 grid((unsigned)std::min((M + 256) / 256, 64), (unsigned)ncols);
    legendre_assemble_kernel<<<grid, 256, 0, s>>>(dots, ld, ncols, M, n, vec0, zeta);
    return hipGetLastError();
}

// a_m = prod_{j <= m} (2j - 1)/(2j), m = 0..M (host).
void legendre_connection_weights(int M, double* a) {
    a[0] = 1.0;
    for (int m = 1; m <= M; ++m) a[m] = a[m - 1] * (double)(2 * m - 1) / (double)(2 * m);
}

hipError_t launch_cheb_to_legendre(hipStream_t s, const double* zeta, int nvec, int M, const double* a,
                                   double* out) {
    cheb_to_legendre_kernel<<<nvec, 256, 0, s>>>(zeta, M, a, out);
    return hipGetLastError();
}

}  // namespace kpm

using namespace kpm;

static kpm_status upload(kpm_ctx* ctx, const char* role, const void* src, size_t bytes, void** dst) {
    kpm_status st = kpm_ws(ctx, role, bytes, dst);
    if (st != KPM_OK) return st;
    KPM_HIP(ctx, hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
    return KPM_OK;
}

extern "C" kpm_status kpm_dgl_dos(kpm_ctx* ctx, const double* mu, int M, double lb, double ub, double sigma,
                                  double tol, const double* x, int npts, double* phi, int* degree_used) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!mu || !x || !phi || M < 0 || M > (1 << 20) || npts < 0) return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (!(std::isfinite(lb) && std::isfinite(ub) && ub > lb)) return kpm_fail(ctx, KPM_ERR_ARG, "need finite lb < ub");
    if (!(sigma > 0.0) || !std::isfinite(sigma) || !(tol >= 0.0) || !std::isfinite(tol))
        return kpm_fail(ctx, KPM_ERR_ARG, "sigma must be positive and tol non-negative");
    if (npts == 0) return KPM_OK;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    const double c = 0.5 * (lb + ub), d = 0.5 * (ub - lb);
    void *mud, *xd, *pd, *dd, *bd;
    kpm_status st;
    if ((st = upload(ctx, "leg_mu", mu, (size_t)(M + 1) * 8, &mud)) != KPM_OK) return st;
    if ((st = upload(ctx, "dos_x", x, (size_t)npts * 8, &xd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dos_phi", (size_t)npts * 8, &pd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dgl_deg", (size_t)npts * 8, &dd)) != KPM_OK) return st;
    bd = (char*)dd + (size_t)npts * 4;
    dgl_dos_kernel<<<(npts + 255) / 256, 256, 0, ctx->stream>>>((const double*)mud, M, c, d, sigma / d, tol,
                                                               (const double*)xd, npts, (double*)pd, (int*)dd,
                                                               (int*)bd);
    KPM_HIP(ctx, hipGetLastError());
    std::vector<int> hd((size_t)npts * 2);
    KPM_HIP(ctx, hipMemcpyAsync(phi, pd, (size_t)npts * 8, hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(hd.data(), dd, (size_t)npts * 8, hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < npts; ++i)
        if (hd[(size_t)npts + i]) {
            char msg[200];
            snprintf(msg, sizeof msg,
                     "gamma recurrence diverged at point %d (degree %d) before the stopping rule held: "
                     "tol %g is too small for sigma %g",
                     i, hd[i], tol, sigma);
            return kpm_fail(ctx, KPM_ERR_NOCONV, msg);
        }
    if (degree_used) std::copy(hd.begin(), hd.begin() + npts, degree_used);
    return KPM_OK;
}

extern "C" kpm_status kpm_legendre_dos(kpm_ctx* ctx, const double* mu, const double* g, int M, double lb,
                                       double ub, const double* x, int npts, double* phi) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!mu || !x || !phi || M < 0 || M > (1 << 20) || npts < 0) return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (!(std::isfinite(lb) && std::isfinite(ub) && ub > lb)) return kpm_fail(ctx, KPM_ERR_ARG, "need finite lb < ub");
    if (npts == 0) return KPM_OK;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    const double c = 0.5 * (lb + ub), d = 0.5 * (ub - lb);
    void *mud, *gd = nullptr, *xd, *pd;
    kpm_status st;
    if ((st = upload(ctx, "leg_mu", mu, (size_t)(M + 1) * 8, &mud)) != KPM_OK) return st;
    if (g && (st = upload(ctx, "leg_g", g, (size_t)(M + 1) * 8, &gd)) != KPM_OK) return st;
    if ((st = upload(ctx, "dos_x", x, (size_t)npts * 8, &xd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dos_phi", (size_t)npts * 8, &pd)) != KPM_OK) return st;
    legendre_dos_kernel<<<(npts + 255) / 256, 256, 0, ctx->stream>>>((const double*)mud, (const double*)gd, M, c, d,
                                                                    (const double*)xd, npts, (double*)pd);
    KPM_HIP(ctx, hipGetLastError());
    KPM_HIP(ctx, hipMemcpyAsync(phi, pd, (size_t)npts * 8, hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return KPM_OK;
}
