// Haydock's method (Lin, Saad & Yang, section 3.2.2): the density
// regularised by Lorentzians of half-width eta,
//   phi_eta(x) = (1/nvec) sum_l -(1/pi) Im e_1^T ((x + i eta) I - T_l)^{-1} e_1,
// from the tridiagonal Lanczos matrices T_l of the probes (the coefficients
// kpm_slq returns) without their eigenvalues.  The (1,1) entry of the
// resolvent is the continued fraction of eq. (cfHaydock), evaluated from
// the bottom:
//   w_{m-1} = z - alpha_{m-1},   w_k = z - alpha_k - beta_k^2 / w_{k+1},
//   e_1^T (z - T)^{-1} e_1 = 1 / w_0.
// With eta > 0 every w_k has imaginary part >= eta (beta_k^2 / w adds
// beta_k^2 Im(w) / |w|^2 >= 0), so no step divides by zero.  The run is in
// B's units (z_B = (x - c + i eta) / d, T of B) and the density in A's units
// is the B density over d.  The minus sign of -Im makes the density
// non-negative; the paper's second form writes +Im.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "kpm_internal.h"

namespace kpm {
namespace {

constexpr int kHayPoints = 64;  // points per workgroup (one wavefront)
constexpr int kHayChunk = 512;  // coefficients staged in LDS at a time

// One workgroup per (64 points, probe l): the probe's coefficients are
// staged in LDS from the bottom of the fraction up, a chunk at a time, and
// every lane runs the recursion for its point.  Writes
// partial[l * npts + i] = Im(w_0) / |w_0|^2 = -Im(1 / w_0).
__global__ __launch_bounds__(kHayPoints) void haydock_partial_kernel(
    const double* __restrict__ alpha, const double* __restrict__ beta, const int* __restrict__ used, int M,
    double c, double d, double eta, const double* __restrict__ x, int npts, double* __restrict__ partial) {
    __shared__ double sa[kHayChunk], sb2[kHayChunk];
    const int l = blockIdx.y;
    const int i = blockIdx.x * kHayPoints + threadIdx.x;
    const double* __restrict__ a = alpha + (int64_t)l * M;
    const double* __restrict__ b = beta + (int64_t)l * M;
    const int m = used[l];
    const double zr = i < npts ? (x[i] - c) / d : 0.0;
    const double zi = eta / d;
    double wr = 0.0, wi = 0.0;
    bool started = false;
    for (int top = ((m - 1) / kHayChunk) * kHayChunk; top >= 0; top -= kHayChunk) {
        const int end = std::min(m, top + kHayChunk);
        __syncthreads();
        for (int k = top + threadIdx.x; k < end; k += kHayPoints) {
            sa[k - top] = a[k];
            sb2[k - top] = b[k] * b[k];
        }
        __syncthreads();
        for (int k = end - 1; k >= top; --k) {
            if (!started) {  // k = m - 1: the last diagonal entry
                wr = zr - sa[k - top];
                wi = zi;
                started = true;
            } else {
                const double s = sb2[k - top] / fma(wr, wr, wi * wi);  // beta_k^2 / |w_{k+1}|^2
                wr = zr - sa[k - top] - wr * s;
                wi = fma(wi, s, zi);
            }
        }
    }
    if (i < npts) partial[(int64_t)l * npts + i] = wi / fma(wr, wr, wi * wi);
}

// phi[i] = sum over probes in order / (pi d nvec).
__global__ __launch_bounds__(256) void haydock_sum_kernel(const double* __restrict__ partial, int nvec, int npts,
                                                          double scale, double* __restrict__ phi) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= npts) return;
    double s = 0.0;
    for (int l = 0; l < nvec; ++l) s += partial[(int64_t)l * npts + i];
    phi[i] = s * scale;
}

}  // namespace
}  // namespace kpm

using namespace kpm;

extern "C" kpm_status kpm_haydock_dos(kpm_ctx* ctx, const double* alpha, const double* beta,
                                      const int* steps_used, int nvec, int M, double lb, double ub, double eta,
                                      const double* x, int npts, double* phi) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!alpha || !beta || !steps_used || !x || !phi || nvec < 1 || nvec > 65535 || M < 1 || npts < 0)
        return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (!(eta > 0.0) || !std::isfinite(eta) || !std::isfinite(lb) || !std::isfinite(ub) || !(lb < ub))
        return kpm_fail(ctx, KPM_ERR_ARG, "eta must be positive and lb < ub finite");
    for (int l = 0; l < nvec; ++l) {
        const int m = steps_used[l];
        if (m < 1 || m > M) return kpm_fail(ctx, KPM_ERR_ARG, "steps_used out of [1, M]");
        for (int k = 0; k < m; ++k)
            if (!std::isfinite(alpha[(size_t)l * M + k]) || (k + 1 < m && !std::isfinite(beta[(size_t)l * M + k])))
                return kpm_fail(ctx, KPM_ERR_ARG, "non-finite Lanczos coefficient");
    }
    if (npts == 0) return KPM_OK;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    const double c = 0.5 * (lb + ub), d = 0.5 * (ub - lb);
    const size_t nn = (size_t)nvec * M;
    void *ad, *bd, *ud, *xd, *qd, *pd;
    kpm_status st;
    if ((st = kpm_ws(ctx, "hay_alpha", nn * 8, &ad)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "hay_beta", nn * 8, &bd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "hay_used", (size_t)nvec * 4, &ud)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dos_x", (size_t)npts * 8, &xd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "hay_partial", (size_t)nvec * npts * 8, &qd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dos_phi", (size_t)npts * 8, &pd)) != KPM_OK) return st;
    KPM_HIP(ctx, hipMemcpyAsync(ad, alpha, nn * 8, hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(bd, beta, nn * 8, hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(ud, steps_used, (size_t)nvec * 4, hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(xd, x, (size_t)npts * 8, hipMemcpyHostToDevice, ctx->stream));
    const dim3 grid((npts + kHayPoints - 1) / kHayPoints, nvec);
    haydock_partial_kernel<<<grid, kHayPoints, 0, ctx->stream>>>((const double*)ad, (const double*)bd,
                                                                  (const int*)ud, M, c, d, eta,
                                                                  (const double*)xd, npts, (double*)qd);
    KPM_HIP(ctx, hipGetLastError());
    haydock_sum_kernel<<<(npts + 255) / 256, 256, 0, ctx->stream>>>((const double*)qd, nvec, npts,
                                                                    1.0 / (M_PI * d * nvec), (double*)pd);
    KPM_HIP(ctx, hipGetLastError());
    KPM_HIP(ctx, hipMemcpyAsync(phi, pd, (size_t)npts * 8, hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return KPM_OK;
}
