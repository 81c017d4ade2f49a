// Damping factors and density evaluation (Lin, Saad & Yang, eq. (tdosFinal),
// eq. (expmu) and Appendix A eq. (jackson)).  All FP64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kpm_internal.h"

namespace kpm {

// g_k = [(1 - k/(M+2)) sin(a) cos(k a) + (1/(M+2)) cos(a) sin(k a)] / sin(a),
// a = pi/(M+2).
__global__ void jackson_kernel(int M, double* __restrict__ g) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > M) return;
    const double a = M_PI / (double)(M + 2);
    const double sa = sin(a), ca = cos(a);
    g[k] = ((1.0 - (double)k / (double)(M + 2)) * sa * cos(k * a) +
            (1.0 / (double)(M + 2)) * ca * sin(k * a)) / sa;
}

hipError_t launch_jackson(hipStream_t s, int M, double* g) {
    jackson_kernel<<<(M + 1 + 127) / 128, 128, 0, s>>>(M, g);
    return hipGetLastError();
}

// phi(x) = [g_0 mu_0 + 2 sum_{k>=1} g_k mu_k T_k(t)] / (pi d sqrt(1 - t^2)),
// t = (x - c)/d, the Chebyshev sum evaluated by Clenshaw's recurrence.  The
// coefficients g_k mu_k are first staged in LDS when they fit.
constexpr int kDosLds = 4096;

__device__ __forceinline__ void dos_stage(const double* __restrict__ mu, const double* __restrict__ g, int M,
                                          double* cf) {
    if (M + 1 <= kDosLds)
        for (int k = threadIdx.x; k <= M; k += blockDim.x) cf[k] = g[k] * mu[k];
    __syncthreads();
}

__device__ __forceinline__ double dos_point(const double* __restrict__ mu, const double* __restrict__ g, int M,
                                            const double* cf, double c, double d, double x) {
    const bool lds = M + 1 <= kDosLds;
    const double t = (x - c) / d;
    if (!(fabs(t) < 1.0)) return 0.0;
    double b1 = 0.0, b2 = 0.0;
    for (int k = M; k >= 1; --k) {
        const double ck = lds ? cf[k] : g[k] * mu[k];
        const double b0 = 2.0 * ck + 2.0 * t * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    const double sum = g[0] * mu[0] + t * b1 - b2;
    return sum / (M_PI * d * sqrt(1.0 - t * t));
}

__global__ __launch_bounds__(128) void dos_kernel(const double* __restrict__ mu, const double* __restrict__ g,
                                                  int M, double c, double d, const double* __restrict__ x,
                                                  int npts, double* __restrict__ phi) {
    __shared__ double cf[kDosLds];
    dos_stage(mu, g, M, cf);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    phi[i] = dos_point(mu, g, M, cf, c, d, x[i]);
}

hipError_t launch_dos(hipStream_t s, const double* mu, const double* g, int M, double c, double d,
                      const double* x, int npts, double* phi) {
    dos_kernel<<<(npts + 127) / 128, 128, 0, s>>>(mu, g, M, c, d, x, npts, phi);
    return hipGetLastError();
}

// Many matrices: workgroup (i, m) evaluates points 128 i ... of matrix m,
// whose series is row m of mu (and of g when g_stride > 0) and whose points
// are row m of x; c and d from lb[m], ub[m] as on the host.
__global__ __launch_bounds__(128) void dos_batched_kernel(const double* __restrict__ mu,
                                                          const double* __restrict__ g, int64_t g_stride, int M,
                                                          const double* __restrict__ lb,
                                                          const double* __restrict__ ub,
                                                          const double* __restrict__ x, int npts,
                                                          double* __restrict__ phi) {
    __shared__ double cf[kDosLds];
    const int m = blockIdx.y;
    mu += (int64_t)m * (M + 1);
    g += g_stride * m;
    dos_stage(mu, g, M, cf);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const double c = 0.5 * (lb[m] + ub[m]), d = 0.5 * (ub[m] - lb[m]);
    phi[(int64_t)m * npts + i] = dos_point(mu, g, M, cf, c, d, x[(int64_t)m * npts + i]);
}

hipError_t launch_dos_batched(hipStream_t s, int nmat, const double* mu, const double* g, int64_t g_stride, int M,
                              const double* lb, const double* ub, const double* x, int npts, double* phi) {
    dim3 grid((npts + 127) / 128, nmat);
    dos_batched_kernel<<<grid, 128, 0, s>>>(mu, g, g_stride, M, lb, ub, x, npts, phi);
    return hipGetLastError();
}

// Antiderivative of the density in t, written in theta = arccos t:
// F(t) = -(1/pi) [g_0 mu_0 theta + 2 sum_k g_k mu_k sin(k theta)/k];
// mass[i] = F(t_{i+1}) - F(t_i) with t clamped to [-1, 1].
__device__ double dos_antiderivative(const double* mu, const double* g, int M, double t) {
    t = fmin(1.0, fmax(-1.0, t));
    const double th = acos(t);
    double s = g[0] * mu[0] * th;
    for (int k = 1; k <= M; ++k) s += 2.0 * g[k] * mu[k] * sin(k * th) / (double)k;
    return -s / M_PI;
}

__global__ void dos_bins_kernel(const double* __restrict__ mu, const double* __restrict__ g, int M,
                                double c, double d, const double* __restrict__ edges, int nbins,
                                double* __restrict__ mass) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nbins) return;
    const double fa = dos_antiderivative(mu, g, M, (edges[i] - c) / d);
    const double fb = dos_antiderivative(mu, g, M, (edges[i + 1] - c) / d);
    mass[i] = fb - fa;
}

hipError_t launch_dos_bins(hipStream_t s, const double* mu, const double* g, int M, double c,
                           double d, const double* edges, int nbins, double* mass) {
    dos_bins_kernel<<<(nbins + 127) / 128, 128, 0, s>>>(mu, g, M, c, d, edges, nbins, mass);
    return hipGetLastError();
}

}  // namespace kpm
