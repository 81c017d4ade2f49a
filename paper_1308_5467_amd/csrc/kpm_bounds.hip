// Spectral bounds (Lin, Saad & Yang, section 3.1.1, the paragraph after
// eq. (cd)): a k-step Lanczos run in FP64 on the device, two passes of full
// re-orthogonalisation per step, leaving alpha[0..m-1] and beta[0..m-1]
// (beta[j] = norm of the residual after step j) in device memory.  The
// m x m tridiagonal eigenproblem and the residual widening are done by the
// host part of kpm_bounds.
//
// Each Lanczos step j is eight launches, all enqueued without a host sync:
//   1 spmv_alpha   q_j = w / beta_{j-1} (j > 0, also stored as row j of Q),
//                  w = A q_j, partial sums of q_j . w
//   2 reduce       alpha_j
//   3 axpy_dots    w -= alpha_j q_j + beta_{j-1} q_{j-1}; partial Q^T w
//   4 reduce       h
//   5 update_dots  w -= Q h; partial Q^T w            (second pass)
//   6 reduce       h
//   7 update_norm  w -= Q h; partial w . w
//   8 reduce       beta_j = sqrt(w . w)
// Reductions: per-thread sums in row order, fixed-shape wavefront butterflies,
// then a fixed-order compensated sum over workgroups: results are
// deterministic run to run.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kpm_internal.h"

namespace kpm {

constexpr int LZ_MAXJ = 32;   // max Lanczos steps (dot slots per step)
constexpr int LZ_THREADS = 256;

__device__ __forceinline__ uint64_t lz_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// coef layout: alpha[0..63], beta[64..127], h[128..191] (only the first 32 of each are used)
#define ALPHA(j) coef[(j)]
#define BETA(j) coef[64 + (j)]
#define HCOEF(t) coef[128 + (t)]

__device__ __forceinline__ double wave_sum(double v) {
    // Butterfly over the 64 lanes; every lane ends with the same value.
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Reduce J per-thread values across the workgroup and write partial[blk][t].
template <int JMAX>
__device__ __forceinline__ void block_partials(const double (&v)[JMAX], int J, double* partial) {
    __shared__ double sh[LZ_THREADS / 64][LZ_MAXJ];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = 0; t < J; ++t) {
        const double s = wave_sum(v[t]);
        if (lane == 0) sh[wave][t] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < J) {
        double s = 0.0;
        for (int w = 0; w < LZ_THREADS / 64; ++w) s += sh[w][threadIdx.x];
        partial[(int64_t)blockIdx.x * LZ_MAXJ + threadIdx.x] = s;
    }
}

// 1: optional normalisation of the previous residual, then w = A q_j and
// the partial sums of q_j . w.
template <typename TA>
__global__ __launch_bounds__(LZ_THREADS) void lz_spmv_alpha(const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const TA* __restrict__ val, int32_t n,
                                                            double* __restrict__ Q, int j,
                                                            double* __restrict__ w,
                                                            double* __restrict__ wn,
                                                            const double* __restrict__ coef,
                                                            double* __restrict__ partial) {
    double* __restrict__ qj = Q + (int64_t)j * n;
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s = fma((double)val[k], qj[ci[k]], s);
        wn[i] = s;
        acc[0] = fma(qj[i], s, acc[0]);
    }
    block_partials<1>(acc, 1, partial);
}

// q_j = w / beta_{j-1} (zero after a breakdown), stored as row j of Q.
__global__ void lz_normalize(double* __restrict__ Q, int j, const double* __restrict__ w, int32_t n,
                             const double* __restrict__ coef) {
    const double b = BETA(j - 1);
    const double inv = b > 0.0 ? 1.0 / b : 0.0;
    double* qj = Q + (int64_t)j * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        qj[i] = w[i] * inv;
}

// q_0 = probe vector 2^31-1 of `seed` / sqrt(n)
__global__ void lz_start(double* __restrict__ Q, int32_t n, uint64_t seed) {
    const double inv = 1.0 / sqrt((double)n);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = ((((uint64_t)0x7fffffffu) << 32) | (uint64_t)i) + 1ull;
        const double sgn = (lz_mix(seed + k * 0x9e3779b97f4a7c15ull) >> 63) ? -1.0 : 1.0;
        Q[i] = sgn * inv;
    }
}

// mode 0: w -= alpha_j q_j + beta_{j-1} q_{j-1}  then partial Q^T w (J = j+1)
// mode 1: w -= sum_t h_t q_t                       then partial Q^T w
// mode 2: w -= sum_t h_t q_t                       then partial w . w
template <int MODE>
__global__ __launch_bounds__(LZ_THREADS) void lz_update(const double* __restrict__ Q, int j, int32_t n,
                                                        double* __restrict__ w,
                                                        const double* __restrict__ coef,
                                                        double* __restrict__ partial) {
    const int J = j + 1;
    double acc[LZ_MAXJ];
#pragma unroll
    for (int t = 0; t < LZ_MAXJ; ++t) acc[t] = 0.0;
    __shared__ double hs[LZ_MAXJ];
    if ((int)threadIdx.x < J) hs[threadIdx.x] = MODE == 0 ? 0.0 : HCOEF(threadIdx.x);
    __syncthreads();
    const double a = ALPHA(j);
    const double bprev = j > 0 ? BETA(j - 1) : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double x = w[i];
        if (MODE == 0) {
            x = x - a * Q[(int64_t)j * n + i];
            if (j > 0) x = x - bprev * Q[(int64_t)(j - 1) * n + i];
        } else {
            double s = 0.0;
            for (int t = 0; t < J; ++t) s = fma(hs[t], Q[(int64_t)t * n + i], s);
            x = x - s;
        }
        w[i] = x;
        if (MODE == 2) {
            acc[0] = fma(x, x, acc[0]);
        } else {
#pragma unroll
            for (int t = 0; t < LZ_MAXJ; ++t)
                if (t < J) acc[t] = fma(Q[(int64_t)t * n + i], x, acc[t]);
        }
    }
    block_partials<LZ_MAXJ>(acc, MODE == 2 ? 1 : J, partial);
}

// out slot: 0 -> alpha_j, 1 -> h[0..J), 2 -> beta_j = sqrt(sum)
__global__ __launch_bounds__(256) void lz_reduce(const double* __restrict__ partial, int nblk, int J,
                                                 int j, int slot, double* __restrict__ coef) {
    const int t = blockIdx.x;
    if (t >= J) return;
    __shared__ double shs[256], shc[256];
    double s = 0.0, c = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
        const double x = partial[(int64_t)b * LZ_MAXJ + t];
        const double u = s + x;
        c += (fabs(s) >= fabs(x)) ? (s - u) + x : (x - u) + s;
        s = u;
    }
    shs[threadIdx.x] = s;
    shc[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        double S = 0.0, C = 0.0;
        for (int i = 0; i < 256; ++i) {
            const double x = shs[i];
            const double u = S + x;
            C += (fabs(S) >= fabs(x)) ? (S - u) + x : (x - u) + S;
            S = u;
            C += shc[i];
        }
        const double r = S + C;
        if (slot == 0) ALPHA(j) = r;
        else if (slot == 1) HCOEF(t) = r;
        else BETA(j) = sqrt(r > 0.0 ? r : 0.0);
    }
}

hipError_t launch_lanczos(hipStream_t s, const CsrDev& A, int m, uint64_t seed, LanczosWork& W) {
    const int32_t n = A.n;
    const int nblk = W.nblk;
    lz_start<<<nblk, LZ_THREADS, 0, s>>>(W.Q, n, seed);
    for (int j = 0; j < m; ++j) {
        if (j > 0) lz_normalize<<<nblk, LZ_THREADS, 0, s>>>(W.Q, j, W.w, n, W.coef);
        if (A.val_f64)
            lz_spmv_alpha<double><<<nblk, LZ_THREADS, 0, s>>>(A.rp, A.ci, (const double*)A.val, n, W.Q,
                                                              j, W.w, W.w, W.coef, W.partial);
        else
            lz_spmv_alpha<float><<<nblk, LZ_THREADS, 0, s>>>(A.rp, A.ci, (const float*)A.val, n, W.Q, j,
                                                             W.w, W.w, W.coef, W.partial);
        lz_reduce<<<1, 256, 0, s>>>(W.partial, nblk, 1, j, 0, W.coef);
        lz_update<0><<<nblk, LZ_THREADS, 0, s>>>(W.Q, j, n, W.w, W.coef, W.partial);
        lz_reduce<<<j + 1, 256, 0, s>>>(W.partial, nblk, j + 1, j, 1, W.coef);
        lz_update<1><<<nblk, LZ_THREADS, 0, s>>>(W.Q, j, n, W.w, W.coef, W.partial);
        lz_reduce<<<j + 1, 256, 0, s>>>(W.partial, nblk, j + 1, j, 1, W.coef);
        lz_update<2><<<nblk, LZ_THREADS, 0, s>>>(W.Q, j, n, W.w, W.coef, W.partial);
        lz_reduce<<<1, 256, 0, s>>>(W.partial, nblk, 1, j, 2, W.coef);
    }
    return hipGetLastError();
}

// Gershgorin hull: out[2b] = min over the block's rows of a_ii - sum|a_ij|,
// out[2b+1] = max of a_ii + sum|a_ij|.
template <typename TA>
__global__ __launch_bounds__(256) void gershgorin_kernel(const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const TA* __restrict__ val, int32_t n,
                                                         double* __restrict__ out) {
    double lo = 1e308, hi = -1e308;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double diag = 0.0, off = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const double v = (double)val[k];
            if (ci[k] == i) diag += v;
            else off += fabs(v);
        }
        lo = fmin(lo, diag - off);
        hi = fmax(hi, diag + off);
    }
    __shared__ double slo[256], shi[256];
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + st]);
            shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = slo[0];
        out[2 * blockIdx.x + 1] = shi[0];
    }
}

hipError_t launch_gershgorin(hipStream_t s, const CsrDev& A, double* out, int nblk) {
    if (A.val_f64)
        gershgorin_kernel<double><<<nblk, 256, 0, s>>>(A.rp, A.ci, (const double*)A.val, A.n, out);
    else
        gershgorin_kernel<float><<<nblk, 256, 0, s>>>(A.rp, A.ci, (const float*)A.val, A.n, out);
    return hipGetLastError();
}

}  // namespace kpm
