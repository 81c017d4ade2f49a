// Spectral bounds (Lin, Saad & Yang, section 3.1.1, the paragraph after
// eq. (cd)): a k-step Lanczos run in FP64 on the device with two passes of
// full re-orthogonalisation per step.  It leaves alpha[0..m-1] and
// beta[0..m-1] (beta[j] = norm of the residual after step j) in device
// memory; the host part of kpm_bounds solves the m x m tridiagonal
// eigenproblem and widens the extreme Ritz values by their residuals.
//
// Work split: workgroup b owns the contiguous row chunk [b*C, (b+1)*C).
// Each Lanczos step j is four launches, enqueued without any host sync:
//   A spmv    q_j = r_{j-1} / beta_{j-1} (beta reduced from the previous
//             norm partials; q_0 = start probe / sqrt(n)), row j of Q
//             stored, w = A q_j into the other residual buffer, partial
//             sums of q_j . w
//   B axpy    w -= alpha_j q_j + beta_{j-1} q_{j-1}; partials of Q^T w
//   C reorth  w -= Q h (h reduced from B's partials); partials of Q^T w
//   D reorth  w -= Q h (from C's partials); partials of w . w
// Every consumer reduces the per-workgroup partials itself with one fixed
// summation tree, so all workgroups see bit-identical coefficients and
// results are deterministic run to run.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kpm_internal.h"

namespace kpm {

constexpr int LZ_THREADS = 256;
constexpr int LZ_SLOTS = 32;  // partial slots per workgroup (max Lanczos steps)

__device__ __forceinline__ uint64_t lz_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Entry i of the start vector: probe vector 2^31-1 of `seed`, divided by sqrt(n).
__device__ __forceinline__ double lz_start_entry(uint64_t seed, int64_t i, double inv_sqrt_n) {
    const uint64_t k = ((((uint64_t)0x7fffffffu) << 32) | (uint64_t)i) + 1ull;
    return ((lz_mix(seed + k * 0x9e3779b97f4a7c15ull) >> 63) ? -1.0 : 1.0) * inv_sqrt_n;
}

// coef layout: alpha[0..63], beta[64..127]
#define ALPHA(j) coef[(j)]
#define BETA(j) coef[64 + (j)]

struct LzArgs {
    const int32_t* rp;
    const int32_t* ci;
    const void* val;
    double* Q;       // [m][n]
    double* W[2];    // residual buffers
    double* coef;
    double* part;    // [4 kinds][nblk][LZ_SLOTS]
    uint64_t seed;
    int32_t n, nblk, chunk;
};

__device__ __forceinline__ double* part_of(const LzArgs& a, int kind, int b) {
    return a.part + ((int64_t)kind * a.nblk + b) * LZ_SLOTS;
}

// Sum of slot t over all workgroups of `kind`, by one wavefront: lane l adds
// workgroups l, l+64, ... in order, then a fixed butterfly combines the
// lanes.  Every workgroup that calls this gets the same bits.
__device__ __forceinline__ double lz_wave_sum_partials(const LzArgs& a, int kind, int t) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int b = lane; b < a.nblk; b += 64) s += part_of(a, kind, b)[t];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// Reduce slots [0, J) of `kind` into hs[]: wavefront w handles t = w, w+4, ...
__device__ __forceinline__ void lz_reduce_into(const LzArgs& a, int kind, int J, double* hs) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = wave; t < J; t += LZ_THREADS / 64) {
        const double v = lz_wave_sum_partials(a, kind, t);
        if (lane == 0) hs[t] = v;
    }
    __syncthreads();
}

// Workgroup sum of one value per thread: butterfly per wavefront, then the
// four wavefront sums in order.  Every thread returns the total.
__device__ __forceinline__ double lz_block_sum(double v, double* sh4) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh4[wave] = v;
    __syncthreads();
    return ((sh4[0] + sh4[1]) + sh4[2]) + sh4[3];
}

template <typename TA>
__global__ __launch_bounds__(LZ_THREADS) void lz_spmv(LzArgs a, int j) {
    __shared__ double sh4[4];
    __shared__ double s_inv;
    const int b = blockIdx.x;
    const double* __restrict__ wr = a.W[(j + 1) & 1];
    double* __restrict__ ww = a.W[j & 1];
    const TA* __restrict__ val = static_cast<const TA*>(a.val);
    const double inv_sqrt_n = 1.0 / sqrt((double)a.n);
    if (threadIdx.x < 64) {
        double inv = 0.0;
        if (j > 0) {
            const double nrm2 = lz_wave_sum_partials(a, 3, 0);
            const double beta = sqrt(nrm2 > 0.0 ? nrm2 : 0.0);
            inv = beta > 0.0 ? 1.0 / beta : 0.0;
            if (b == 0 && threadIdx.x == 0) a.coef[64 + j - 1] = beta;
        }
        if (threadIdx.x == 0) s_inv = inv;
    }
    __syncthreads();
    const double inv = s_inv;
    double* __restrict__ qj = a.Q + (int64_t)j * a.n;
    const int64_t i0 = (int64_t)b * a.chunk;
    const int64_t i1 = min((int64_t)a.n, i0 + a.chunk);
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += LZ_THREADS) {
        double s = 0.0;
        for (int32_t k = a.rp[i]; k < a.rp[i + 1]; ++k) {
            const int32_t c = a.ci[k];
            const double q = j == 0 ? lz_start_entry(a.seed, c, inv_sqrt_n) : wr[c] * inv;
            s = fma((double)val[k], q, s);
        }
        const double qi = j == 0 ? lz_start_entry(a.seed, i, inv_sqrt_n) : wr[i] * inv;
        qj[i] = qi;
        ww[i] = s;
        acc = fma(qi, s, acc);
    }
    const double tot = lz_block_sum(acc, sh4);
    if (threadIdx.x == 0) part_of(a, 0, b)[0] = tot;
}

// MODE 0: w -= alpha_j q_j + beta_{j-1} q_{j-1}, partials of Q^T w -> kind 1
// MODE 1: w -= Q h (h from kind 1),              partials of Q^T w -> kind 2
// MODE 2: w -= Q h (h from kind 2),              partial of w . w  -> kind 3
template <int MODE>
__global__ __launch_bounds__(LZ_THREADS) void lz_orth(LzArgs a, int j) {
    extern __shared__ double xs[];  // the workgroup's chunk of w
    __shared__ double hs[LZ_SLOTS];
    __shared__ double sh4[4];
    const int b = blockIdx.x;
    const int J = j + 1;
    double* __restrict__ ww = a.W[j & 1];
    const double* __restrict__ coef = a.coef;
    lz_reduce_into(a, MODE, MODE == 0 ? 1 : J, hs);
    if (MODE == 0 && b == 0 && threadIdx.x == 0) a.coef[j] = hs[0];
    const int64_t i0 = (int64_t)b * a.chunk;
    const int64_t i1 = min((int64_t)a.n, i0 + a.chunk);
    const double* __restrict__ Q = a.Q;
    const int64_t n = a.n;
    double nrm = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += LZ_THREADS) {
        double x = ww[i];
        if (MODE == 0) {
            x = x - hs[0] * Q[(int64_t)j * n + i];
            if (j > 0) x = x - BETA(j - 1) * Q[(int64_t)(j - 1) * n + i];
        } else {
            double s = 0.0;
            for (int t = 0; t < J; ++t) s = fma(hs[t], Q[(int64_t)t * n + i], s);
            x = x - s;
        }
        ww[i] = x;
        if (MODE == 2) nrm = fma(x, x, nrm);
        else xs[i - i0] = x;
    }
    if (MODE == 2) {
        const double tot = lz_block_sum(nrm, sh4);
        if (threadIdx.x == 0) part_of(a, 3, b)[0] = tot;
        return;
    }
    __syncthreads();
    for (int t = 0; t < J; ++t) {
        const double* __restrict__ qt = Q + (int64_t)t * n;
        double acc = 0.0;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += LZ_THREADS) acc = fma(qt[i], xs[i - i0], acc);
        const double tot = lz_block_sum(acc, sh4);
        if (threadIdx.x == 0) part_of(a, MODE + 1, b)[t] = tot;
    }
}

// beta_{m-1} from the last norm partials.
__global__ void lz_last_beta(LzArgs a, int m) {
    const double nrm2 = lz_wave_sum_partials(a, 3, 0);
    if (threadIdx.x == 0) a.coef[64 + m - 1] = sqrt(nrm2 > 0.0 ? nrm2 : 0.0);
}

hipError_t launch_lanczos(hipStream_t s, const CsrDev& A, int m, uint64_t seed, LanczosWork& W) {
    LzArgs a;
    a.rp = A.rp;
    a.ci = A.ci;
    a.val = A.val;
    a.Q = W.Q;
    a.W[0] = W.w;
    a.W[1] = W.w + A.n;
    a.coef = W.coef;
    a.part = W.partial;
    a.seed = seed;
    a.n = A.n;
    a.nblk = W.nblk;
    a.chunk = W.chunk;
    const size_t lds = (size_t)W.chunk * sizeof(double);
    for (int j = 0; j < m; ++j) {
        if (A.val_f64) lz_spmv<double><<<a.nblk, LZ_THREADS, 0, s>>>(a, j);
        else lz_spmv<float><<<a.nblk, LZ_THREADS, 0, s>>>(a, j);
        lz_orth<0><<<a.nblk, LZ_THREADS, lds, s>>>(a, j);
        lz_orth<1><<<a.nblk, LZ_THREADS, lds, s>>>(a, j);
        lz_orth<2><<<a.nblk, LZ_THREADS, 0, s>>>(a, j);
    }
    lz_last_beta<<<1, 64, 0, s>>>(a, m);
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
