// Spectral bounds (Lin, Saad & Yang, section 3.1.1, the paragraph after
// eq. (cd)): a k-step Lanczos run in FP64 on the device with full
// re-orthogonalisation (one classical Gram-Schmidt pass against every
// previous Lanczos vector).  It leaves
// alpha[0..m-1] and beta[0..m-1] (beta[j] = norm of the residual after step
// j) in device memory; the host part of kpm_bounds solves the m x m
// tridiagonal eigenproblem and widens the extreme Ritz values by their
// residuals.
//
// Step j is two data-parallel launches, each followed by a small reduction
// launch, all enqueued without any host sync:
//   A  q_j = r_{j-1} / beta_{j-1} (q_0 = start probe / sqrt(n)), stored as
//      row j of Q;  w = A q_j;  partials of h = Q^T w    (alpha_j = h_j)
//   B  w -= Q h;  partial of ||w||^2                      (-> beta_j)
// (h_{j-1} plays the part of beta_{j-1} in the three-term recurrence and
// the other h_t remove the components along older vectors.)
// Every workgroup owns a contiguous chunk of rows (R rows per thread, held
// in registers) and writes one partial per coefficient; the reduction
// launch adds them in a fixed order (one workgroup per coefficient), so
// results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kpm_internal.h"

namespace kpm {

constexpr int LZ_THREADS = 256;
constexpr int LZ_SLOTS = 32;  // max Lanczos steps

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

// coef layout (doubles): alpha[0..63], beta[64..127], h[128..159]
struct LzArgs {
    const int32_t* rp;
    const int32_t* ci;
    const void* val;
    double* Q;       // [m][n]
    double* W[2];    // residual buffers
    double* coef;
    double* part;    // [3 kinds][LZ_SLOTS][nblk]
    uint64_t seed;
    int32_t n, nblk, chunk;
};

__device__ __forceinline__ double* part_slot(const LzArgs& a, int kind, int t) {
    return a.part + ((int64_t)kind * LZ_SLOTS + t) * a.nblk;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Store this workgroup's J partial sums (wavefront sums in sh[wave][t]).
__device__ __forceinline__ void lz_store_partials(const LzArgs& a, int kind, int J, double (*sh)[LZ_SLOTS]) {
    __syncthreads();
    if ((int)threadIdx.x < J) {
        const int t = threadIdx.x;
        part_slot(a, kind, t)[blockIdx.x] = ((sh[0][t] + sh[1][t]) + sh[2][t]) + sh[3][t];
    }
}

// out[t] = sum over workgroups of partial slot t of `kind` (square root when
// MODE == 2; MODE == 0 also copies slot j to alpha_j).  Kinds: 0 projection
// partials of launch A, 2 norm partials of launch B.  Workgroup t: each
// thread adds workgroups tid, tid+256, ... in order, then a fixed tree.
template <int MODE>
__global__ __launch_bounds__(LZ_THREADS) void lz_reduce(LzArgs a, int kind, int j, double* out) {
    __shared__ double sh[LZ_THREADS / 64];
    const int t = blockIdx.x;
    const double* p = part_slot(a, kind, t);
    double s = 0.0;
    for (int b = threadIdx.x; b < a.nblk; b += LZ_THREADS) s += p[b];
    s = wave_sum(s);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
        if (MODE == 2) {
            out[t] = sqrt(r > 0.0 ? r : 0.0);
        } else {
            out[t] = r;
            if (MODE == 0 && t == j) a.coef[j] = r;  // alpha_j = q_j^T A q_j
        }
    }
}

// A: normalise, w = A q_j, first projection h = Q^T w.
template <typename TA, int R>
__global__ __launch_bounds__(LZ_THREADS) void lz_spmv_project(LzArgs a, int j) {
    __shared__ double sh[LZ_THREADS / 64][LZ_SLOTS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double* __restrict__ wr = a.W[(j + 1) & 1];
    double* __restrict__ ww = a.W[j & 1];
    const TA* __restrict__ val = static_cast<const TA*>(a.val);
    const double inv_sqrt_n = 1.0 / sqrt((double)a.n);
    double inv = 0.0;
    if (j > 0) {
        const double beta = a.coef[64 + j - 1];
        inv = beta > 0.0 ? 1.0 / beta : 0.0;
    }
    const int64_t n = a.n;
    double* __restrict__ qj = a.Q + (int64_t)j * n;
    const int64_t i0 = (int64_t)blockIdx.x * a.chunk + threadIdx.x;
    double x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = i0 + (int64_t)r * LZ_THREADS;
        x[r] = 0.0;
        if (i < n) {
            // Row entries in batches of 8: indices and values first, then 8
            // independent gathers (slots past the row's end repeat the
            // batch's first entry with value 0), then the sums in order.
            double s = 0.0;
            const int32_t kb = a.rp[i], ke = a.rp[i + 1];
            for (int32_t k = kb; k < ke; k += 8) {
                int32_t c[8];
                double v[8], q[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool on = k + u < ke;
                    const int32_t ks = on ? k + u : k;
                    c[u] = a.ci[ks];
                    // value 0 past the end, as a bit mask so that the load
                    // stays unconditional
                    const double vv = (double)val[ks];
                    v[u] = __longlong_as_double(__double_as_longlong(vv) & (on ? ~0ll : 0ll));
                }
                if (j == 0) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) q[u] = lz_start_entry(a.seed, c[u], inv_sqrt_n);
                } else {
#pragma unroll
                    for (int u = 0; u < 8; ++u) q[u] = wr[c[u]] * inv;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) s = fma(v[u], q[u], s);
            }
            qj[i] = j == 0 ? lz_start_entry(a.seed, i, inv_sqrt_n) : wr[i] * inv;
            ww[i] = s;
            x[r] = s;
        }
    }
    // h_t = q_t . w for t <= j (this thread wrote its rows of q_j above).
    // Vectors go in groups of TG (up to 16 loads per thread in flight) whose
    // loads are all issued before any sum, so a step costs ceil((j+1)/TG)
    // memory round trips instead of j+1; slots past j are skipped by a
    // wavefront-uniform test (groups of 8 cost about 5 us each on a 64^3
    // stencil).
    constexpr int TG = R >= 16 ? 1 : 16 / R;
    for (int t0 = 0; t0 <= j; t0 += TG) {
        double q[TG][R];
#pragma unroll
        for (int u = 0; u < TG; ++u) {
            if (t0 + u > j) break;
            const double* __restrict__ qt = a.Q + (int64_t)(t0 + u) * n;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t i = i0 + (int64_t)r * LZ_THREADS;
                q[u][r] = i < n ? qt[i] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < TG; ++u) {
            if (t0 + u > j) break;
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) acc = fma(q[u][r], x[r], acc);
            acc = wave_sum(acc);
            if (lane == 0) sh[wave][t0 + u] = acc;
        }
    }
    lz_store_partials(a, 0, j + 1, sh);
}

// B: w -= Q h (h from A's reduction); partial of ||w||^2 (-> beta_j).
template <int R>
__global__ __launch_bounds__(LZ_THREADS) void lz_orth(LzArgs a, int j) {
    __shared__ double sh[LZ_THREADS / 64][LZ_SLOTS];
    __shared__ double hs[LZ_SLOTS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int J = j + 1;
    double* __restrict__ ww = a.W[j & 1];
    if ((int)threadIdx.x < J) hs[threadIdx.x] = a.coef[128 + threadIdx.x];
    __syncthreads();
    const int64_t n = a.n;
    const double* __restrict__ Q = a.Q;
    const int64_t i0 = (int64_t)blockIdx.x * a.chunk + threadIdx.x;
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = i0 + (int64_t)r * LZ_THREADS;
        if (i < n) {
            double s = 0.0;
            for (int t = 0; t < J; ++t) s = fma(hs[t], Q[(int64_t)t * n + i], s);
            const double x = ww[i] - s;
            ww[i] = x;
            acc = fma(x, x, acc);
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) sh[wave][0] = acc;
    lz_store_partials(a, 2, 1, sh);
}

template <int R>
static void lz_launch_steps(hipStream_t s, const CsrDev& A, int m, const LzArgs& a) {
    for (int j = 0; j < m; ++j) {
        if (A.val_f64) lz_spmv_project<double, R><<<a.nblk, LZ_THREADS, 0, s>>>(a, j);
        else lz_spmv_project<float, R><<<a.nblk, LZ_THREADS, 0, s>>>(a, j);
        lz_reduce<0><<<j + 1, LZ_THREADS, 0, s>>>(a, 0, j, a.coef + 128);
        lz_orth<R><<<a.nblk, LZ_THREADS, 0, s>>>(a, j);
        lz_reduce<2><<<1, LZ_THREADS, 0, s>>>(a, 2, j, a.coef + 64 + j);
    }
}

// Rows per thread: the smallest power of two (<= 16) that keeps the grid
// at or under 512 workgroups.  Measured for 20 steps: 0.48 ms on a 64^3
// stencil (0.52 ms with a 1024-workgroup cap, 0.54 ms with 256) and 5.24 ms
// on 128^3 with long-range pairs (5.48 ms with 1024, 5.80 ms with 2048).
int lanczos_rows_per_thread(int64_t n) {
    int R = 1;
    while (R < 16 && (int64_t)LZ_THREADS * R * 512 < n) R *= 2;
    return R;
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
    switch (W.chunk / LZ_THREADS) {
        case 1: lz_launch_steps<1>(s, A, m, a); break;
        case 2: lz_launch_steps<2>(s, A, m, a); break;
        case 4: lz_launch_steps<4>(s, A, m, a); break;
        case 8: lz_launch_steps<8>(s, A, m, a); break;
        case 16: lz_launch_steps<16>(s, A, m, a); break;
        default: return hipErrorInvalidValue;
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
