// Device kernels of the KPM moment path (Lin, Saad & Yang, section 3.1.1,
// Algorithm 1, with the product identity of Appendix A):
//
//   rademacher_fill   probe block V0 [n x ld], entries +/-1 (SplitMix64 signs)
//   cheb_step<FIRST>  V1 = B V0 (FIRST) or U <- 2 B V - U (in place), fused
//                     with the two per-column dot products the product
//                     identity needs: <U_new, V> and <U_new, U_new>
//   reduce_partials   fixed-order, compensated sum of the per-panel partials
//   assemble          zeta_k per probe vector from the dots
//   mean_moments      mu_k = mean over probe vectors, compensated
//
// Data layout.  A vector block is row-major [n x ld]: the ld values of one
// matrix row are contiguous, so a gathered row of V is one 16-byte load per
// lane (float4 for FP32, double2 for FP64) and ld/VPL lanes cover a row.
// A 64-wide wavefront therefore works on rpw = 64 / lpr rows at once and a
// 256-thread workgroup on 4 * rpw rows per pass over its row panel.
//
// The scaled operator is applied as 2B = alpha A + beta I with
// alpha = 2/d and beta = -2c/d (eq. (cd)), so the matrix values are used as
// given and no shifted copy of A is made.  In the FP32 path the sparse
// product sum is FP32 and the recurrence combination
// alpha*acc + beta*v - u is evaluated in FP64 and rounded once; the dot
// products are exact FP32 x FP32 products accumulated in FP64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kpm_internal.h"

namespace kpm {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Entry i of probe vector l of `seed`: sign of output ((l<<32)|i)+1 of SplitMix64.
__device__ __forceinline__ float rademacher_sign(uint64_t seed, uint64_t l, uint64_t i) {
    const uint64_t k = ((l << 32) | i) + 1ull;
    return (sm64_mix(seed + k * 0x9e3779b97f4a7c15ull) >> 63) ? -1.0f : 1.0f;
}

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X.  Map
// workgroup b to a row panel so that each XCD owns one contiguous run of
// panels: neighbouring rows (and most gathered rows of a banded matrix) then
// share that XCD's L2.  Bijective for every count.
__device__ __forceinline__ int xcd_panel(int b, int nb) {
    const int X = 8;
    const int q = nb / X, r = nb - q * X;
    const int x = b % X, li = b / X;
    return x * q + min(x, r) + li;
}

template <typename T>
struct Pack;
template <>
struct Pack<float> {
    static constexpr int N = 4;
    __device__ static __forceinline__ void load(const float* p, float (&v)[4]) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    }
    __device__ static __forceinline__ void store(float* p, const float (&v)[4]) {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    }
};
template <>
struct Pack<double> {
    static constexpr int N = 2;
    __device__ static __forceinline__ void load(const double* p, double (&v)[2]) {
        const double2 t = *reinterpret_cast<const double2*>(p);
        v[0] = t.x; v[1] = t.y;
    }
    __device__ static __forceinline__ void store(double* p, const double (&v)[2]) {
        *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    }
};

BlockGeom make_geom(int64_t n, int ncols, int precision, int rows_per_block_hint) {
    BlockGeom g;
    const int vpl = precision == KPM_FP64 ? 2 : 4;
    g.ld = (ncols + vpl - 1) / vpl * vpl;
    g.lpr = g.ld / vpl;
    g.rpw = 64 / g.lpr;
    const int rows_per_pass = kWaves * g.rpw;
    int rows;
    if (rows_per_block_hint > 0) {
        rows = (rows_per_block_hint + rows_per_pass - 1) / rows_per_pass * rows_per_pass;
    } else {
        // Aim for about 2048 workgroups (8 per CU) and at most 64 passes each.
        int64_t passes = (n + (int64_t)rows_per_pass * 2048 - 1) / ((int64_t)rows_per_pass * 2048);
        if (passes < 1) passes = 1;
        if (passes > 64) passes = 64;
        rows = (int)passes * rows_per_pass;
    }
    g.rows_per_block = rows;
    g.nblocks = (int)((n + rows - 1) / rows);
    return g;
}

// ---------------------------------------------------------------- probe fill
template <typename T>
__global__ void rademacher_fill_kernel(uint64_t seed, int64_t vec0, int ncols, int64_t ld,
                                       int64_t n, int zero_pad, T* __restrict__ out) {
    const int64_t total = n * ld;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / ld;
        const int64_t j = idx - i * ld;
        if (j < ncols)
            out[idx] = (T)rademacher_sign(seed, (uint64_t)(vec0 + j), (uint64_t)i);
        else if (zero_pad)
            out[idx] = (T)0;
    }
}

hipError_t launch_rademacher(hipStream_t s, uint64_t seed, int64_t vec0, int ncols, int64_t ld,
                             int64_t n, int precision, int zero_pad, void* out) {
    const int64_t total = n * ld;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    if (precision == KPM_FP64)
        rademacher_fill_kernel<double><<<(int)blocks, 256, 0, s>>>(seed, vec0, ncols, ld, n, zero_pad,
                                                                   (double*)out);
    else
        rademacher_fill_kernel<float><<<(int)blocks, 256, 0, s>>>(seed, vec0, ncols, ld, n, zero_pad,
                                                                  (float*)out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- fused step
struct StepParams {
    const int32_t* rp;
    const int32_t* ci;
    const void* val;
    const void* V;    // v_k, gathered
    void* U;          // in: v_{k-1} (unless FIRST), out: v_{k+1}
    double* partial;  // [nblocks][2][ld]: <U_new, V>, <U_new, U_new> per panel
    double alpha, beta;
    int32_t n, ld, lpr, rpw, rows_per_block;
};

template <typename TA, typename TV, bool FIRST>
__global__ __launch_bounds__(kThreads) void cheb_step_kernel(StepParams p) {
    constexpr int N = Pack<TV>::N;
    __shared__ double red[kWaves * 64 * 2 * N];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rw = lane / p.lpr;
    const int cg = lane - rw * p.lpr;
    const bool lane_on = rw < p.rpw;
    const int panel = xcd_panel(blockIdx.x, gridDim.x);
    const int r0 = panel * p.rows_per_block;
    const int r1 = min(p.n, r0 + p.rows_per_block);
    const TA* __restrict__ val = static_cast<const TA*>(p.val);
    const TV* __restrict__ V = static_cast<const TV*>(p.V);
    TV* __restrict__ U = static_cast<TV*>(p.U);
    const int32_t* __restrict__ rp = p.rp;
    const int32_t* __restrict__ ci = p.ci;
    const int64_t ld = p.ld;
    const int coff = cg * N;

    double sx[N], ss[N];
#pragma unroll
    for (int e = 0; e < N; ++e) sx[e] = ss[e] = 0.0;

    if (lane_on) {
        const int pass_rows = kWaves * p.rpw;
        for (int row = r0 + wave * p.rpw + rw; row < r1; row += pass_rows) {
            const int kb = rp[row];
            const int ke = rp[row + 1];
            TV acc[N];
#pragma unroll
            for (int e = 0; e < N; ++e) acc[e] = (TV)0;
            int k = kb;
            for (; k + 4 <= ke; k += 4) {
                const int j0 = ci[k], j1 = ci[k + 1], j2 = ci[k + 2], j3 = ci[k + 3];
                const TV a0 = (TV)val[k], a1 = (TV)val[k + 1], a2 = (TV)val[k + 2], a3 = (TV)val[k + 3];
                TV x0[N], x1[N], x2[N], x3[N];
                Pack<TV>::load(V + j0 * ld + coff, x0);
                Pack<TV>::load(V + j1 * ld + coff, x1);
                Pack<TV>::load(V + j2 * ld + coff, x2);
                Pack<TV>::load(V + j3 * ld + coff, x3);
#pragma unroll
                for (int e = 0; e < N; ++e) {
                    acc[e] = fma(a0, x0[e], acc[e]);
                    acc[e] = fma(a1, x1[e], acc[e]);
                    acc[e] = fma(a2, x2[e], acc[e]);
                    acc[e] = fma(a3, x3[e], acc[e]);
                }
            }
            for (; k < ke; ++k) {
                const int j = ci[k];
                const TV a = (TV)val[k];
                TV x[N];
                Pack<TV>::load(V + j * ld + coff, x);
#pragma unroll
                for (int e = 0; e < N; ++e) acc[e] = fma(a, x[e], acc[e]);
            }
            TV own[N], out[N];
            Pack<TV>::load(V + row * ld + coff, own);
            if (FIRST) {
                // v1 = B v0 = (alpha/2) A v0 + (beta/2) v0
#pragma unroll
                for (int e = 0; e < N; ++e)
                    out[e] = (TV)fma(0.5 * p.alpha, (double)acc[e], 0.5 * p.beta * (double)own[e]);
            } else {
                TV u[N];
                Pack<TV>::load(U + row * ld + coff, u);
#pragma unroll
                for (int e = 0; e < N; ++e)
                    out[e] = (TV)fma(p.alpha, (double)acc[e], fma(p.beta, (double)own[e], -(double)u[e]));
            }
            Pack<TV>::store(U + row * ld + coff, out);
#pragma unroll
            for (int e = 0; e < N; ++e) {
                const double o = (double)out[e];
                sx[e] = fma(o, (double)own[e], sx[e]);
                ss[e] = fma(o, o, ss[e]);
            }
        }
        const int slot = wave * p.rpw + rw;
#pragma unroll
        for (int e = 0; e < N; ++e) {
            red[(slot * 2 + 0) * p.ld + coff + e] = sx[e];
            red[(slot * 2 + 1) * p.ld + coff + e] = ss[e];
        }
    }
    __syncthreads();
    const int nslots = kWaves * p.rpw;
    double* __restrict__ outp = p.partial + (int64_t)panel * 2 * p.ld;
    for (int t = threadIdx.x; t < 2 * p.ld; t += kThreads) {
        const int d = t / p.ld;
        const int c = t - d * p.ld;
        double s = 0.0;
        for (int sl = 0; sl < nslots; ++sl) s += red[(sl * 2 + d) * p.ld + c];
        outp[t] = s;
    }
}

hipError_t launch_cheb_step(hipStream_t s, const CsrDev& A, int precision, bool first,
                            const BlockGeom& g, const void* V, void* U, double alpha, double beta,
                            double* partial) {
    StepParams p;
    p.rp = A.rp;
    p.ci = A.ci;
    p.val = A.val;
    p.V = V;
    p.U = U;
    p.partial = partial;
    p.alpha = alpha;
    p.beta = beta;
    p.n = A.n;
    p.ld = g.ld;
    p.lpr = g.lpr;
    p.rpw = g.rpw;
    p.rows_per_block = g.rows_per_block;
    dim3 grid(g.nblocks), block(kThreads);
    if (precision == KPM_FP64) {
        if (A.val_f64) {
            if (first) cheb_step_kernel<double, double, true><<<grid, block, 0, s>>>(p);
            else cheb_step_kernel<double, double, false><<<grid, block, 0, s>>>(p);
        } else {
            if (first) cheb_step_kernel<float, double, true><<<grid, block, 0, s>>>(p);
            else cheb_step_kernel<float, double, false><<<grid, block, 0, s>>>(p);
        }
    } else {
        if (A.val_f64) return hipErrorInvalidValue;  // FP32 path takes FP32 values
        if (first) cheb_step_kernel<float, float, true><<<grid, block, 0, s>>>(p);
        else cheb_step_kernel<float, float, false><<<grid, block, 0, s>>>(p);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- reductions
// dots[k][t] = sum over panels b of partial[k][b][t], Neumaier-compensated.
// Workgroup (x, k) covers columns t in [64x, 64x+64); its 4 wavefronts take
// contiguous quarters of the panel range and are combined in order.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ partial,
                                                              int nblocks, int width,
                                                              double* __restrict__ dots) {
    __shared__ double sh_s[4][64], sh_c[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + lane;
    const int k = blockIdx.y;
    const int per = (nblocks + 3) / 4;
    const int b0 = wave * per;
    const int b1 = min(nblocks, b0 + per);
    double s = 0.0, c = 0.0;
    if (t < width) {
        const double* src = partial + (int64_t)k * nblocks * width + t;
        for (int b = b0; b < b1; ++b) {
            const double x = src[(int64_t)b * width];
            const double u = s + x;
            c += (fabs(s) >= fabs(x)) ? (s - u) + x : (x - u) + s;
            s = u;
        }
    }
    sh_s[wave][lane] = s;
    sh_c[wave][lane] = c;
    __syncthreads();
    if (wave == 0 && t < width) {
        double S = 0.0, C = 0.0;
        for (int w = 0; w < 4; ++w) {
            const double x = sh_s[w][lane];
            const double u = S + x;
            C += (fabs(S) >= fabs(x)) ? (S - u) + x : (x - u) + S;
            S = u;
            C += sh_c[w][lane];
        }
        dots[(int64_t)k * width + t] = S + C;
    }
}

hipError_t launch_reduce_partials(hipStream_t s, const double* partial, int nblocks, int width,
                                  int K, double* dots) {
    if (K <= 0) return hipSuccess;
    dim3 grid((width + 63) / 64, K);
    reduce_partials_kernel<<<grid, 256, 0, s>>>(partial, nblocks, width, dots);
    return hipGetLastError();
}

// zeta_norm[(vec0 + c)(M+1) + k] = zeta_k / n for column c of the block.
// Step s produced v_{s+1} with D0[s] = <v_{s+1}, v_s>, D1[s] = <v_{s+1}, v_{s+1}>.
//   zeta_0 = n (entries are +/-1),  zeta_1 = D0[0],
//   zeta_{2m} = 2 D1[m-1] - zeta_0,  zeta_{2m+1} = 2 D0[m] - zeta_1  (m >= 1).
__global__ void assemble_kernel(const double* __restrict__ dots, int K, int ld, int ncols, int M,
                                double n, int64_t vec0, double* __restrict__ zeta_norm) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = idx / (M + 1);
    const int k = idx - c * (M + 1);
    if (c >= ncols) return;
    const int w = 2 * ld;
    double z;
    if (k == 0) {
        z = n;
    } else if (k == 1) {
        z = dots[0 * w + 0 * ld + c];
    } else if ((k & 1) == 0) {
        const int m = k >> 1;
        z = 2.0 * dots[(m - 1) * w + 1 * ld + c] - n;
    } else {
        const int m = k >> 1;
        z = 2.0 * dots[m * w + 0 * ld + c] - dots[0 * w + 0 * ld + c];
    }
    zeta_norm[(vec0 + c) * (M + 1) + k] = z / n;
}

hipError_t launch_assemble(hipStream_t s, const double* dots, int K, int ld, int ncols, int M,
                           double n, int64_t vec0, double* zeta_norm) {
    const int total = ncols * (M + 1);
    assemble_kernel<<<(total + 255) / 256, 256, 0, s>>>(dots, K, ld, ncols, M, n, vec0, zeta_norm);
    return hipGetLastError();
}

// mu[k] = (1/nvec) sum_l zeta_norm[l][k], compensated, in probe order.
__global__ void mean_moments_kernel(const double* __restrict__ zeta_norm, int nvec, int M,
                                    double* __restrict__ mu) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > M) return;
    double s = 0.0, c = 0.0;
    for (int l = 0; l < nvec; ++l) {
        const double x = zeta_norm[(int64_t)l * (M + 1) + k];
        const double u = s + x;
        c += (fabs(s) >= fabs(x)) ? (s - u) + x : (x - u) + s;
        s = u;
    }
    mu[k] = (s + c) / (double)nvec;
}

hipError_t launch_mean_moments(hipStream_t s, const double* zeta_norm, int nvec, int M, double* mu) {
    mean_moments_kernel<<<(M + 1 + 127) / 128, 128, 0, s>>>(zeta_norm, nvec, M, mu);
    return hipGetLastError();
}

// ---------------------------------------------------------------- utilities
__global__ void convert_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

hipError_t launch_convert_f64_to_f32(hipStream_t s, const double* in, float* out, int64_t count) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    convert_kernel<<<(int)blocks, 256, 0, s>>>(in, out, count);
    return hipGetLastError();
}

// flags[0]: bad row_ptr, flags[1]: column out of range or unsorted,
// flags[2]: non-finite value.  Set to 1 when found (never cleared here).
template <typename TA>
__global__ void validate_kernel(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const TA* __restrict__ val, int32_t n, int32_t nnz,
                                int* __restrict__ flags) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t kb = rp[i], ke = rp[i + 1];
        if (kb > ke || kb < 0 || ke > nnz || (i == 0 && kb != 0) || (i == n - 1 && ke != nnz)) {
            flags[0] = 1;
            continue;
        }
        int32_t prev = -1;
        for (int32_t k = kb; k < ke; ++k) {
            const int32_t j = ci[k];
            if (j < 0 || j >= n || j <= prev) flags[1] = 1;
            prev = j;
            const double v = (double)val[k];
            if (!isfinite(v)) flags[2] = 1;
        }
    }
}

hipError_t launch_validate_csr(hipStream_t s, const CsrDev& A, int* flags) {
    int64_t blocks = ((int64_t)A.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    if (A.val_f64)
        validate_kernel<double><<<(int)blocks, 256, 0, s>>>(A.rp, A.ci, (const double*)A.val, A.n,
                                                            A.nnz, flags);
    else
        validate_kernel<float><<<(int)blocks, 256, 0, s>>>(A.rp, A.ci, (const float*)A.val, A.n,
                                                           A.nnz, flags);
    return hipGetLastError();
}

}  // namespace kpm
