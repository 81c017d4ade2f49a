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
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "kpm_internal.h"
#include "kpm_step.h"

namespace kpm {

struct StepTune;
static const StepTune& tune();
static int tune_gather();
static int tune_panel_bytes();

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
        // About 12 KB of vector rows per panel (48 rows at 64 FP32 columns)
        // with at most 4 resident workgroups per CU: the panels one XCD
        // works on at a time then span ~1.5 MB of the gathered block, which
        // keeps most gathers of 3D-stencil neighbours (a plane apart) in
        // that XCD's L2.  Measured against 8 KB panels at 5 workgroups per
        // CU: 2 % faster on a 64^3 stencil, 6 % on 128^3.
        const int row_bytes = g.ld * (precision == KPM_FP64 ? 8 : 4);
        int passes = (tune_panel_bytes() / row_bytes + rows_per_pass / 2) / rows_per_pass;
        if (passes < 1) passes = 1;
        rows = passes * rows_per_pass;
    }
    g.rows_per_block = rows;
    g.nblocks = (int)((n + rows - 1) / rows);
    g.gather = tune_gather();
    return g;
}

// ---------------------------------------------------------------- probe fill
// Thread t of a workgroup owns column t % ld of rows t / ld, t / ld + rpp,
// ... (rpp = 256 / ld rows per pass, ld <= 256): stores are coalesced and
// no 64-bit division is needed per element.
template <typename T>
__global__ __launch_bounds__(256) void rademacher_fill_kernel(uint64_t seed, int64_t vec0, int ncols, int ld,
                                                              int64_t n, int zero_pad, T* __restrict__ out,
                                                              const int32_t* __restrict__ rows) {
    const int rpp = 256 / ld;
    const int r_in = (int)threadIdx.x / ld;
    const int j = (int)threadIdx.x - r_in * ld;
    if (r_in >= rpp || (j >= ncols && !zero_pad)) return;
    for (int64_t i = (int64_t)blockIdx.x * rpp + r_in; i < n; i += (int64_t)gridDim.x * rpp) {
        const uint64_t gi = rows ? (uint64_t)rows[i] : (uint64_t)i;
        out[i * ld + j] = j < ncols ? (T)rademacher_sign(seed, (uint64_t)(vec0 + j), gi) : (T)0;
    }
}

// Any leading dimension (the public fill allows ld > 256): one element per
// thread and pass.
template <typename T>
__global__ __launch_bounds__(256) void rademacher_fill_wide_kernel(uint64_t seed, int64_t vec0, int ncols,
                                                                   int64_t ld, int64_t n, int zero_pad,
                                                                   T* __restrict__ out,
                                                                   const int32_t* __restrict__ rows) {
    const int64_t total = n * ld;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
        const int64_t i = idx / ld;
        const int64_t j = idx - i * ld;
        if (j < ncols)
            out[idx] = (T)rademacher_sign(seed, (uint64_t)(vec0 + j), rows ? (uint64_t)rows[i] : (uint64_t)i);
        else if (zero_pad)
            out[idx] = (T)0;
    }
}

hipError_t launch_rademacher(hipStream_t s, uint64_t seed, int64_t vec0, int ncols, int64_t ld,
                             int64_t n, int precision, int zero_pad, void* out, const int32_t* rows) {
    if (ld < 1) return hipErrorInvalidValue;
    if (ld > 256) {
        const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(16384, (n * ld + 255) / 256));
        if (precision == KPM_FP64)
            rademacher_fill_wide_kernel<double><<<(int)blocks, 256, 0, s>>>(seed, vec0, ncols, ld, n, zero_pad,
                                                                            (double*)out, rows);
        else
            rademacher_fill_wide_kernel<float><<<(int)blocks, 256, 0, s>>>(seed, vec0, ncols, ld, n, zero_pad,
                                                                           (float*)out, rows);
        return hipGetLastError();
    }
    const int64_t rpp = 256 / ld;
    int64_t blocks = (n + rpp - 1) / rpp;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    if (precision == KPM_FP64)
        rademacher_fill_kernel<double><<<(int)blocks, 256, 0, s>>>(seed, vec0, ncols, (int)ld, n, zero_pad,
                                                                   (double*)out, rows);
    else
        rademacher_fill_kernel<float><<<(int)blocks, 256, 0, s>>>(seed, vec0, ncols, (int)ld, n, zero_pad,
                                                                  (float*)out, rows);
    return hipGetLastError();
}

// ---------------------------------------------------------------- fused step
struct StepParams {
    const int32_t* rp;
    const int32_t* ci;
    const void* val;
    const void* V;    // v_k, gathered
    void* U;          // in: v_{k-1} (unless FIRST), out: v_{k+1}
    double* partial;  // [grid][2][ld]: <U_new, V>, <U_new, U_new> per workgroup
    double alpha, beta;
    int32_t n, ld, lpr, rpw, rows_per_block, npanels, stage;
    int32_t reverse;  // walk each XCD's panel range from its end
    int32_t ntu;      // non-temporal loads of U (probe blocks beyond the MALL)
    // Legendre step only: coefficient of v_{k-1}, sign bits of v_0
    double gam;
    const uint32_t* sgn;
    int32_t sw;
};

// Fused step.  The grid is sized to the number of workgroups that fit on
// the device at once; workgroups running on XCD x (hardware round-robin
// b % 8) walk the x-th contiguous eighth of the row panels, so neighbouring
// rows -- and the gathered rows of banded matrices -- share that XCD's L2.
// With `reverse` set the walk runs from the end of each eighth: alternate
// steps then begin on the rows the previous step ended with.  With `stage`
// set, a panel's slice of the CSR arrays (row offsets, column indices,
// values) is first copied to LDS with coalesced loads when it fits (about 60
// entries per row on average at the default FP32 panel height, 30 for FP64),
// so each row costs one round of independent gathers.  Each workgroup accumulates its dot
// products over all the rows it processes and writes one partial pair per
// probe column at the end; the grid size and the panel-to-workgroup map are
// fixed for a device and direction, so results are bitwise reproducible run
// to run.
//
// LEG: the Legendre step of Algorithm DGL, U <- alpha A V + beta V + gam U,
// whose first dot is taken against v_0 (its sign bits) instead of V.
template <typename TA, typename TV, bool FIRST, bool OFF32, int G, bool LEG = false>
__global__ __launch_bounds__(kThreads) void cheb_step_kernel(StepParams p) {
    constexpr int N = Pack<TV>::N;
    constexpr int kLdsDoubles = kWaves * 64 * 2 * N;
    __shared__ __align__(16) double smem[kLdsDoubles];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rw = lane / p.lpr;
    const int cg = lane - rw * p.lpr;
    const bool lane_on = rw < p.rpw;
    const TA* __restrict__ val = static_cast<const TA*>(p.val);
    const char* __restrict__ Vb = static_cast<const char*>(p.V);
    char* __restrict__ Ub = static_cast<char*>(p.U);
    const int32_t* __restrict__ rp = p.rp;
    const int32_t* __restrict__ ci = p.ci;
    const uint32_t ldb = (uint32_t)p.ld * (uint32_t)sizeof(TV);
    const int coff = cg * N;
    const uint32_t coffb = (uint32_t)coff * (uint32_t)sizeof(TV);
    const int nslots = kWaves * p.rpw;

    // Panel range of this workgroup.
    const int nb = gridDim.x;
    int p_begin, p_end, p_stride, first;
    if (nb >= 8) {
        const int x = blockIdx.x & 7, li = blockIdx.x >> 3;
        const int gx = nb / 8 + (x < (nb & 7) ? 1 : 0);
        p_begin = (int)((int64_t)p.npanels * x / 8);
        p_end = (int)((int64_t)p.npanels * (x + 1) / 8);
        first = p_begin + li;
        p_stride = gx;
    } else {
        p_begin = 0;
        p_end = p.npanels;
        first = blockIdx.x;
        p_stride = nb;
    }

    double sx[N], ss[N];
#pragma unroll
    for (int e = 0; e < N; ++e) sx[e] = ss[e] = 0.0;
    const LegArgs leg{p.sgn, p.sw, coff >> 5, coff & 31, p.gam};

    for (int q = first; q < p_end; q += p_stride) {
        const int panel = p.reverse ? p_begin + p_end - 1 - q : q;
        const int r0 = panel * p.rows_per_block;
        const int r1 = min(p.n, r0 + p.rows_per_block);
        process_panel<TA, TV, FIRST, OFF32, G, kLdsDoubles, LEG>(r0, r1, rp, ci, val, Vb, Ub, ldb, coffb, p.alpha,
                                                                 p.beta, p.stage, smem, lane_on, wave, rw, p.rpw, sx,
                                                                 ss, &leg, p.ntu);
    }

    // One partial per workgroup: the lanes' sums over every row they
    // processed, combined over row slots in a fixed order.
    double* red = smem;
    if (lane_on) {
        const int slot = wave * p.rpw + rw;
#pragma unroll
        for (int e = 0; e < N; ++e) {
            red[(slot * 2 + 0) * p.ld + coff + e] = sx[e];
            red[(slot * 2 + 1) * p.ld + coff + e] = ss[e];
        }
    }
    __syncthreads();
    double* __restrict__ outp = p.partial + (int64_t)blockIdx.x * 2 * p.ld;
    for (int t = threadIdx.x; t < 2 * p.ld; t += kThreads) {
        const int d = t / p.ld;
        const int c = t - d * p.ld;
        double s = 0.0;
        for (int sl = 0; sl < nslots; ++sl) s += red[(sl * 2 + d) * p.ld + c];
        outp[t] = s;
    }
}

// Tuning knobs, read once from KPM_TUNE
// ("stage=0|1,persist=0|1,gather=4|7|8,rev=0|1,wpc=N,panel=BYTES").
// Gather batches of 7 fit a 7-point stencil row in one memory round trip and
// keep the FP32 step at 93 VGPRs (5 waves per SIMD; 8 needs 98, 4 waves).
// wpc caps the resident workgroups per CU of the step kernel (0: no cap);
// panel is the default panel height in bytes of vector rows.
struct StepTune {
    int stage = 1;
    int persist = 1;
    int gather = 7;
    int rev = 1;
    int wpc = 4;
    int panel = 12288;
};
static StepTune read_tune() {
    StepTune t;
    const char* e = getenv("KPM_TUNE");
    if (e) {
        const char* s;
        if ((s = strstr(e, "stage="))) t.stage = atoi(s + 6);
        if ((s = strstr(e, "persist="))) t.persist = atoi(s + 8);
        if ((s = strstr(e, "gather="))) {
            const int gv = atoi(s + 7);
            t.gather = gv == 4 || gv == 8 ? gv : 7;
        }
        if ((s = strstr(e, "rev="))) t.rev = atoi(s + 4);
        if ((s = strstr(e, "wpc="))) t.wpc = std::max(0, atoi(s + 4));
        if ((s = strstr(e, "panel="))) t.panel = std::min(1 << 20, std::max(256, atoi(s + 6)));
    }
    return t;
}
static const StepTune& tune() {
    static StepTune t = read_tune();
    return t;
}
static int tune_gather() { return tune().gather; }
static int tune_panel_bytes() { return tune().panel; }

// Workgroups of `kernel` kept resident on the current device at once: the
// occupancy limit, capped at the per-CU limit of the step kernel (0 if
// unknown).  The batched step keeps its full occupancy: its work table
// spreads many small matrices over the resident workgroups, and capping it
// at 4 per CU measured 11 % slower on 48 uneven matrices.
static int resident_blocks(const void* kernel) {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess) return 0;
    if (tune().wpc > 0) per_cu = std::min(per_cu, tune().wpc);
    return per_cu * prop.multiProcessorCount;
}

template <typename TA, typename TV, bool FIRST, bool OFF32, int G>
static int resident_of() {
    static const int r = resident_blocks(reinterpret_cast<const void*>(cheb_step_kernel<TA, TV, FIRST, OFF32, G>));
    return r;
}

template <typename TA, typename TV, bool OFF32, int G>
static int grid_of(int npanels) {
    int grid = npanels;
    if (tune().persist) {
        const int r = std::min(resident_of<TA, TV, true, OFF32, G>(), resident_of<TA, TV, false, OFF32, G>());
        if (r > 0 && r < grid) grid = r;
    }
    return grid;
}

template <typename TA, typename TV, bool FIRST, bool OFF32, int G, bool LEG = false>
static hipError_t launch_step_variant(hipStream_t s, const StepParams& p, int grid) {
    cheb_step_kernel<TA, TV, FIRST, OFF32, G, LEG><<<grid, kThreads, 0, s>>>(p);
    return hipGetLastError();
}

static bool step_off32(const CsrDev& A, const BlockGeom& g, int precision) {
    const int esz = precision == KPM_FP64 ? 8 : 4;
    return (uint64_t)A.n * (uint64_t)g.ld * (uint64_t)esz < (1ull << 32);
}

int cheb_step_grid(const CsrDev& A, int precision, const BlockGeom& g) {
    const bool off32 = step_off32(A, g, precision);
#define KPM_GRID_V(TA, TV, O)                                                              \
    return g.gather == 4 ? grid_of<TA, TV, O, 4>(g.nblocks)                                \
                         : (g.gather == 8 ? grid_of<TA, TV, O, 8>(g.nblocks) : grid_of<TA, TV, O, 7>(g.nblocks))
#define KPM_GRID(TA, TV)          \
    if (off32) {                  \
        KPM_GRID_V(TA, TV, true); \
    }                             \
    KPM_GRID_V(TA, TV, false)
    if (precision == KPM_FP64) {
        if (A.val_f64) KPM_GRID(double, double);
        KPM_GRID(float, double);
    }
    KPM_GRID(float, float);
#undef KPM_GRID
#undef KPM_GRID_V
}

hipError_t launch_cheb_step(hipStream_t s, const CsrDev& A, int precision, bool first,
                            const BlockGeom& g, int grid, const void* V, void* U, double alpha,
                            double beta, double* partial, bool reverse, const LegStep* leg) {
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
    p.npanels = g.nblocks;
    p.stage = tune().stage;
    p.reverse = reverse && tune().rev;
    // probe blocks larger than 128 MiB (the MALL holds 256 MB and the U
    // stream would otherwise evict the gathered rows from it)
    p.ntu = (uint64_t)A.n * (uint64_t)g.ld * (precision == KPM_FP64 ? 8u : 4u) > (128ull << 20);
    p.gam = leg ? leg->gam : 0.0;
    p.sgn = leg ? leg->sgn : nullptr;
    p.sw = leg ? leg->sw : 0;
    const bool lg = leg != nullptr && !first;
    const bool off32 = step_off32(A, g, precision);
#define KPM_STEP_G(TA, TV, GG)                                                                             \
    if (lg)                                                                                                \
        return off32 ? launch_step_variant<TA, TV, false, true, GG, true>(s, p, grid)                      \
                     : launch_step_variant<TA, TV, false, false, GG, true>(s, p, grid);                    \
    return off32 ? (first ? launch_step_variant<TA, TV, true, true, GG>(s, p, grid)                        \
                          : launch_step_variant<TA, TV, false, true, GG>(s, p, grid))                      \
                 : (first ? launch_step_variant<TA, TV, true, false, GG>(s, p, grid)                       \
                          : launch_step_variant<TA, TV, false, false, GG>(s, p, grid))
#define KPM_STEP_DISPATCH(TA, TV)    \
    if (g.gather == 4) {             \
        KPM_STEP_G(TA, TV, 4);       \
    } else if (g.gather == 8) {      \
        KPM_STEP_G(TA, TV, 8);       \
    } else {                         \
        KPM_STEP_G(TA, TV, 7);       \
    }
    if (precision == KPM_FP64) {
        if (A.val_f64) KPM_STEP_DISPATCH(double, double);
        KPM_STEP_DISPATCH(float, double);
    }
    if (A.val_f64) return hipErrorInvalidValue;  // the FP32 path takes FP32 values
    KPM_STEP_DISPATCH(float, float);
#undef KPM_STEP_DISPATCH
#undef KPM_STEP_G
}

// ---------------------------------------------------------------- reductions
// dots[k][t] = sum over workgroups b of partial[k][b][t], Neumaier-compensated.
// Workgroup (x, k) covers columns t in [64x, 64x+64); its 16 wavefronts take
// contiguous slices of the workgroup range and are combined in order.
constexpr int kRedWaves = 16;
__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
    const double u = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - u) + x : (x - u) + s;
    s = u;
}

__global__ __launch_bounds__(64 * kRedWaves) void reduce_partials_kernel(const double* __restrict__ partial,
                                                                        int nblocks, int width,
                                                                        double* __restrict__ dots) {
    __shared__ double sh_s[kRedWaves][64], sh_c[kRedWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + lane;
    const int k = blockIdx.y;
    const int per = (nblocks + kRedWaves - 1) / kRedWaves;
    const int b0 = wave * per;
    const int b1 = min(nblocks, b0 + per);
    double s = 0.0, c = 0.0;
    if (t < width) {
        const double* src = partial + (int64_t)k * nblocks * width + t;
        int b = b0;
        for (; b + 4 <= b1; b += 4) {
            const double x0 = src[(int64_t)b * width], x1 = src[(int64_t)(b + 1) * width];
            const double x2 = src[(int64_t)(b + 2) * width], x3 = src[(int64_t)(b + 3) * width];
            neumaier_add(s, c, x0);
            neumaier_add(s, c, x1);
            neumaier_add(s, c, x2);
            neumaier_add(s, c, x3);
        }
        for (; b < b1; ++b) neumaier_add(s, c, src[(int64_t)b * width]);
    }
    sh_s[wave][lane] = s;
    sh_c[wave][lane] = c;
    __syncthreads();
    if (wave == 0 && t < width) {
        double S = 0.0, C = 0.0;
        for (int w = 0; w < kRedWaves; ++w) {
            neumaier_add(S, C, sh_s[w][lane]);
            C += sh_c[w][lane];
        }
        dots[(int64_t)k * width + t] = S + C;
    }
}

hipError_t launch_reduce_partials(hipStream_t s, const double* partial, int nblocks, int width,
                                  int K, double* dots) {
    if (K <= 0) return hipSuccess;
    dim3 grid((width + 63) / 64, K);
    reduce_partials_kernel<<<grid, 64 * kRedWaves, 0, s>>>(partial, nblocks, width, dots);
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

// mu[k] = (1/nvec) sum_l zeta_norm[l][k]: one wavefront per k; lane j adds
// probes j, j+64, ... with compensation, then a fixed butterfly.
__global__ __launch_bounds__(64) void mean_moments_kernel(const double* __restrict__ zeta_norm, int nvec, int M,
                                                          double* __restrict__ mu) {
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    double s = 0.0, c = 0.0;
    for (int l = lane; l < nvec; l += 64) neumaier_add(s, c, zeta_norm[(int64_t)l * (M + 1) + k]);
    s += c;
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) mu[k] = s / (double)nvec;
}

hipError_t launch_mean_moments(hipStream_t s, const double* zeta_norm, int nvec, int M, double* mu) {
    mean_moments_kernel<<<M + 1, 64, 0, s>>>(zeta_norm, nvec, M, mu);
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
