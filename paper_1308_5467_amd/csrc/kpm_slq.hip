// Stochastic Lanczos DOS (Lin, Saad & Yang, section 3.2.1): for every probe
// vector v_l an M-step Lanczos factorisation A V_M = V_M T_M + f_M e_M^T
// (eq. (lanfact)) started from v_l / ||v_l||, the eigenvalues theta_k of
// T_M and the squared first components tau_k^2 of its eigenvectors
// (eq. (landist)), and the Gaussian-blurred average over probes
// (eq. (landos)).  The run is on B = (A - cI)/d (eq. (cd)), which only
// conditions the arithmetic (Lanczos is shift- and scale-invariant); Ritz
// values are returned in A's units.
//
// Device part: a block of b <= 64 probes runs the plain three-term
// recurrence (no re-orthogonalisation), one sparse product per step, with
// the same LDS-staged CSR panels and XCD-aware resident grid as the
// Chebyshev step.  The state of a row is stored as interleaved pairs
// (u_{k-1}, q_{k-1}) per probe, [n][b][2] FP64, one lane per probe column,
// so a gathered neighbour is one 16-byte load.  Step k reads
// u_{k-1} = B q_{k-1} - beta_{k-2} q_{k-2} and q_{k-1} and forms, per row,
//   q_k     = (u_{k-1} - alpha_{k-1} q_{k-1}) / beta_{k-1}
//   u_k     = B q_k - beta_{k-1} q_{k-1}
// (neighbour entries of q_k are formed the same way from gathered u_{k-1},
// q_{k-1}), stores q_k and u_k, and accumulates per column q_k.u_k,
// u_k.u_k and q_k.q_k.  A reduction launch then sets
//   alpha_k = q_k.u_k,   beta_k = ||u_k - alpha_k q_k||
//           = sqrt(u.u - 2 alpha_k q.u + alpha_k^2 q.q),
// so one step is one data-parallel launch plus one small reduction.  The
// last form cancels as beta_k -> 0 (near a breakdown u_k is almost parallel
// to q_k), so the three sums are carried as unevaluated pairs hi + lo
// (error-free products by FMA, error-free additions) through the per-lane
// accumulation, the workgroup combination and the reduction, and the
// expression is evaluated in the same pair arithmetic: beta_k keeps full
// relative accuracy down to the rounding noise of u_k - alpha_k q_k.  Step 0
// starts from u_{-1} = v, q_{-1} = 0, alpha_{-1} = 0, beta_{-1} = ||v|| = sqrt(n).
//
// Host part: per probe, the breakdown rule (stop at the first beta_k below
// 1e-12 of the largest coefficient so far), the eigenvalues and first
// eigenvector components of the symmetric tridiagonal matrix by implicit
// QR steps with Wilkinson shifts accumulating only the first row of the
// eigenvector matrix (Golub & Welsch), and the blurred density on the device.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "kpm_internal.h"
#include "kpm_step.h"

namespace kpm {

namespace {

// Gathers per batch: 7 (one memory round trip per 7-point stencil row, 100
// VGPRs, 4 wavefronts per SIMD) with 12 KB panels measured 178 us per step
// on a 64^3 stencil with 64 probes, against 188 us for batches of 4 (82
// VGPRs, 5 wavefronts) and 187 us for 8.
constexpr int kSlqG = 7;

// Pair ("double-double") arithmetic: a value is hi + lo with |lo| <= ulp(hi)/2.
struct Dd {
    double hi, lo;
};
__device__ __forceinline__ Dd two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ Dd dd_add(Dd a, Dd b) {
    Dd s = two_sum(a.hi, b.hi);
    s.lo += a.lo + b.lo;
    return two_sum(s.hi, s.lo);
}
// a += x * y with the product's rounding error kept
__device__ __forceinline__ void dd_fma_acc(Dd& a, double x, double y) {
    const double p = x * y;
    const double e = fma(x, y, -p);
    const Dd s = two_sum(a.hi, p);
    a.hi = s.hi;
    a.lo += s.lo + e;
}
__device__ __forceinline__ Dd dd_mul_d(Dd a, double b) {
    const double p = a.hi * b;
    const double e = fma(a.hi, b, -p);
    return two_sum(p, fma(a.lo, b, e));
}

struct SlqParams {
    const int32_t* rp;
    const int32_t* ci;
    const void* val;
    const char* Zp;        // (u_{k-1}, q_{k-1}) pairs, [S][n][ld][2]
    char* Zn;              // (u_k, q_k) pairs
    const double* coef;    // slice s at coef + s * coef_stride: [2][ld] alpha_{k-1}, beta_{k-1}
    double* partial;       // [S][6][ld][pstride]: q.u, u.u, q.q per workgroup as (hi, lo) pairs
    double sA, sI;         // B = sA A + sI I
    int64_t zstride;       // bytes between the slices' (u, q) blocks
    int64_t coef_stride;   // doubles between the slices' coefficient tables
    int32_t n, ld, rpw, rows_per_block, npanels, stage, reverse;
    int32_t slices, pstride;
};

// Slices: S probe blocks run in one launch, block s on the XCDs
// [s * 8/S, (s+1) * 8/S) (hardware round-robin: workgroup b runs on XCD
// b % 8).  Workgroups of one slice are numbered densely, XCD by XCD.
__device__ __forceinline__ void slq_slice_of(int b, int nb, int S, int& slice, int& xg, int& li, int& local,
                                             int& nlocal) {
    const int x = b & 7, q = nb >> 3, r = nb & 7, gsz = 8 / S;
    slice = x / gsz;
    xg = x - slice * gsz;
    li = b >> 3;
    const int x0 = slice * gsz;
    // workgroups on XCDs x0 .. x-1 of this slice, then on the whole slice
    local = (x - x0) * q + max(0, min(x, r) - min(x0, r)) + li;
    nlocal = gsz * q + max(0, min(x0 + gsz, r) - min(x0, r));
}

// One matrix row for one lane (one probe column).  The state of a row is
// stored as (u, q) pairs, so a gathered neighbour is one 16-byte load.
template <typename TA, bool EARLY, int G, typename E>
__device__ __forceinline__ void slq_row(int row, int kb, int ke, const E& csr, const SlqParams& p, uint32_t ldb,
                                        uint32_t coffb, double ap, double inv, double bp, Dd& s_qu, Dd& s_uu,
                                        Dd& s_qq) {
    const uint32_t orow = row * ldb + coffb;
    double z0[2];
    if (EARLY) Pack<double>::load(reinterpret_cast<const double*>(p.Zp + orow), z0);
    double accw = 0.0, accq = 0.0;
    for (int k = kb; k < ke; k += G) {
        int j[G];
        double a[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const bool on = k + i < ke;
            const int ks = on ? k + i : k;
            int jj;
            TA vv;
            csr.get(ks, jj, vv);
            j[i] = on ? jj : row;
            a[i] = on ? (double)vv : 0.0;
        }
        double x[G][2];
#pragma unroll
        for (int i = 0; i < G; ++i)
            Pack<double>::load(reinterpret_cast<const double*>(p.Zp + ((uint32_t)j[i] * ldb + coffb)), x[i]);
#pragma unroll
        for (int i = 0; i < G; ++i) {
            accw = fma(a[i], x[i][0], accw);
            accq = fma(a[i], x[i][1], accq);
        }
    }
    if (!EARLY) Pack<double>::load(reinterpret_cast<const double*>(p.Zp + orow), z0);
    double zn[2];
    const double qn = fma(-ap, z0[1], z0[0]) * inv;
    const double aq = fma(-ap, accq, accw) * inv;  // (A q_k)_row
    zn[0] = fma(p.sA, aq, fma(p.sI, qn, -bp * z0[1]));
    zn[1] = qn;
    Pack<double>::store_nt(reinterpret_cast<double*>(p.Zn + orow), zn);
    dd_fma_acc(s_qu, zn[1], zn[0]);
    dd_fma_acc(s_uu, zn[0], zn[0]);
    dd_fma_acc(s_qq, zn[1], zn[1]);
}

template <typename TA>
__global__ __launch_bounds__(kThreads) void slq_step_kernel(SlqParams p) {
    constexpr int kLdsDoubles = kWaves * 64 * 6;
    __shared__ __align__(16) double smem[kLdsDoubles];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rw = lane / p.ld;
    const int col = lane - rw * p.ld;
    const bool lane_on = rw < p.rpw;
    const TA* __restrict__ val = static_cast<const TA*>(p.val);
    const uint32_t ldb = (uint32_t)p.ld * 16u;
    const uint32_t coffb = (uint32_t)col * 16u;
    const int pass_rows = kWaves * p.rpw;
    const int nslots = kWaves * p.rpw;

    const int nb = gridDim.x;
    int slice = 0, p_begin, p_end, p_stride, first, local = blockIdx.x;
    if (nb >= 8) {
        int xg, li, nlocal;
        slq_slice_of(blockIdx.x, nb, p.slices, slice, xg, li, local, nlocal);
        const int gsz = 8 / p.slices;
        const int x = blockIdx.x & 7;
        p_begin = (int)((int64_t)p.npanels * xg / gsz);
        p_end = (int)((int64_t)p.npanels * (xg + 1) / gsz);
        first = p_begin + li;
        p_stride = nb / 8 + (x < (nb & 7) ? 1 : 0);
    } else {  // one slice only (the host never splits a grid this small)
        p_begin = 0;
        p_end = p.npanels;
        first = blockIdx.x;
        p_stride = nb;
    }
    SlqParams ps = p;  // this slice's blocks
    ps.Zp = p.Zp + slice * p.zstride;
    ps.Zn = p.Zn + slice * p.zstride;
    const double* coef = p.coef + slice * p.coef_stride;

    const int cc = lane_on ? col : 0;
    const double ap = coef[cc];
    const double bp = coef[p.ld + cc];
    const double inv = bp > 0.0 ? 1.0 / bp : 0.0;

    Dd s_qu = {0.0, 0.0}, s_uu = {0.0, 0.0}, s_qq = {0.0, 0.0};
    for (int q = first; q < p_end; q += p_stride) {
        const int panel = p.reverse ? p_begin + p_end - 1 - q : q;
        const int r0 = panel * p.rows_per_block;
        const int r1 = min(p.n, r0 + p.rows_per_block);
        const int R = r1 - r0;
        const int kbase = p.rp[r0];
        const int pnnz = p.rp[r1] - kbase;
        const int off_e = ((R + 1) * 4 + 15) & ~15;
        const bool staged = p.stage && off_e + pnnz * (int)sizeof(CsrPair<TA>) <= (int)sizeof(smem);
        if (staged) {
            char* base = reinterpret_cast<char*>(smem);
            int32_t* s_rp = reinterpret_cast<int32_t*>(base);
            CsrPair<TA>* s_e = reinterpret_cast<CsrPair<TA>*>(base + off_e);
            for (int t = threadIdx.x; t <= R; t += kThreads) s_rp[t] = p.rp[r0 + t] - kbase;
            for (int t = threadIdx.x; t < pnnz; t += kThreads) {
                s_e[t].c = p.ci[kbase + t];
                s_e[t].v = val[kbase + t];
            }
            __syncthreads();
            if (lane_on) {
                const CsrPairs<TA> csr{s_e};
                for (int row = r0 + wave * p.rpw + rw; row < r1; row += pass_rows) {
                    const int lr = row - r0;
                    slq_row<TA, true, kSlqG>(row, s_rp[lr], s_rp[lr + 1], csr, ps, ldb, coffb, ap, inv, bp, s_qu,
                                             s_uu, s_qq);
                }
            }
            __syncthreads();
        } else if (lane_on) {
            const CsrArrays<TA> csr{p.ci, val};
            for (int row = r0 + wave * p.rpw + rw; row < r1; row += pass_rows)
                slq_row<TA, false, kSlqG>(row, p.rp[row], p.rp[row + 1], csr, ps, ldb, coffb, ap, inv, bp, s_qu,
                                          s_uu, s_qq);
        }
    }

    // One partial triple (as hi, lo pairs) per workgroup and column,
    // combined over row slots in a fixed order.
    double* red = smem;
    if (lane_on) {
        const int slot = wave * p.rpw + rw;
        const Dd v[3] = {s_qu, s_uu, s_qq};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            red[(slot * 6 + 2 * d) * p.ld + col] = v[d].hi;
            red[(slot * 6 + 2 * d + 1) * p.ld + col] = v[d].lo;
        }
    }
    __syncthreads();
    // layout [S][6][ld][pstride], entry `local` of this slice: the reduction
    // reads each (quantity, column) row contiguously
    double* __restrict__ part = p.partial + (int64_t)slice * 6 * p.ld * p.pstride;
    for (int t = threadIdx.x; t < 3 * p.ld; t += kThreads) {
        const int d = t / p.ld;
        const int c = t - d * p.ld;
        Dd s = {0.0, 0.0};
        for (int sl = 0; sl < nslots; ++sl)
            s = dd_add(s, Dd{red[(sl * 6 + 2 * d) * p.ld + c], red[(sl * 6 + 2 * d + 1) * p.ld + c]});
        part[((int64_t)(2 * d) * p.ld + c) * p.pstride + local] = s.hi;
        part[((int64_t)(2 * d + 1) * p.ld + c) * p.pstride + local] = s.lo;
    }
}

// alpha_k, beta_k of column blockIdx.x from the partial triples of step k
// (pairs): each of the 256 threads adds a strided subset of the workgroup
// partials in pair arithmetic, then a fixed tree combines them;
// beta_k^2 = u.u - 2 alpha q.u + alpha^2 q.q is evaluated in pairs.
__global__ __launch_bounds__(256) void slq_reduce_kernel(const double* __restrict__ partial_all, int nb, int S,
                                                         int pstride, int ld, double* __restrict__ coef_next_all,
                                                         int64_t coef_stride) {
    __shared__ double sh[3][2][256];
    const int t = threadIdx.x;
    const int c = blockIdx.x;
    const int slice = blockIdx.y;
    int nblocks = nb;
    if (nb >= 8) {  // workgroups of this slice (same count as slq_slice_of)
        const int q = nb >> 3, r = nb & 7, gsz = 8 / S, x0 = slice * gsz;
        nblocks = gsz * q + max(0, min(x0 + gsz, r) - min(x0, r));
    }
    const double* __restrict__ partial = partial_all + (int64_t)slice * 6 * ld * pstride;
    double* __restrict__ coef_next = coef_next_all + slice * coef_stride;
    for (int kind = 0; kind < 3; ++kind) {
        Dd s = {0.0, 0.0};
        const double* __restrict__ ph = partial + ((int64_t)(2 * kind) * ld + c) * pstride;
        const double* __restrict__ pl = partial + ((int64_t)(2 * kind + 1) * ld + c) * pstride;
        for (int b = t; b < nblocks; b += 256) s = dd_add(s, Dd{ph[b], pl[b]});
        sh[kind][0][t] = s.hi;
        sh[kind][1][t] = s.lo;
    }
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st)
            for (int kind = 0; kind < 3; ++kind) {
                const Dd r = dd_add(Dd{sh[kind][0][t], sh[kind][1][t]}, Dd{sh[kind][0][t + st], sh[kind][1][t + st]});
                sh[kind][0][t] = r.hi;
                sh[kind][1][t] = r.lo;
            }
        __syncthreads();
    }
    if (t == 0) {
        const Dd qu = {sh[0][0][0], sh[0][1][0]}, uu = {sh[1][0][0], sh[1][1][0]}, qq = {sh[2][0][0], sh[2][1][0]};
        const double alpha = qu.hi + qu.lo;
        // u.u - 2 alpha q.u + alpha^2 q.q
        const Dd t1 = dd_mul_d(qu, -2.0 * alpha);
        const Dd t2 = dd_mul_d(dd_mul_d(qq, alpha), alpha);
        const Dd b2 = dd_add(dd_add(uu, t1), t2);
        const double b2d = b2.hi + b2.lo;
        coef_next[c] = alpha;
        coef_next[ld + c] = sqrt(b2d > 0.0 ? b2d : 0.0);
    }
}

// Slice s = blockIdx.y of a group: Z_s = (u_{-1}, q_{-1}) = (v, 0) for its
// probe columns vec0_s .. (vec0_s = vec0 + s * ld, ncols_s of them), (0, 0)
// for padding columns; coef_s = (alpha_{-1} = 0, beta_{-1} = ||v|| = sqrt(n))
// for probe columns, (0, 0) for padding.
// rows (nullable): row i takes entry rows[i] of each probe (a renumbered
// matrix's probes at the original indices).
__global__ void slq_init_kernel(uint64_t seed, int64_t vec0, int nvec_left, int ld, int64_t n, double sqrt_n,
                                double* __restrict__ Zall, int64_t zstride_d, double* __restrict__ coef_all,
                                int64_t coef_stride, const int32_t* __restrict__ rows) {
    const int s = blockIdx.y;
    const int64_t v0 = vec0 + (int64_t)s * ld;
    const int ncols = (int)min<int64_t>(ld, max<int64_t>(0, nvec_left - (int64_t)s * ld));
    double* __restrict__ Z = Zall + s * zstride_d;
    double* __restrict__ coef0 = coef_all + s * coef_stride;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 < ld) {
        coef0[i0] = 0.0;
        coef0[ld + i0] = i0 < ncols ? sqrt_n : 0.0;
    }
    const int64_t total = n * ld;
    for (int64_t idx = i0; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / ld;
        const int c = (int)(idx - i * ld);
        const uint64_t gi = rows ? (uint64_t)rows[i] : (uint64_t)i;
        const double v = c < ncols ? (double)rademacher_sign(seed, (uint64_t)(v0 + c), gi) : 0.0;
        Z[2 * idx] = v;
        Z[2 * idx + 1] = 0.0;
    }
}

// Eq. (landos): phi(x_i) = (1/nvec) sum over nodes of tau2 g_sigma(x_i - theta);
// one workgroup per point, fixed-order tree.
__global__ __launch_bounds__(256) void slq_dos_kernel(const double* __restrict__ theta,
                                                      const double* __restrict__ tau2, int64_t nnodes, int nvec,
                                                      double sigma, const double* __restrict__ x,
                                                      double* __restrict__ phi) {
    __shared__ double sh[256];
    const double xi = x[blockIdx.x];
    const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
    const double norm = 1.0 / sqrt(2.0 * M_PI * sigma * sigma);
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < nnodes; k += 256) {
        const double w = tau2[k];
        if (w != 0.0) {
            const double t = xi - theta[k];
            s = fma(w, exp(-t * t * inv2s2), s);
        }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) phi[blockIdx.x] = sh[0] * norm / nvec;
}

// Probe-block geometry: one lane per probe column (ld = columns <= 64),
// rpw = 64 / ld rows per wavefront, row panels of about 12 KB of (u, q) rows.
constexpr int kSlqDefaultBlock = 16;
struct SlqGeom {
    int ld = 0, rpw = 0, rows_per_block = 0, nblocks = 0;
};
SlqGeom slq_geom(int64_t n, int ncols, int hint) {
    SlqGeom g;
    g.ld = ncols;
    g.rpw = 64 / ncols;
    const int rpp = kWaves * g.rpw;
    int passes = hint > 0 ? (hint + rpp - 1) / rpp : (12288 / (16 * ncols) + rpp / 2) / rpp;
    if (passes < 1) passes = 1;
    g.rows_per_block = passes * rpp;
    g.nblocks = (int)((n + g.rows_per_block - 1) / g.rows_per_block);
    return g;
}

int slq_grid(bool f64vals, int npanels) {
    // resident workgroups per kernel variant, found once (threads that race
    // here compute and store the same value)
    static std::atomic<int> res[2] = {{-1}, {-1}};
    int r = res[f64vals ? 1 : 0].load(std::memory_order_relaxed);
    if (r < 0) {
        int dev = 0, per_cu = 0;
        hipDeviceProp_t prop;
        const void* k = f64vals ? reinterpret_cast<const void*>(slq_step_kernel<double>)
                                : reinterpret_cast<const void*>(slq_step_kernel<float>);
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kThreads, 0) == hipSuccess)
            r = per_cu * prop.multiProcessorCount;
        else
            r = 0;
        res[f64vals ? 1 : 0].store(r, std::memory_order_relaxed);
    }
    return r > 0 && r < npanels ? r : npanels;
}

}  // namespace

}  // namespace kpm

using namespace kpm;

// ---------------------------------------------------------------- host eigensolver
// Eigenvalues (ascending) and squared first eigenvector components of the
// symmetric tridiagonal matrix with diagonal a[0..m-1] and off-diagonal
// b[0..m-2]: implicit symmetric QR steps with Wilkinson shifts (Golub & Van
// Loan, section 8.3), each Givens rotation also applied to the first row z
// of the accumulated orthogonal matrix (z starts as e_1), so the weights
// z_k^2 come out without forming eigenvectors (Golub & Welsch).
static bool tridiag_first_row(int m, std::vector<double>& a, std::vector<double>& b, std::vector<double>& z) {
    z.assign(m, 0.0);
    z[0] = 1.0;
    if (m == 1) return true;
    const double eps = 2.220446049250313e-16;
    double anorm = 0.0;
    for (int k = 0; k < m; ++k) anorm = std::max(anorm, fabs(a[k]) + (k > 0 ? fabs(b[k - 1]) : 0.0) +
                                                            (k + 1 < m ? fabs(b[k]) : 0.0));
    // a coupling is negligible against its neighbours or against the norm
    auto small = [&](int i) { return fabs(b[i]) <= eps * (fabs(a[i]) + fabs(a[i + 1])) || fabs(b[i]) <= 0.5 * eps * anorm; };
    int hi = m - 1;
    int iter = 0;
    while (hi > 0) {
        // deflate negligible couplings at the bottom
        if (small(hi - 1)) {
            b[hi - 1] = 0.0;
            --hi;
            iter = 0;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && !small(lo - 1)) --lo;
        if (lo > 0) b[lo - 1] = 0.0;
        if (++iter > 60) return false;
        // Wilkinson shift from the trailing 2 x 2 block
        const double dd = 0.5 * (a[hi - 1] - a[hi]);
        const double e2 = b[hi - 1] * b[hi - 1];
        const double mu = a[hi] - e2 / (dd + copysign(sqrt(dd * dd + e2), dd == 0.0 ? 1.0 : dd));
        double x = a[lo] - mu, y = b[lo];
        for (int k = lo; k < hi; ++k) {
            // rotation G = [c s; -s c] with G^T [x; y] = [r; 0]
            double c, s;
            if (y == 0.0) {
                c = 1.0;
                s = 0.0;
            } else if (fabs(y) > fabs(x)) {
                const double t = -x / y;
                s = 1.0 / sqrt(1.0 + t * t);
                c = s * t;
            } else {
                const double t = -y / x;
                c = 1.0 / sqrt(1.0 + t * t);
                s = c * t;
            }
            if (k > lo) b[k - 1] = c * x - s * y;  // the bulge row becomes the new coupling
            const double p = a[k], q = b[k], r = a[k + 1];
            a[k] = c * c * p - 2.0 * c * s * q + s * s * r;
            a[k + 1] = s * s * p + 2.0 * c * s * q + c * c * r;
            b[k] = c * s * (p - r) + (c * c - s * s) * q;
            if (k + 1 < hi) {
                y = -s * b[k + 1];  // new bulge below the coupling
                b[k + 1] = c * b[k + 1];
            }
            x = b[k];
            const double z0 = z[k], z1 = z[k + 1];
            z[k] = c * z0 - s * z1;
            z[k + 1] = s * z0 + c * z1;
        }
    }
    return true;
}

extern "C" kpm_status kpm_tridiag_eig(int m, const double* alpha, const double* beta, double* theta,
                                      double* tau2) {
    if (m < 1 || !alpha || !theta || !tau2 || (m > 1 && !beta)) return KPM_ERR_ARG;
    std::vector<double> a(alpha, alpha + m), b(m > 1 ? m - 1 : 1, 0.0), z;
    for (int k = 0; k + 1 < m; ++k) {
        if (!std::isfinite(beta[k]) || !std::isfinite(alpha[k])) return KPM_ERR_ARG;
        b[k] = beta[k];
    }
    if (!std::isfinite(alpha[m - 1])) return KPM_ERR_ARG;
    if (!tridiag_first_row(m, a, b, z)) return KPM_ERR_NOCONV;
    std::vector<int> idx(m);
    for (int k = 0; k < m; ++k) idx[k] = k;
    std::sort(idx.begin(), idx.end(), [&](int i, int j) { return a[i] < a[j] || (a[i] == a[j] && i < j); });
    for (int k = 0; k < m; ++k) {
        theta[k] = a[idx[k]];
        tau2[k] = z[idx[k]] * z[idx[k]];
    }
    return KPM_OK;
}

// ---------------------------------------------------------------- kpm_slq
extern "C" kpm_status kpm_slq(kpm_ctx* ctx, const kpm_csr* Ain, double lb, double ub, const kpm_moment_opts* o,
                              double* theta, double* tau2, int* steps_used, double* alpha_out,
                              double* beta_out) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!o) return kpm_fail(ctx, KPM_ERR_ARG, "opts is NULL");
    if ((!theta || !tau2) && !(alpha_out && beta_out && !theta && !tau2))
        return kpm_fail(ctx, KPM_ERR_ARG, "theta and tau2 are needed unless both are NULL and alpha, beta are given");
    if (o->M < 1 || o->M > 4096) return kpm_fail(ctx, KPM_ERR_ARG, "M (Lanczos steps) must be in [1, 4096]");
    if (o->nvec < 1 || o->nvec > (1 << 24)) return kpm_fail(ctx, KPM_ERR_ARG, "nvec must be in [1, 2^24]");
    if (o->precision != KPM_FP64)
        return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "the Lanczos method runs in FP64 (precision KPM_FP64)");
    if (o->block < 0 || o->block > 64) return kpm_fail(ctx, KPM_ERR_ARG, "block out of range (<= 64)");
    if (o->rows_per_block < 0 || o->rows_per_block > (1 << 20))
        return kpm_fail(ctx, KPM_ERR_ARG, "rows_per_block out of range");
    if (!(std::isfinite(lb) && std::isfinite(ub) && ub > lb)) return kpm_fail(ctx, KPM_ERR_ARG, "need finite lb < ub");
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    CsrDev A;
    kpm_status st = kpm_prepare_csr(ctx, Ain, KPM_FP64, &A, "");
    if (st != KPM_OK) return st;
    if (o->validate && (st = kpm_validate_csr(ctx, A)) != KPM_OK) return st;
    // KPM_FLAG_LOCALITY: Lanczos on P A P^T from P v gives the same T
    const int32_t* rows = nullptr;
    if (o->flags & KPM_FLAG_LOCALITY) {
        if (!Ain->on_device) kpm_locality_free(ctx);
        CsrDev R;
        if ((st = kpm_locality_view(ctx, A, &R, &rows)) != KPM_OK) return st;
        A = R;
    }

    const double c = 0.5 * (lb + ub), d = 0.5 * (ub - lb);
    const int M = o->M, nvec = o->nvec;
    int b = o->block > 0 ? std::min(o->block, nvec) : std::min(nvec, kSlqDefaultBlock);
    while (b > 1 && (uint64_t)A.n * b * 16 >= (1ull << 32)) b /= 2;
    if ((uint64_t)A.n * b * 16 >= (1ull << 32))
        return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "probe blocks of the Lanczos method must be smaller than 4 GiB");
    const SlqGeom g = slq_geom(A.n, b, o->rows_per_block);
    const int grid = slq_grid(A.val_f64 != 0, g.nblocks);
    const int nblk_vec = (nvec + b - 1) / b;
    // Slices per launch: up to 8 probe blocks at once, one group of XCDs each
    // (a grid of at least 8 workgroups and 64 panels per XCD of a slice).
    int Smax = 1;
    while (Smax < 8 && Smax * 2 <= nblk_vec && grid >= 8 && g.nblocks >= 64 * Smax * 2 &&
           (uint64_t)A.n * g.ld * 16 * (Smax * 2) <= (32ull << 30))
        Smax *= 2;
    const size_t zbytes = (size_t)A.n * g.ld * 16;
    void *Z0, *Z1, *part, *coef;
    if ((st = kpm_ws(ctx, "X0", zbytes * Smax, &Z0)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "X1", zbytes * Smax, &Z1)) != KPM_OK) return st;
    // S * pstride <= 8 * (grid / 8 + 1) for every S
    const int pmax = grid >= 8 ? 8 * (grid / 8 + 1) : grid;
    if ((st = kpm_ws(ctx, "partial", (size_t)6 * g.ld * pmax * 8, &part)) != KPM_OK) return st;
    const int64_t cstride = (int64_t)(M + 1) * 2 * g.ld;
    if ((st = kpm_ws(ctx, "slq_coef", (size_t)Smax * cstride * 8, &coef)) != KPM_OK) return st;

    std::vector<double> hc((size_t)Smax * cstride);
    std::vector<double> al((size_t)nvec * M), be((size_t)nvec * M);
    kpm_prof_begin(ctx, "slq_step");
    int launches = 0;
    for (int blk = 0; blk < nblk_vec;) {
        int S = Smax;
        while (S > nblk_vec - blk) S /= 2;
        const int ps = grid >= 8 ? (8 / S) * (grid / 8 + 1) : grid;
        const int64_t vec0 = (int64_t)blk * b;
        const int64_t total = (int64_t)A.n * g.ld;
        const int ib = (int)std::min<int64_t>(4096, (total + 255) / 256);
        slq_init_kernel<<<dim3(std::max(ib, 1), S), 256, 0, ctx->stream>>>(
            o->seed, vec0, (int)(nvec - vec0), g.ld, A.n, sqrt((double)A.n), (double*)Z0, (int64_t)(zbytes / 8),
            (double*)coef, cstride, rows);
        KPM_HIP(ctx, hipGetLastError());
        char* Z[2] = {(char*)Z0, (char*)Z1};
        SlqParams p;
        p.rp = A.rp;
        p.ci = A.ci;
        p.val = A.val;
        p.partial = (double*)part;
        p.sA = 1.0 / d;
        p.sI = -c / d;
        p.zstride = (int64_t)zbytes;
        p.coef_stride = cstride;
        p.n = A.n;
        p.ld = g.ld;
        p.rpw = g.rpw;
        p.rows_per_block = g.rows_per_block;
        p.npanels = g.nblocks;
        p.stage = 1;
        p.slices = S;
        p.pstride = ps;
        for (int k = 0; k < M; ++k) {
            p.Zp = Z[k & 1];
            p.Zn = Z[(k + 1) & 1];
            p.coef = (const double*)coef + (size_t)k * 2 * g.ld;
            p.reverse = k & 1;  // start on the rows the previous step ended with
            if (A.val_f64) slq_step_kernel<double><<<grid, kThreads, 0, ctx->stream>>>(p);
            else slq_step_kernel<float><<<grid, kThreads, 0, ctx->stream>>>(p);
            KPM_HIP(ctx, hipGetLastError());
            slq_reduce_kernel<<<dim3(g.ld, S), 256, 0, ctx->stream>>>(
                (double*)part, grid, S, ps, g.ld, (double*)coef + (size_t)(k + 1) * 2 * g.ld, cstride);
            KPM_HIP(ctx, hipGetLastError());
            ++launches;
        }
        KPM_HIP(ctx, hipMemcpyAsync(hc.data(), coef, (size_t)S * cstride * 8, hipMemcpyDeviceToHost, ctx->stream));
        KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
        for (int sl = 0; sl < S; ++sl) {
            const int64_t v0 = vec0 + (int64_t)sl * b;
            const int ncols = (int)std::min<int64_t>(b, nvec - v0);
            const double* h = hc.data() + (size_t)sl * cstride;
            for (int col = 0; col < ncols; ++col)
                for (int k = 0; k < M; ++k) {
                    al[(size_t)(v0 + col) * M + k] = h[(size_t)(k + 1) * 2 * g.ld + col];
                    be[(size_t)(v0 + col) * M + k] = h[(size_t)(k + 1) * 2 * g.ld + g.ld + col];
                }
        }
        blk += S;
    }
    kpm_prof_end(ctx, "slq_step", launches);
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    kpm_prof_collect(ctx);
    if ((st = kpm_locality_check(ctx)) != KPM_OK) return st;
    if (alpha_out) memcpy(alpha_out, al.data(), al.size() * 8);
    if (beta_out) memcpy(beta_out, be.data(), be.size() * 8);
    if (!theta) {  // coefficients only (Haydock's method needs no Ritz values)
        if (steps_used) {
            for (int l = 0; l < nvec; ++l) {
                const double* a = &al[(size_t)l * M];
                const double* bb = &be[(size_t)l * M];
                int m = M;
                double scale = 0.0;
                for (int k = 0; k + 1 < M; ++k) {
                    if (!std::isfinite(a[k]) || !std::isfinite(bb[k]))
                        return kpm_fail(ctx, KPM_ERR_ARG, "non-finite Lanczos coefficient (matrix values not finite?)");
                    scale = std::max(scale, std::max(fabs(a[k]), bb[k]));
                    if (bb[k] <= 1e-12 * scale) {
                        m = k + 1;
                        break;
                    }
                }
                steps_used[l] = m;
            }
        }
        return KPM_OK;
    }
    // Per probe: breakdown rule, nodes and weights, Ritz values in A's units.
    // The probes are independent: up to 16 host threads take every T-th
    // probe (each writes only its probes' rows); errors are reported for the
    // lowest failing probe, as a serial loop would.
    std::vector<kpm_status> pst((size_t)nvec, KPM_OK);
    auto solve = [&](int t, int T) {
        std::vector<double> th(M), w(M);
        for (int l = t; l < nvec; l += T) {
            const double* a = &al[(size_t)l * M];
            const double* bb = &be[(size_t)l * M];
            int m = M;
            double scale = 0.0;
            bool finite = true;
            for (int k = 0; k + 1 < M; ++k) {
                if (!std::isfinite(a[k]) || !std::isfinite(bb[k])) {
                    finite = false;
                    break;
                }
                scale = std::max(scale, std::max(fabs(a[k]), bb[k]));
                if (bb[k] <= 1e-12 * scale) {
                    m = k + 1;
                    break;
                }
            }
            const kpm_status es = finite ? kpm_tridiag_eig(m, a, bb, th.data(), w.data()) : KPM_ERR_ARG;
            if (es != KPM_OK) {
                pst[l] = es;
                continue;
            }
            for (int k = 0; k < M; ++k) {
                theta[(size_t)l * M + k] = k < m ? c + d * th[k] : 0.0;
                tau2[(size_t)l * M + k] = k < m ? w[k] : 0.0;
            }
            if (steps_used) steps_used[l] = m;
        }
    };
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int T = std::max(1, std::min(std::min((int)hw, 16), nvec / 4));
    if (T == 1) {
        solve(0, 1);
    } else {
        std::vector<std::thread> pool;
        pool.reserve(T - 1);
        for (int t = 1; t < T; ++t) pool.emplace_back(solve, t, T);
        solve(0, T);
        for (std::thread& th : pool) th.join();
    }
    for (int l = 0; l < nvec; ++l) {
        if (pst[l] == KPM_ERR_NOCONV)
            return kpm_fail(ctx, KPM_ERR_NOCONV, "tridiagonal eigenvalue iteration did not converge");
        if (pst[l] != KPM_OK)
            return kpm_fail(ctx, KPM_ERR_ARG, "non-finite Lanczos coefficient (matrix values not finite?)");
    }
    return KPM_OK;
}

extern "C" kpm_status kpm_slq_dos(kpm_ctx* ctx, const double* theta, const double* tau2, int nvec, int M,
                                  double sigma, const double* x, int npts, double* phi) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!theta || !tau2 || !x || !phi || nvec < 1 || M < 1 || npts < 0 || !(sigma > 0.0) || !std::isfinite(sigma))
        return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (npts == 0) return KPM_OK;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    const size_t nn = (size_t)nvec * M;
    void *thd, *wd, *xd, *pd;
    kpm_status st;
    if ((st = kpm_ws(ctx, "slq_theta", nn * 8, &thd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "slq_tau2", nn * 8, &wd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dos_x", (size_t)npts * 8, &xd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dos_phi", (size_t)npts * 8, &pd)) != KPM_OK) return st;
    KPM_HIP(ctx, hipMemcpyAsync(thd, theta, nn * 8, hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(wd, tau2, nn * 8, hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(xd, x, (size_t)npts * 8, hipMemcpyHostToDevice, ctx->stream));
    slq_dos_kernel<<<npts, 256, 0, ctx->stream>>>((const double*)thd, (const double*)wd, (int64_t)nn, nvec, sigma,
                                                  (const double*)xd, (double*)pd);
    KPM_HIP(ctx, hipGetLastError());
    KPM_HIP(ctx, hipMemcpyAsync(phi, pd, (size_t)npts * 8, hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return KPM_OK;
}
