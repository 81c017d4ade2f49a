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

#include <algorithm>
#include <vector>

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
    int32_t m;       // Lanczos steps of this matrix
};

__device__ __forceinline__ double* part_slot(const LzArgs& a, int kind, int t) {
    return a.part + ((int64_t)kind * LZ_SLOTS + t) * a.nblk;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Store this workgroup's J partial sums (wavefront sums in sh[wave][t]).
__device__ __forceinline__ void lz_store_partials(const LzArgs& a, int kind, int J, int blk,
                                                  double (*sh)[LZ_SLOTS]) {
    __syncthreads();
    if ((int)threadIdx.x < J) {
        const int t = threadIdx.x;
        part_slot(a, kind, t)[blk] = ((sh[0][t] + sh[1][t]) + sh[2][t]) + sh[3][t];
    }
}

// out[t] = sum over workgroups of partial slot t of `kind` (square root when
// MODE == 2; MODE == 0 also copies slot j to alpha_j).  Kinds: 0 projection
// partials of launch A, 2 norm partials of launch B.  Workgroup t: each
// thread adds workgroups tid, tid+256, ... in order, then a fixed tree.
template <int MODE>
__device__ __forceinline__ void lz_reduce_body(const LzArgs& a, int kind, int t, int j, double* out,
                                               double* sh) {
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

template <int MODE>
__global__ __launch_bounds__(LZ_THREADS) void lz_reduce(LzArgs a, int kind, int j, double* out) {
    __shared__ double sh[LZ_THREADS / 64];
    lz_reduce_body<MODE>(a, kind, blockIdx.x, j, out, sh);
}

// A: normalise, w = A q_j, first projection h = Q^T w (workgroup `blk` of
// the matrix's row chunks).
template <typename TA, int R>
__device__ __forceinline__ void lz_spmv_project_body(const LzArgs& a, int blk, int j, double (*sh)[LZ_SLOTS]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // selects, not an index into W: an indexed member array of a struct
    // read from memory (the many-matrix form) would be copied to scratch
    const double* __restrict__ wr = (j & 1) ? a.W[0] : a.W[1];
    double* __restrict__ ww = (j & 1) ? a.W[1] : a.W[0];
    const TA* __restrict__ val = static_cast<const TA*>(a.val);
    const double inv_sqrt_n = 1.0 / sqrt((double)a.n);
    double inv = 0.0;
    if (j > 0) {
        const double beta = a.coef[64 + j - 1];
        inv = beta > 0.0 ? 1.0 / beta : 0.0;
    }
    const int64_t n = a.n;
    double* __restrict__ qj = a.Q + (int64_t)j * n;
    const int64_t i0 = (int64_t)blk * a.chunk + threadIdx.x;
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
    lz_store_partials(a, 0, j + 1, blk, sh);
}

template <typename TA, int R>
__global__ __launch_bounds__(LZ_THREADS) void lz_spmv_project(LzArgs a, int j) {
    __shared__ double sh[LZ_THREADS / 64][LZ_SLOTS];
    lz_spmv_project_body<TA, R>(a, blockIdx.x, j, sh);
}

// B: w -= Q h (h from A's reduction); partial of ||w||^2 (-> beta_j).
template <int R>
__device__ __forceinline__ void lz_orth_body(const LzArgs& a, int blk, int j, double (*sh)[LZ_SLOTS],
                                             double* hs) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int J = j + 1;
    double* __restrict__ ww = (j & 1) ? a.W[1] : a.W[0];
    if ((int)threadIdx.x < J) hs[threadIdx.x] = a.coef[128 + threadIdx.x];
    __syncthreads();
    const int64_t n = a.n;
    const double* __restrict__ Q = a.Q;
    const int64_t i0 = (int64_t)blk * a.chunk + threadIdx.x;
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
    lz_store_partials(a, 2, 1, blk, sh);
}

template <int R>
__global__ __launch_bounds__(LZ_THREADS) void lz_orth(LzArgs a, int j) {
    __shared__ double sh[LZ_THREADS / 64][LZ_SLOTS];
    __shared__ double hs[LZ_SLOTS];
    lz_orth_body<R>(a, blockIdx.x, j, sh, hs);
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
    a.m = m;
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

// ---------------------------------------------------------------- many matrices
// The same run for many matrices at once (kpm_bounds_batched).  Matrices are
// grouped by (rows per thread, value type); per step, one launch of each of
// the four kinds covers every matrix of a group.  Workgroup b of a group's
// A or B launch runs row chunk tab[b].y of matrix tab[b].x with the
// single-matrix code above, and the reductions add each matrix's partials in
// the single-matrix order, so every matrix gets bitwise the coefficients of
// its own launch_lanczos run.  A matrix with fewer steps (n < steps) leaves
// the later launches at once (a workgroup-uniform test).

template <typename TA, int R>
__global__ __launch_bounds__(LZ_THREADS) void lzb_spmv_project(const LzArgs* __restrict__ mats,
                                                               const int2* __restrict__ tab, int j) {
    __shared__ double sh[LZ_THREADS / 64][LZ_SLOTS];
    const int2 e = tab[blockIdx.x];
    const LzArgs a = mats[e.x];
    if (j >= a.m) return;
    lz_spmv_project_body<TA, R>(a, e.y, j, sh);
}

template <int R>
__global__ __launch_bounds__(LZ_THREADS) void lzb_orth(const LzArgs* __restrict__ mats,
                                                       const int2* __restrict__ tab, int j) {
    __shared__ double sh[LZ_THREADS / 64][LZ_SLOTS];
    __shared__ double hs[LZ_SLOTS];
    const int2 e = tab[blockIdx.x];
    const LzArgs a = mats[e.x];
    if (j >= a.m) return;
    lz_orth_body<R>(a, e.y, j, sh, hs);
}

// Workgroup b reduces coefficient b % J of matrix mlist[b / J] (J = j + 1
// projections for MODE 0, the one norm for MODE 2).
template <int MODE>
__global__ __launch_bounds__(LZ_THREADS) void lzb_reduce(const LzArgs* __restrict__ mats,
                                                         const int* __restrict__ mlist, int J, int kind, int j) {
    __shared__ double sh[LZ_THREADS / 64];
    const LzArgs a = mats[mlist[blockIdx.x / J]];
    if (j >= a.m) return;
    lz_reduce_body<MODE>(a, kind, blockIdx.x % J, j, MODE == 2 ? a.coef + 64 + j : a.coef + 128, sh);
}

namespace {
struct LzGroup {
    int R = 1, f64 = 0, m_max = 0;
    int64_t tab_off = 0, entries = 0;  // in the work table
    int64_t list_off = 0, nmats = 0;   // in the matrix list
};

// Groups in a fixed order (R, then value type), matrices in index order.
std::vector<LzGroup> lz_groups(int nmat, const CsrDev* A, const LanczosBatchLayout& L) {
    std::vector<LzGroup> g;
    int64_t tab = 0, list = 0;
    for (int R = 1; R <= 16; R *= 2)
        for (int f = 0; f < 2; ++f) {
            LzGroup G;
            G.R = R;
            G.f64 = f;
            G.tab_off = tab;
            G.list_off = list;
            for (int m = 0; m < nmat; ++m)
                if (L.chunk[m] == LZ_THREADS * R && A[m].val_f64 == f) {
                    G.entries += L.nblk[m];
                    G.nmats += 1;
                    G.m_max = std::max(G.m_max, L.m[m]);
                }
            if (G.nmats == 0) continue;
            tab += G.entries;
            list += G.nmats;
            g.push_back(G);
        }
    return g;
}

template <int R>
void lzb_launch_group(hipStream_t s, const LzGroup& G, int j, const LzArgs* mats, const int2* tab,
                      const int* mlist) {
    const int2* t = tab + G.tab_off;
    const int* ml = mlist + G.list_off;
    if (G.f64) lzb_spmv_project<double, R><<<(unsigned)G.entries, LZ_THREADS, 0, s>>>(mats, t, j);
    else lzb_spmv_project<float, R><<<(unsigned)G.entries, LZ_THREADS, 0, s>>>(mats, t, j);
    lzb_reduce<0><<<(unsigned)(G.nmats * (j + 1)), LZ_THREADS, 0, s>>>(mats, ml, j + 1, 0, j);
    lzb_orth<R><<<(unsigned)G.entries, LZ_THREADS, 0, s>>>(mats, t, j);
    lzb_reduce<2><<<(unsigned)G.nmats, LZ_THREADS, 0, s>>>(mats, ml, 1, 2, j);
}
}  // namespace

void lanczos_batch_layout(int nmat, const CsrDev* A, int steps, LanczosBatchLayout* L) {
    L->m.assign(nmat, 0);
    L->nblk.assign(nmat, 0);
    L->chunk.assign(nmat, 0);
    L->q_off.assign(nmat, 0);
    L->w_off.assign(nmat, 0);
    L->part_off.assign(nmat, 0);
    L->q_total = L->w_total = L->part_total = 0;
    int64_t entries = 0;
    for (int m = 0; m < nmat; ++m) {
        const int64_t n = A[m].n;
        L->m[m] = (int)std::min<int64_t>(steps, n);
        L->chunk[m] = LZ_THREADS * lanczos_rows_per_thread(n);
        L->nblk[m] = (int)((n + L->chunk[m] - 1) / L->chunk[m]);
        L->q_off[m] = L->q_total;
        L->w_off[m] = L->w_total;
        L->part_off[m] = L->part_total;
        L->q_total += (int64_t)L->m[m] * n;
        L->w_total += 2 * n;
        // projection and norm partials, then the Gershgorin hull's [2 x nblk]
        L->part_total += (int64_t)3 * LZ_SLOTS * L->nblk[m] + 2 * L->nblk[m];
        entries += L->nblk[m];
    }
    L->desc_bytes = ((size_t)nmat * sizeof(LzArgs) + 255) / 256 * 256;
    L->tab_bytes = ((size_t)entries * sizeof(int2) + 255) / 256 * 256;
    L->table_bytes = L->desc_bytes + L->tab_bytes + (size_t)nmat * sizeof(int);
}

int64_t lanczos_batch_gershgorin_off(const LanczosBatchLayout& L, int m) {
    return L.part_off[m] + (int64_t)3 * LZ_SLOTS * L.nblk[m];
}

hipError_t launch_lanczos_batched(hipStream_t s, int nmat, const CsrDev* A, uint64_t seed,
                                  const LanczosBatchLayout& L, double* Q, double* w, double* coef, double* part,
                                  void* dev_tables, void* host_stage, int* launches, hipStream_t s2,
                                  hipEvent_t fork, hipEvent_t join) {
    // descriptors, work table and matrix lists, built in the staging buffer
    char* h = static_cast<char*>(host_stage);
    LzArgs* hd = reinterpret_cast<LzArgs*>(h);
    int2* ht = reinterpret_cast<int2*>(h + L.desc_bytes);
    int* hl = reinterpret_cast<int*>(h + L.desc_bytes + L.tab_bytes);
    for (int m = 0; m < nmat; ++m) {
        LzArgs& a = hd[m];
        a.rp = A[m].rp;
        a.ci = A[m].ci;
        a.val = A[m].val;
        a.Q = Q + L.q_off[m];
        a.W[0] = w + L.w_off[m];
        a.W[1] = w + L.w_off[m] + A[m].n;
        a.coef = coef + (int64_t)256 * m;
        a.part = part + L.part_off[m];
        a.seed = seed;
        a.n = A[m].n;
        a.nblk = L.nblk[m];
        a.chunk = L.chunk[m];
        a.m = L.m[m];
    }
    const std::vector<LzGroup> groups = lz_groups(nmat, A, L);
    int m_max = 0;
    for (const LzGroup& G : groups) {
        int64_t t = G.tab_off, l = G.list_off;
        for (int m = 0; m < nmat; ++m) {
            if (L.chunk[m] != LZ_THREADS * G.R || A[m].val_f64 != G.f64) continue;
            hl[l++] = m;
            for (int b = 0; b < L.nblk[m]; ++b) ht[t++] = make_int2(m, b);
        }
        m_max = std::max(m_max, G.m_max);
    }
    hipError_t e = hipMemcpyAsync(dev_tables, host_stage, L.table_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    const LzArgs* dd = static_cast<const LzArgs*>(dev_tables);
    const int2* dt = reinterpret_cast<const int2*>(static_cast<char*>(dev_tables) + L.desc_bytes);
    const int* dl = reinterpret_cast<const int*>(static_cast<char*>(dev_tables) + L.desc_bytes + L.tab_bytes);
    // Groups touch disjoint memory: with a second stream their chains run
    // side by side (odd groups on s2, after the tables' upload).
    const bool two = s2 && fork && join && groups.size() > 1;
    if (two) {
        if ((e = hipEventRecord(fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s2, fork, 0)) != hipSuccess) return e;
    }
    int count = 0;
    for (int j = 0; j < m_max; ++j)
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const LzGroup& G = groups[gi];
            if (j >= G.m_max) continue;
            hipStream_t sg = two && (gi & 1) ? s2 : s;
            switch (G.R) {
                case 1: lzb_launch_group<1>(sg, G, j, dd, dt, dl); break;
                case 2: lzb_launch_group<2>(sg, G, j, dd, dt, dl); break;
                case 4: lzb_launch_group<4>(sg, G, j, dd, dt, dl); break;
                case 8: lzb_launch_group<8>(sg, G, j, dd, dt, dl); break;
                case 16: lzb_launch_group<16>(sg, G, j, dd, dt, dl); break;
                default: return hipErrorInvalidValue;
            }
            count += 4;
        }
    if (two) {
        if ((e = hipEventRecord(join, s2)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, join, 0)) != hipSuccess) return e;
    }
    if (launches) *launches = count;
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
