// Batched moments for many matrices of uneven size (Lin, Saad & Yang,
// Algorithm 1 applied to a set of matrices, with the product identity of
// Appendix A).
//
// Work decomposition.  Every (matrix, probe block) pair -- an "mv" -- has
// its own ping-pong vector blocks.  One launch per recurrence step covers
// every mv of every matrix: a host-built work table gives each workgroup a
// share of the row panels of one mv, the number of workgroups per mv
// proportional to its bytes of work and the total close to the number of
// workgroups resident on the device, so small matrices never leave the GPU
// idle and each workgroup writes exactly one dot partial per step (with more
// mvs than resident workgroups, every mv gets at least kMinEntriesPerMv).
// Workgroup b reads table entry xcd_panel(b), so consecutive entries run on
// the same XCD; the entries of one mv on one XCD share a contiguous panel
// range and stride through it together (one moving band of rows per mv and
// XCD, whose plane-apart gathers stay in that XCD's L2).
//
// On-chip path.  When every matrix is small enough that two probe blocks of
// it fit in one workgroup's LDS (160 KB on gfx950: n = 2,048 with 8 FP32 or
// 4 FP64 probes per block), each (matrix, probe block) pair is owned by one
// workgroup for all ceil(M/2) steps: the probes are generated in LDS, both
// recurrence vectors stay there, the CSR is read from global memory (L2:
// the pairs of one matrix run side by side on one XCD), each step's dots are
// reduced in a fixed order and assembled into the per-probe moments at once.
// No vector ever reaches HBM and no barrier is needed beyond the
// workgroup's own, which answers the cross-step fence cost below for pairs
// that fit.  Per row the arithmetic is that of the streaming step (same
// FP32 sum order over the row's entries, the same FP64 combination), so
// the vectors are bitwise those of the streaming path; only the dots'
// summation order differs.
//
// Steps are separate launches rather than one kernel with device-wide
// barriers between steps: on MI355X a device-scope release/acquire writes
// back and invalidates an XCD's L2, while back-to-back launches on one
// stream have no measurable gap.  The whole sequence (probe fill, K steps,
// reductions, assembly, means, range check) is captured once per shape in a
// HIP graph and replayed; per-call scalars (alpha, beta, seed) live in a
// device table uploaded before the replay, so the graph never changes.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <vector>

#include "kpm_step.h"

namespace kpm {

// One workgroup: panels first, first + stride, ... < end of mv, one of the
// `stride` workgroups that share the panel range [base, end) on one XCD.
struct BatchEntryDev {
    int32_t mv, first, end, stride, base, pad0, pad1, pad2;
};

struct BatchMvDev {  // one (matrix, probe block)
    const int32_t* rp;
    const int32_t* ci;
    const void* val;
    char* X0;
    char* X1;
    double alpha, beta;
    uint64_t seed;
    int32_t n, ncols, mat, vec0;
};

__device__ __forceinline__ void bneumaier(double& s, double& c, double x) {
    const double u = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - u) + x : (x - u) + s;
    s = u;
}

// Step k also reduces earlier steps' dots, in two levels, so that no
// workgroup adds more than a few memory round trips to a step and only two
// steps of partials are stored whatever the number of table entries:
//  - the workgroup that runs entry e of an mv with (e - first entry) a
//    multiple of kChunk adds step k - 1's partials (`prev`) of entries
//    e .. e + kChunk - 1 in order (compensated) into chunk_out[e];
//  - the workgroup that runs the mv's first entry adds step k - 2's chunk
//    sums (`chunk_in`, written by the previous launch) in order into the
//    mv's dots.
// batched_final_reduce_kernel finishes the last two steps in the same order.
constexpr int kChunk = 16;

template <typename TA, typename TV, bool FIRST, int G>
__global__ __launch_bounds__(kThreads) void batched_step_kernel(const BatchEntryDev* __restrict__ entries,
                                                                const BatchMvDev* __restrict__ mvs, int parity,
                                                                int ld, int lpr, int rpw, int rows_per_panel,
                                                                int stage, double* __restrict__ partial,
                                                                const double* __restrict__ prev,
                                                                const int32_t* __restrict__ e0,
                                                                const int32_t* __restrict__ e1,
                                                                double* __restrict__ chunk_out,
                                                                const double* __restrict__ chunk_in,
                                                                double* __restrict__ dots_prev2) {
    constexpr int N = Pack<TV>::N;
    __shared__ __align__(16) double smem[kWaves * 64 * 2 * N];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rw = lane / lpr;
    const int cg = lane - rw * lpr;
    const bool lane_on = rw < rpw;
    const int e = xcd_panel(blockIdx.x, gridDim.x);
    const BatchEntryDev E = entries[e];
    const BatchMvDev& mv = mvs[E.mv];
    const char* Vb = parity ? mv.X1 : mv.X0;
    char* Ub = parity ? mv.X0 : mv.X1;
    const uint32_t ldb = (uint32_t)ld * (uint32_t)sizeof(TV);
    const uint32_t coffb = (uint32_t)(cg * N) * (uint32_t)sizeof(TV);
    const TA* val = static_cast<const TA*>(mv.val);
    double sx[N], ss[N];
#pragma unroll
    for (int i = 0; i < N; ++i) sx[i] = ss[i] = 0.0;
    // The workgroups sharing a range stride through it together, so the rows
    // they work on at a time form one band and the gathered rows a few
    // planes away stay in the XCD's L2.  Odd steps walk the range backwards,
    // starting on the rows the previous step ended with.
    for (int q = E.first; q < E.end; q += E.stride) {
        const int panel = parity ? E.base + E.end - 1 - q : q;
        const int r0 = panel * rows_per_panel;
        const int r1 = min(mv.n, r0 + rows_per_panel);
        process_panel<TA, TV, FIRST, true, G>(r0, r1, mv.rp, mv.ci, val, Vb, Ub, ldb, coffb, mv.alpha, mv.beta,
                                              stage, smem, lane_on, wave, rw, rpw, sx, ss);
    }
    double* red = smem;
    if (lane_on) {
        const int slot = wave * rpw + rw;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            red[(slot * 2 + 0) * ld + cg * N + i] = sx[i];
            red[(slot * 2 + 1) * ld + cg * N + i] = ss[i];
        }
    }
    __syncthreads();
    const int nslots = kWaves * rpw;
    double* __restrict__ outp = partial + (int64_t)e * 2 * ld;
    for (int t = threadIdx.x; t < 2 * ld; t += kThreads) {
        const int d = t / ld;
        const int c = t - d * ld;
        double s = 0.0;
        for (int sl = 0; sl < nslots; ++sl) s += red[(sl * 2 + d) * ld + c];
        outp[t] = s;
    }
    if (!FIRST) {
        const int width = 2 * ld, ef = e0[E.mv], el = e1[E.mv];
        if ((e - ef) % kChunk == 0) {  // one memory round trip
            const int f1 = min(el, e + kChunk);
            for (int t = threadIdx.x; t < width; t += kThreads) {
                double x[kChunk];
#pragma unroll
                for (int u = 0; u < kChunk; ++u) x[u] = e + u < f1 ? prev[(int64_t)(e + u) * width + t] : 0.0;
                double s = 0.0, c = 0.0;
#pragma unroll
                for (int u = 0; u < kChunk; ++u)
                    if (e + u < f1) bneumaier(s, c, x[u]);
                chunk_out[(int64_t)e * width + t] = s + c;
            }
        }
        if (chunk_in && e == ef) {  // chunk sums loaded 16 per round trip
            for (int t = threadIdx.x; t < width; t += kThreads) {
                double s = 0.0, c = 0.0;
                for (int f = ef; f < el; f += 16 * kChunk) {
                    double x[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u)
                        x[u] = f + u * kChunk < el ? chunk_in[(int64_t)(f + u * kChunk) * width + t] : 0.0;
#pragma unroll
                    for (int u = 0; u < 16; ++u)
                        if (f + u * kChunk < el) bneumaier(s, c, x[u]);
                }
                dots_prev2[(int64_t)E.mv * width + t] = s + c;
            }
        }
    }
}

// ---------------------------------------------------------------- on-chip path
constexpr int kResWaves = 16;
constexpr int kResThreads = 64 * kResWaves;

// Dynamic LDS of the on-chip kernel: two [n x LD] vector blocks and the
// per-wave dot partials of two steps.
__host__ __device__ constexpr size_t resident_lds_bytes(int n, int LD, int esz) {
    return (((size_t)2 * n * LD * esz + 15) & ~(size_t)15) + (size_t)2 * kResWaves * 2 * LD * 8;
}

// Sliced layout of the matrices for the on-chip kernel.  A wavefront works
// on C rows at a time (C = rows per wavefront), and its loads of the k-th
// entry of those rows from CSR touch C different rows' entries -- many
// cache lines per instruction, which made the texture path, not the bytes,
// the limit.  Here each matrix's rows are ordered by decreasing length
// (ties by index) and cut into slices of C; slice s stores its entries
// slot-major, entry q of its l-th row at [slo[s] + q C + l] for q < W_s,
// the slice's longest row, with that row's index in srow[s C + l] (-1 past
// the last row); slots are stored in pairs, slots 2p and 2p + 1 of row l
// at [slo[s] + p 2C + 2l + {0, 1}], the width rounded up to even.  Slots
// past a row's end hold the row itself with weight 0 (exact), as the
// streaming step pads its gather batches.  A wavefront's load of two slots
// is then one 16-byte load per lane over 2C consecutive pairs (FP32
// values); ordering by length keeps
// each slice's rows about equally long, so few slots are padding; and each
// row's entries keep their CSR order, so the FP32 row sums are those of the
// streaming path (only the order in which a lane accumulates its rows' dot
// products changes).  Order, widths and offsets are fixed when the plan is
// built; the entries are refilled from the CSR at every call (values may
// change between calls, the sparsity structure of a matrix at a given
// address not: a row longer than its slice's width is reported).
struct SellMatDev {
    const int32_t* rp;
    const int32_t* ci;
    const void* val;
    void* sell;          // the slots of all matrices
    const int32_t* slw;  // width of each slice of this matrix
    const int64_t* slo;  // first slot of each slice (index into sell)
    const int32_t* srow; // row of each slice lane [nsl * C], -1 past the last row
    int32_t n, nsl;
};

// Row lengths of every matrix (grid: x over rows, y over matrices).
__global__ void row_length_kernel(const SellMatDev* __restrict__ mats, const int64_t* __restrict__ row_base,
                                  int32_t* __restrict__ len) {
    const SellMatDev& m = mats[blockIdx.y];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < m.n) len[row_base[blockIdx.y] + r] = m.rp[r + 1] - m.rp[r];
}

// Fill every matrix's slots from its CSR (grid: x over slice lanes, y over matrices).
template <typename TA>
__global__ void sell_fill_kernel(const SellMatDev* __restrict__ mats, int C, int* __restrict__ bad) {
    const SellMatDev& m = mats[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = i / C, l = i - s * C;
    if (s >= m.nsl) return;
    const int W = m.slw[s];
    const int r = m.srow[i];
    CsrPair<TA>* e = static_cast<CsrPair<TA>*>(m.sell) + m.slo[s] + 2 * l;
    const TA* val = static_cast<const TA*>(m.val);
    int kb = 0, len = 0;
    if (r >= 0) {
        kb = m.rp[r];
        len = m.rp[r + 1] - kb;
        if (len > W) bad[0] = 1;
    }
    const int Wp = (W + 1) & ~1;
    for (int q = 0; q < Wp; ++q) {
        CsrPair<TA> t;
        if (q < len) {
            t.c = m.ci[kb + q];
            t.v = val[kb + q];
        } else {
            t.c = r >= 0 ? r : 0;
            t.v = (TA)0;
        }
        e[(int64_t)(q >> 1) * 2 * C + (q & 1)] = t;
    }
}

// Sum of v over the lanes of the wavefront with the same lane % LPR (LPR =
// 1, 2 or 4), returned in every such lane.  Within each row of 16 lanes by
// DPP lane moves (quad permutations for the strides below 4, row rotations
// by 4 and 8), then across rows by gfx950's row swaps: permlane16_swap of a
// value with itself gives every lane the value of its even-row partner and
// of its odd-row partner, permlane32_swap those of its lower-half and
// upper-half partners, so one add per level (even + odd, lower + upper, the
// same order in every lane).  All on the vector ALU: the LDS unit, which
// the gathers keep busy, sees no shuffles.  A fixed pattern: bitwise
// reproducible.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
__device__ __forceinline__ double from_halves(uint32_t lo, uint32_t hi) {
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint64_t)lo);
}
__device__ __forceinline__ double sum_row_pairs(double v) {  // rows 2i + 2i+1
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)u, (uint32_t)u, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
    return from_halves(lo[0], hi[0]) + from_halves(lo[1], hi[1]);
}
__device__ __forceinline__ double sum_halves(double v) {  // lanes l and l ^ 32
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)u, (uint32_t)u, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
    return from_halves(lo[0], hi[0]) + from_halves(lo[1], hi[1]);
}
template <int LPR>
__device__ __forceinline__ double wave_sum_strided(double v) {
    static_assert(LPR == 1 || LPR == 2 || LPR == 4, "lane stride");
    if (LPR == 1) v += dpp_move<0xB1>(v);  // quad_perm [1,0,3,2]: lane ^ 1
    if (LPR <= 2) v += dpp_move<0x4E>(v);  // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_move<0x124>(v);               // row_ror:4
    v += dpp_move<0x128>(v);               // row_ror:8
    return sum_halves(sum_row_pairs(v));
}

// Two consecutive slots of the sliced layout: one 16-byte load for FP32
// values, two for FP64.
template <typename TA>
__device__ __forceinline__ void load_slot_pair(const __attribute__((address_space(1))) CsrPair<TA>* p, int& j0,
                                               TA& a0, int& j1, TA& a1);
template <>
__device__ __forceinline__ void load_slot_pair<float>(const __attribute__((address_space(1))) CsrPair<float>* p,
                                                      int& j0, float& a0, int& j1, float& a1) {
    typedef int i4 __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) i4* gi4;
    const i4 t = *reinterpret_cast<gi4>(p);
    j0 = t[0];
    a0 = __int_as_float(t[1]);
    j1 = t[2];
    a1 = __int_as_float(t[3]);
}
template <>
__device__ __forceinline__ void load_slot_pair<double>(const __attribute__((address_space(1))) CsrPair<double>* p,
                                                       int& j0, double& a0, int& j1, double& a1) {
    j0 = p[0].c;
    a0 = p[0].v;
    j1 = p[1].c;
    a1 = p[1].v;
}

// One workgroup per (matrix, probe block) pair for all K steps (see the
// file comment).  Writes zeta_norm[(mat * nvec + vec0 + c) * (M+1) + k] for
// k = 0..M and the pair's columns c < ncols, as batched_assemble_kernel does
// from the streaming path's dots:
//   zeta_0 = n, zeta_1 = D0[0], zeta_{2m} = 2 D1[m-1] - n, zeta_{2m+1} = 2 D0[m] - zeta_1,
// with D0[k] = <v_{k+1}, v_k> and D1[k] = <v_{k+1}, v_{k+1}> of step k.
template <typename TA, typename TV, int LD, int G>
__global__ __launch_bounds__(kResThreads) void resident_kernel(const BatchMvDev* __restrict__ mvs,
                                                               const SellMatDev* __restrict__ mats, int nmv, int K,
                                                               int M, int nvec, double* __restrict__ zeta_norm) {
    constexpr int N = Pack<TV>::N;
    constexpr int LPR = LD / N;            // lanes per matrix row
    constexpr int RPW = 64 / LPR;          // rows per wavefront = slice height
    extern __shared__ __align__(16) char lds_raw[];
    const int pi = xcd_panel(blockIdx.x, nmv);  // consecutive pairs (one matrix's blocks) on one XCD
    const BatchMvDev& mv = mvs[pi];
    const SellMatDev& sm = mats[mv.mat];
    const int n = mv.n;
    TV* const buf0 = reinterpret_cast<TV*>(lds_raw);
    TV* const buf1 = buf0 + (size_t)n * LD;
    double* const red = reinterpret_cast<double*>(lds_raw + (((size_t)2 * n * LD * sizeof(TV) + 15) & ~(size_t)15));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rw = lane / LPR, cg = lane - rw * LPR;
    const int c0 = cg * N;
    const double nn = (double)n;
    double* const zrow = zeta_norm + ((int64_t)mv.mat * nvec + mv.vec0) * (M + 1);
    // zeta_0 = n: normalised 1
    if ((int)threadIdx.x < mv.ncols) zrow[(int64_t)threadIdx.x * (M + 1)] = 1.0;
    if (K == 0) return;

    // v_0: Rademacher probes vec0 .. vec0 + ncols - 1, zero padding columns
    for (int idx = threadIdx.x; idx < n * LD; idx += kResThreads) {
        const int i = idx / LD, j = idx - i * LD;
        buf0[idx] = j < mv.ncols ? (TV)rademacher_sign(mv.seed, (uint64_t)(mv.vec0 + j), (uint64_t)i) : (TV)0;
    }
    __syncthreads();
    // global (not generic) pointers: the slot loads become global loads
    typedef const __attribute__((address_space(1))) CsrPair<TA>* gpair;
    const gpair sell = (gpair)sm.sell;
    const int32_t* __restrict__ slw = sm.slw;
    const int64_t* __restrict__ slo = sm.slo;
    double zeta1 = 0.0;  // D0[0] of column threadIdx.x (threads < LD)
    const int32_t* __restrict__ srow = sm.srow;
    // G slots q0 .. q0 + G - 1 of this lane's row in slice s (slots at or past
    // the slice width W, which is the same for the whole wavefront, are not
    // loaded: the row itself with weight 0).
    static_assert(G % 2 == 0, "slots are loaded in pairs");
    auto load_batch = [&](int64_t base, int W, int q0, int row, int (&j)[G], TV (&a)[G]) {
#pragma unroll
        for (int i = 0; i < G; i += 2) {
            if (q0 + i < W) {
                const int64_t at = base + (int64_t)((q0 + i) >> 1) * 2 * RPW + 2 * rw;
                TA v0, v1;
                load_slot_pair<TA>(sell + at, j[i], v0, j[i + 1], v1);
                a[i] = (TV)v0;
                a[i + 1] = (TV)v1;
            } else {
                j[i] = j[i + 1] = row;
                a[i] = a[i + 1] = (TV)0;
            }
        }
    };
    // The first batch of a wavefront's next slice is loaded while the
    // current one gathers (the slots do not change between steps, so the
    // last slice of a step loads the first one's batch for the next step).
    const int nsl = sm.nsl;
    int jn[G];
    TV an[G];
    int rown = 0;
    if (wave < nsl) {
        rown = srow[wave * RPW + rw];
        load_batch(slo[wave], slw[wave], 0, rown, jn, an);
    }
    for (int k = 0; k < K; ++k) {
        const TV* V = (k & 1) ? buf1 : buf0;
        TV* U = (k & 1) ? buf0 : buf1;
        const double alpha = k == 0 ? 0.5 * mv.alpha : mv.alpha;
        const double beta = k == 0 ? 0.5 * mv.beta : mv.beta;
        double sx[N], ss[N];
#pragma unroll
        for (int e = 0; e < N; ++e) sx[e] = ss[e] = 0.0;
#pragma unroll 1
        for (int sl = wave; sl < nsl; sl += kResWaves) {
            const int row = rown;
            int jc[G];
            TV ac[G];
#pragma unroll
            for (int i = 0; i < G; ++i) {
                jc[i] = jn[i];
                ac[i] = an[i];
            }
            const int W = slw[sl];
            const int64_t base = slo[sl];
            const int sn = sl + kResWaves < nsl ? sl + kResWaves : wave;
            rown = srow[sn * RPW + rw];
            if (sn != wave || k + 1 < K) load_batch(slo[sn], slw[sn], 0, rown, jn, an);
            TV acc[N];
#pragma unroll
            for (int e = 0; e < N; ++e) acc[e] = (TV)0;
            for (int q = 0; q < W; q += G) {
                if (q != 0) load_batch(base, W, q, row, jc, ac);
                if (row >= 0) {
                    // only the slice's W slots: the slots of the last batch
                    // past W are not gathered (W is the same for the wavefront)
                    TV x[G][N];
#pragma unroll
                    for (int i = 0; i < G; ++i)
                        if (q + i < W) Pack<TV>::load(V + (size_t)jc[i] * LD + c0, x[i]);
#pragma unroll
                    for (int i = 0; i < G; ++i)
                        if (q + i < W)
#pragma unroll
                            for (int e = 0; e < N; ++e) acc[e] = fma(ac[i], x[i][e], acc[e]);
                }
            }
            if (row < 0) continue;
            TV own[N], out[N];
            Pack<TV>::load(V + (size_t)row * LD + c0, own);
            if (k == 0) {
#pragma unroll
                for (int e = 0; e < N; ++e) out[e] = (TV)fma(alpha, (double)acc[e], beta * (double)own[e]);
            } else {
                TV u[N];
                Pack<TV>::load(U + (size_t)row * LD + c0, u);
#pragma unroll
                for (int e = 0; e < N; ++e)
                    out[e] = (TV)fma(alpha, (double)acc[e], fma(beta, (double)own[e], -(double)u[e]));
            }
            Pack<TV>::store(U + (size_t)row * LD + c0, out);
#pragma unroll
            for (int e = 0; e < N; ++e) {
                const double o = (double)out[e];
                sx[e] = fma(o, (double)own[e], sx[e]);
                ss[e] = fma(o, o, ss[e]);
            }
        }
        // rows of the wavefront -> one value per column
#pragma unroll
        for (int e = 0; e < N; ++e) {
            sx[e] = wave_sum_strided<LPR>(sx[e]);
            ss[e] = wave_sum_strided<LPR>(ss[e]);
        }
        double* rk = red + (size_t)(k & 1) * kResWaves * 2 * LD;
        if (rw == 0) {
#pragma unroll
            for (int e = 0; e < N; ++e) {
                rk[(wave * 2 + 0) * LD + c0 + e] = sx[e];
                rk[(wave * 2 + 1) * LD + c0 + e] = ss[e];
            }
        }
        __syncthreads();  // U complete for the next step; the partials of step k readable
        const int t = threadIdx.x;
        if (t < 2 * LD) {
            const int d = t / LD, c = t - d * LD;
            double s = 0.0;
            for (int w = 0; w < kResWaves; ++w) s += rk[(w * 2 + d) * LD + c];
            if (c < mv.ncols) {
                if (d == 0) {  // D0[k]: zeta_{2k+1}
                    if (k == 0) zeta1 = s;
                    const double z = k == 0 ? s : 2.0 * s - zeta1;
                    if (2 * k + 1 <= M) zrow[(int64_t)c * (M + 1) + 2 * k + 1] = z / nn;
                } else if (2 * k + 2 <= M) {  // D1[k]: zeta_{2k+2}
                    zrow[(int64_t)c * (M + 1) + 2 * k + 2] = (2.0 * s - nn) / nn;
                }
            }
        }
    }
}

// Probe blocks of every mv: X0 = Rademacher probes vec0.. of seed_mv (zero padding).
template <typename T>
__global__ void batched_fill_kernel(const BatchMvDev* __restrict__ mvs, int ld) {
    const BatchMvDev& mv = mvs[blockIdx.y];
    T* out = reinterpret_cast<T*>(mv.X0);
    // thread t: column t % ld of rows t / ld + k (256 / ld) (ld <= 256)
    const int rpp = 256 / ld;
    const int r_in = (int)threadIdx.x / ld;
    const int j = (int)threadIdx.x - r_in * ld;
    if (r_in >= rpp) return;
    for (int64_t i = (int64_t)blockIdx.x * rpp + r_in; i < mv.n; i += (int64_t)gridDim.x * rpp)
        out[i * ld + j] = j < mv.ncols ? (T)rademacher_sign(mv.seed, (uint64_t)(mv.vec0 + j), (uint64_t)i) : (T)0;
}

// The last two steps' dots, in the order of the step kernels' two levels:
// dots_prev2 (step K - 2, when chunk_prev is given) adds the stored chunk
// sums; dots_last (step K - 1) forms each chunk's sum of `partial` as a
// chunk leader would and adds those.
__global__ __launch_bounds__(64) void batched_final_reduce_kernel(const double* __restrict__ partial,
                                                                  const double* __restrict__ chunk_prev,
                                                                  int width, const int32_t* __restrict__ e0,
                                                                  const int32_t* __restrict__ e1, int nmv,
                                                                  double* __restrict__ dots_prev2,
                                                                  double* __restrict__ dots_last) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    const int mv = blockIdx.z;
    if (t >= width) return;
    const int ef = e0[mv], el = e1[mv];
    if (chunk_prev) {
        double s = 0.0, c = 0.0;
        for (int f = ef; f < el; f += kChunk) bneumaier(s, c, chunk_prev[(int64_t)f * width + t]);
        dots_prev2[(int64_t)mv * width + t] = s + c;
    }
    double s = 0.0, c = 0.0;
    for (int f = ef; f < el; f += kChunk) {
        const int f1 = min(el, f + kChunk);
        double s1 = 0.0, c1 = 0.0;
        for (int e = f; e < f1; ++e) bneumaier(s1, c1, partial[(int64_t)e * width + t]);
        bneumaier(s, c, s1 + c1);
    }
    dots_last[(int64_t)mv * width + t] = s + c;
}

// zeta_norm[mat][vec0 + c][k] = zeta_k / n of probe vec0 + c.
__global__ void batched_assemble_kernel(const double* __restrict__ dots, const BatchMvDev* __restrict__ mvs,
                                        int nmv, int ld, int M, int nvec, double* __restrict__ zeta_norm) {
    const int mv = blockIdx.y;
    const BatchMvDev& d = mvs[mv];
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = idx / (M + 1);
    const int k = idx - c * (M + 1);
    if (c >= d.ncols) return;
    const int64_t w = (int64_t)nmv * 2 * ld;  // stride between steps
    const double* dm = dots + (int64_t)mv * 2 * ld;
    const double n = (double)d.n;
    double z;
    if (k == 0) z = n;
    else if (k == 1) z = dm[c];
    else if ((k & 1) == 0) z = 2.0 * dm[(int64_t)((k >> 1) - 1) * w + ld + c] - n;
    else z = 2.0 * dm[(int64_t)(k >> 1) * w + c] - dm[c];
    zeta_norm[((int64_t)d.mat * nvec + d.vec0 + c) * (M + 1) + k] = z / n;
}

// mu[mat][k] = mean over probes; maxabs[mat] = max |zeta_norm| (inf if any is non-finite).
__global__ __launch_bounds__(64) void batched_mean_kernel(const double* __restrict__ zeta_norm, int nvec, int M,
                                                          double* __restrict__ mu) {
    const int k = blockIdx.x, mat = blockIdx.y, lane = threadIdx.x;
    const double* z = zeta_norm + (int64_t)mat * nvec * (M + 1);
    double s = 0.0, c = 0.0;
    for (int l = lane; l < nvec; l += 64) bneumaier(s, c, z[(int64_t)l * (M + 1) + k]);
    s += c;
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) mu[(int64_t)mat * (M + 1) + k] = s / (double)nvec;
}

__global__ __launch_bounds__(256) void batched_check_kernel(const double* __restrict__ zeta_norm, int nvec, int M,
                                                            double* __restrict__ maxabs) {
    __shared__ double sh[256];
    const int mat = blockIdx.x;
    const int64_t cnt = (int64_t)nvec * (M + 1);
    const double* z = zeta_norm + (int64_t)mat * cnt;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < cnt; i += 256) {
        const double a = fabs(z[i]);
        m = isfinite(a) ? fmax(m, a) : INFINITY;
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) maxabs[mat] = sh[0];
}

}  // namespace kpm

using namespace kpm;

// ---------------------------------------------------------------- host side
namespace {

struct BatchShape {  // what a captured graph depends on
    std::vector<uintptr_t> ptrs;
    std::vector<int64_t> dims;
    bool operator==(const BatchShape& o) const { return ptrs == o.ptrs && dims == o.dims; }
};

struct BatchPlan {
    BatchShape shape;
    int nmat = 0, nmv = 0, nentries = 0, M = 0, K = 0, nvec = 0, ld = 0, lpr = 0, rpw = 0, rows = 0;
    int precision = 0, val_f64 = 0, stage = 1;
    bool resident = false;  // the on-chip path: one workgroup per mv for all steps
    size_t lds_bytes = 0;   // its dynamic LDS per workgroup
    int sell_C = 0, max_nsl = 0;   // its slice height and the most slices of a matrix
    void* sell_mem = nullptr;      // its slots (second allocation)
    SellMatDev* d_mats = nullptr;  // per matrix: CSR and slice tables
    int* d_bad = nullptr;          // set when a row outgrows its slice
    std::vector<BatchMvDev> mvs;  // host copy (alpha/beta/seed refreshed per call)
    void* mem = nullptr;          // one device allocation for everything below
    size_t mem_bytes = 0;
    BatchEntryDev* d_entries = nullptr;
    BatchMvDev* d_mvs = nullptr;
    int32_t* d_e0 = nullptr;
    int32_t* d_e1 = nullptr;
    double* d_partial = nullptr;
    double* d_chunk = nullptr;  // chunk sums of two steps, at their leaders' entries
    double* d_dots = nullptr;
    double* d_zeta = nullptr;
    double* d_mu = nullptr;
    double* d_maxabs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t gstream = nullptr;
};

template <typename TA, typename TV>
int batched_resident() {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(batched_step_kernel<TA, TV, false, 7>), kThreads, 0) !=
        hipSuccess)
        return 0;
    return per_cu * prop.multiProcessorCount;
}

template <typename TA, typename TV, int LD>
const void* resident_fn() {
    // 8 slots per batch; 4 with FP64 vectors (16-byte slots and FP64 rows
    // would spill at 8)
    return reinterpret_cast<const void*>(resident_kernel<TA, TV, LD, sizeof(TV) == 8 ? 4 : 8>);
}

// The on-chip kernel for this precision and block width (ld), or nullptr.
template <typename TA, typename TV>
const void* resident_kernel_for(int ld) {
    constexpr int N = Pack<TV>::N;
    if (ld == 4 * N) return resident_fn<TA, TV, 4 * N>();
    if (ld == 2 * N) return resident_fn<TA, TV, 2 * N>();
    if (ld == N) return resident_fn<TA, TV, N>();
    return nullptr;
}

__global__ void clear_flag_kernel(int* flag) { flag[0] = 0; }

template <typename TA, typename TV>
hipError_t enqueue_resident(hipStream_t s, const BatchPlan& P) {
    const void* fn = resident_kernel_for<TA, TV>(P.ld);
    if (!fn) return hipErrorInvalidValue;
    clear_flag_kernel<<<1, 1, 0, s>>>(P.d_bad);
    const dim3 fg((unsigned)(((int64_t)P.max_nsl * P.sell_C + 255) / 256), P.nmat);
    sell_fill_kernel<TA><<<fg, 256, 0, s>>>(P.d_mats, P.sell_C, P.d_bad);
    int nmv = P.nmv, K = P.K, M = P.M, nvec = P.nvec;
    double* z = P.d_zeta;
    const BatchMvDev* mvs = P.d_mvs;
    const SellMatDev* mats = P.d_mats;
    void* args[] = {(void*)&mvs, (void*)&mats, &nmv, &K, &M, &nvec, &z};
    hipError_t e = hipLaunchKernel(fn, dim3(P.nmv), dim3(kResThreads), args, P.lds_bytes, s);
    if (e != hipSuccess) return e;
    dim3 mg(P.M + 1, P.nmat);
    batched_mean_kernel<<<mg, 64, 0, s>>>(P.d_zeta, P.nvec, P.M, P.d_mu);
    batched_check_kernel<<<P.nmat, 256, 0, s>>>(P.d_zeta, P.nvec, P.M, P.d_maxabs);
    return hipGetLastError();
}

template <typename TA, typename TV>
hipError_t enqueue_batched(hipStream_t s, const BatchPlan& P) {
    if (P.resident) return enqueue_resident<TA, TV>(s, P);
    dim3 fill_grid(256, P.nmv);
    batched_fill_kernel<TV><<<fill_grid, 256, 0, s>>>(P.d_mvs, P.ld);
    const size_t width = 2 * (size_t)P.ld;
    // partials of step k go to half k & 1 and step k - 1's chunk sums to
    // chunk half (k - 1) & 1; step k reads the other halves
    const size_t half = (size_t)P.nentries * width;
    for (int k = 0; k < P.K; ++k) {
        double* pk = P.d_partial + (size_t)(k & 1) * half;
        if (k == 0)
            batched_step_kernel<TA, TV, true, 7><<<P.nentries, kThreads, 0, s>>>(
                P.d_entries, P.d_mvs, 0, P.ld, P.lpr, P.rpw, P.rows, P.stage, pk, nullptr, P.d_e0, P.d_e1,
                nullptr, nullptr, nullptr);
        else
            batched_step_kernel<TA, TV, false, 7><<<P.nentries, kThreads, 0, s>>>(
                P.d_entries, P.d_mvs, k & 1, P.ld, P.lpr, P.rpw, P.rows, P.stage, pk,
                P.d_partial + (size_t)((k - 1) & 1) * half, P.d_e0, P.d_e1,
                P.d_chunk + (size_t)((k - 1) & 1) * half, k >= 2 ? P.d_chunk + (size_t)(k & 1) * half : nullptr,
                k >= 2 ? P.d_dots + (size_t)(k - 2) * P.nmv * width : nullptr);
    }
    if (P.K > 0) {  // the last two steps' dots
        dim3 rg((unsigned)((width + 63) / 64), 1, P.nmv);
        const bool two = P.K >= 2;
        batched_final_reduce_kernel<<<rg, 64, 0, s>>>(
            P.d_partial + (size_t)((P.K - 1) & 1) * half, two ? P.d_chunk + (size_t)((P.K - 2) & 1) * half : nullptr,
            (int)width, P.d_e0, P.d_e1, P.nmv, two ? P.d_dots + (size_t)(P.K - 2) * P.nmv * width : nullptr,
            P.d_dots + (size_t)(P.K - 1) * P.nmv * width);
    }
    dim3 ag((P.ld * (P.M + 1) + 255) / 256, P.nmv);
    batched_assemble_kernel<<<ag, 256, 0, s>>>(P.d_dots, P.d_mvs, P.nmv, P.ld, P.M, P.nvec, P.d_zeta);
    dim3 mg(P.M + 1, P.nmat);
    batched_mean_kernel<<<mg, 64, 0, s>>>(P.d_zeta, P.nvec, P.M, P.d_mu);
    batched_check_kernel<<<P.nmat, 256, 0, s>>>(P.d_zeta, P.nvec, P.M, P.d_maxabs);
    return hipGetLastError();
}

hipError_t enqueue_plan(hipStream_t s, const BatchPlan& P) {
    if (P.precision == KPM_FP64)
        return P.val_f64 ? enqueue_batched<double, double>(s, P) : enqueue_batched<float, double>(s, P);
    return enqueue_batched<float, float>(s, P);
}

void free_plan(BatchPlan& P) {
    if (P.exec) hipGraphExecDestroy(P.exec);
    if (P.graph) hipGraphDestroy(P.graph);
    if (P.mem) hipFree(P.mem);
    if (P.sell_mem) hipFree(P.sell_mem);
    P.shape = BatchShape();  // a plan is reused only once its build has completed
    P.exec = nullptr;
    P.graph = nullptr;
    P.mem = nullptr;
    P.sell_mem = nullptr;
    P.mem_bytes = 0;
}

}  // namespace

// The plans of the two most recently used shapes (a caller alternating
// between two batches, or a batch and the sub-batch of its escaping
// matrices, keeps both captured).
struct kpm_batch_state {
    BatchPlan plan[2];
    int mru = 0;
};

void kpm_batch_free(kpm_ctx* ctx) {
    if (!ctx->batch) return;
    for (BatchPlan& P : ctx->batch->plan) {
        hipStreamSynchronize(P.gstream ? P.gstream : ctx->stream);
        free_plan(P);
        if (P.gstream) hipStreamDestroy(P.gstream);
    }
    delete ctx->batch;
    ctx->batch = nullptr;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// LDS bytes one workgroup may use on `device` (queried once per device).
static size_t lds_per_workgroup(int device) {
    static std::atomic<size_t> cache[64];
    if (device < 0 || device >= 64) return 0;
    size_t v = cache[device].load(std::memory_order_relaxed);
    if (!v) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 0;
        v = prop.sharedMemPerBlock;
        cache[device].store(v, std::memory_order_relaxed);
    }
    return v;
}

// Lower bound on the table entries (workgroups) per mv when there are more
// mvs than resident workgroups.  The proportional share then rounds to one
// workgroup each, so about as many mvs as resident workgroups are in flight
// at once and their gathered probe blocks (512 KB each at n = 2,048, 64 FP32
// probes) far exceed the caches.  Splitting each mv over at least 16
// workgroups keeps a few mvs per XCD in flight: 9,216 matrices of n = 2,048,
// degree 127, 256 probes took 1.34 s instead of 2.07 s (32 or 43 workgroups
// per mv: no further gain).  With fewer mvs the table stays at one wave of
// resident workgroups: the same bound on the 48-matrix uneven batch pushed
// it past one wave and cost 30 %.
constexpr int kMinEntriesPerMv = 16;

kpm_status kpm_moments_batched_seeded(kpm_ctx* ctx, int nmat, const kpm_csr* A, const double* lb, const double* ub,
                                     const kpm_moment_opts* o, const uint64_t* seeds, double* mu, double* max_abs_mu) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (nmat < 1 || nmat > 65535 || !A || !lb || !ub || !o || !mu)
        return kpm_fail(ctx, KPM_ERR_ARG, "bad argument (nmat in [1, 65535], arrays non-NULL)");
    if (o->M < 0 || o->M > (1 << 16)) return kpm_fail(ctx, KPM_ERR_ARG, "M must be in [0, 65536]");
    if (o->nvec < 1 || o->nvec > (1 << 20)) return kpm_fail(ctx, KPM_ERR_ARG, "nvec must be in [1, 2^20]");
    if (o->precision != KPM_FP32 && o->precision != KPM_FP64)
        return kpm_fail(ctx, KPM_ERR_ARG, "precision must be KPM_FP32 or KPM_FP64");
    const int maxb = o->precision == KPM_FP64 ? 128 : 256;
    if (o->block < 0 || o->block > maxb) return kpm_fail(ctx, KPM_ERR_ARG, "block out of range");
    for (int m = 0; m < nmat; ++m) {
        if (!(std::isfinite(lb[m]) && std::isfinite(ub[m]) && ub[m] > lb[m]))
            return kpm_fail(ctx, KPM_ERR_ARG, "need finite lb[m] < ub[m] for every matrix");
        if (!A[m].on_device) return kpm_fail(ctx, KPM_ERR_ARG, "batched matrices must be device-resident");
        if (A[m].val_is_f64 != A[0].val_is_f64)
            return kpm_fail(ctx, KPM_ERR_ARG, "all batched matrices must share one value type");
        if (o->precision == KPM_FP32 && A[m].val_is_f64)
            return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "batched FP32 path needs FP32 values");
    }
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    kpm_status st;
    std::vector<CsrDev> D(nmat);
    for (int m = 0; m < nmat; ++m) {
        if ((st = kpm_prepare_csr(ctx, &A[m], o->precision, &D[m], "")) != KPM_OK) return st;
        if (o->validate && (st = kpm_validate_csr(ctx, D[m])) != KPM_OK) return st;
    }
    const int M = o->M, nvec = o->nvec;
    int64_t nmax = 0;
    for (int m = 0; m < nmat; ++m) nmax = std::max<int64_t>(nmax, D[m].n);
    const int esz = o->precision == KPM_FP64 ? 8 : 4;
    // On-chip path (file comment): the widest block of N, 2N or 4N probes
    // (N = 4 FP32, 2 FP64 per lane) whose two vector blocks of the largest
    // matrix fit one workgroup's LDS; used unless the caller fixes the block
    // width or asks for the streaming path.
    const bool force_stream = (o->flags & KPM_FLAG_BATCH_STREAM) != 0;
    const bool force_res = (o->flags & KPM_FLAG_BATCH_RESIDENT) != 0;
    if (force_stream && force_res)
        return kpm_fail(ctx, KPM_ERR_ARG, "KPM_FLAG_BATCH_STREAM and KPM_FLAG_BATCH_RESIDENT exclude each other");
    int rld = 0;
    if (!force_stream && (o->block == 0 || force_res)) {
        const size_t lds_max = lds_per_workgroup(ctx->device);
        if (!lds_max) return kpm_fail(ctx, KPM_ERR_HIP, "could not query the device's LDS size");
        const int N = o->precision == KPM_FP64 ? 2 : 4;
        for (int cand = 4 * N; cand >= N && !rld; cand /= 2) {
            if (o->block > 0 && cand < (o->block + N - 1) / N * N) break;
            if (o->block > 0 && cand / 2 >= (o->block + N - 1) / N * N && cand > N) continue;
            if (resident_lds_bytes((int)nmax, cand, esz) <= lds_max) rld = cand;
        }
        // a narrower block when the probes do not fill the chosen one
        while (rld > N && o->block == 0 && rld / 2 >= nvec) rld /= 2;
        if (force_res && !rld)
            return kpm_fail(ctx, KPM_ERR_UNSUPPORTED,
                            "the on-chip batched path needs two probe blocks of every matrix in one workgroup's LDS");
    }
    const bool resident = rld > 0;
    const int b = o->block > 0 ? std::min(o->block, nvec)
                               : (resident ? std::min(rld, nvec) : kpm_default_block(nvec, o->precision));
    const BlockGeom g = make_geom(nmax, b, o->precision, o->rows_per_block);
    if ((uint64_t)nmax * g.ld * esz >= (1ull << 32))
        return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "batched probe blocks must be smaller than 4 GiB");
    const int nvb = (nvec + b - 1) / b;
    if (!resident && (int64_t)nmat * nvb > 65535)
        return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "at most 65535 (matrix, probe block) pairs per batch");
    if ((int64_t)nmat * nvb > (1 << 26))
        return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "at most 2^26 (matrix, probe block) pairs per batch");

    BatchShape shape;
    for (int m = 0; m < nmat; ++m) {
        shape.ptrs.push_back((uintptr_t)D[m].rp);
        shape.ptrs.push_back((uintptr_t)D[m].ci);
        shape.ptrs.push_back((uintptr_t)D[m].val);
        shape.dims.push_back(D[m].n);
        shape.dims.push_back(D[m].nnz);
    }
    const int64_t tail[] = {nmat, M, nvec, b, o->precision, D[0].val_f64, g.rows_per_block, rld};
    shape.dims.insert(shape.dims.end(), tail, tail + 8);

    if (!ctx->batch) ctx->batch = new kpm_batch_state();
    kpm_batch_state& S = *ctx->batch;
    int pi = -1;
    for (int i = 0; i < 2; ++i)
        if (S.plan[i].mem && S.plan[i].shape == shape) pi = i;
    const bool reuse = pi >= 0;
    if (!reuse) pi = !S.plan[0].mem ? 0 : !S.plan[1].mem ? 1 : 1 - S.mru;  // an empty slot, else the older plan
    S.mru = pi;
    BatchPlan& P = S.plan[pi];
    BatchPlan& other = S.plan[1 - pi];
    if (!P.gstream) KPM_HIP(ctx, hipStreamCreateWithFlags(&P.gstream, hipStreamNonBlocking));
    // A new plan's device memory: when it does not fit beside the other
    // plan, that plan is released and the allocation tried once more.
    auto plan_malloc = [&](void** ptr, size_t bytes) -> bool {
        if (hipMalloc(ptr, bytes) == hipSuccess) return true;
        *ptr = nullptr;
        (void)hipGetLastError();
        if (!other.mem && !other.sell_mem) return false;
        hipStreamSynchronize(other.gstream ? other.gstream : ctx->stream);
        free_plan(other);
        if (hipMalloc(ptr, bytes) == hipSuccess) return true;
        *ptr = nullptr;
        (void)hipGetLastError();
        return false;
    };
    if (!reuse) {
        KPM_HIP(ctx, hipStreamSynchronize(P.gstream));
        free_plan(P);
        P.nmat = nmat;
        P.M = M;
        P.K = (M + 1) / 2;
        P.nvec = nvec;
        P.ld = g.ld;
        P.lpr = g.lpr;
        P.rpw = g.rpw;
        P.rows = g.rows_per_block;
        P.precision = o->precision;
        P.val_f64 = D[0].val_f64;
        P.nmv = nmat * nvb;
        P.resident = resident;
    }
    if (!reuse && resident) {
        P.ld = rld;
        P.lds_bytes = resident_lds_bytes((int)nmax, rld, esz);
        const void* fn = o->precision == KPM_FP64
                             ? (P.val_f64 ? resident_kernel_for<double, double>(rld) : resident_kernel_for<float, double>(rld))
                             : resident_kernel_for<float, float>(rld);
        if (!fn) return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "no on-chip kernel for this block width");
        KPM_HIP(ctx, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_bytes));
        // slices of the sliced layout: one per wavefront's rows (rows per
        // wavefront = 64 lanes / (block values per row / values per lane))
        const int N = o->precision == KPM_FP64 ? 2 : 4;
        P.sell_C = 64 / (rld / N);
        std::vector<int64_t> slice_base(nmat + 1, 0);
        P.max_nsl = 0;
        for (int m = 0; m < nmat; ++m) {
            const int nsl = (int)((D[m].n + P.sell_C - 1) / P.sell_C);
            slice_base[m + 1] = slice_base[m] + nsl;
            P.max_nsl = std::max(P.max_nsl, nsl);
        }
        const int64_t nslices = slice_base[nmat];
        const int C = P.sell_C;
        std::vector<int64_t> row_base(nmat + 1, 0);
        for (int m = 0; m < nmat; ++m) row_base[m + 1] = row_base[m] + D[m].n;
        // one device allocation: tables and outputs; the slots in a second
        // one once their count is known
        size_t off = 0;
        const size_t o_mvs = off;
        off += align256((size_t)P.nmv * sizeof(BatchMvDev));
        const size_t o_mats = off;
        off += align256((size_t)nmat * sizeof(SellMatDev));
        const size_t o_slw = off;
        off += align256((size_t)nslices * 4);
        const size_t o_slo = off;
        off += align256((size_t)nslices * 8);
        const size_t o_srow = off;
        off += align256((size_t)nslices * C * 4);
        const size_t o_len = off;
        off += align256((size_t)row_base[nmat] * 4);
        const size_t o_rb = off;
        off += align256((size_t)nmat * 8);
        const size_t o_bad = off;
        off += 256;
        const size_t o_zeta = off;
        off += align256((size_t)nmat * nvec * (M + 1) * 8);
        const size_t o_mu = off;
        off += align256((size_t)nmat * (M + 1) * 8);
        const size_t o_max = off;
        off += align256((size_t)nmat * 8);
        if (!plan_malloc(&P.mem, off)) {
            P.mem = nullptr;
            return kpm_fail(ctx, KPM_ERR_ALLOC, "hipMalloc for the batched plan failed");
        }
        P.mem_bytes = off;
        char* base = (char*)P.mem;
        P.d_mvs = (BatchMvDev*)(base + o_mvs);
        P.d_mats = (SellMatDev*)(base + o_mats);
        int32_t* d_slw = (int32_t*)(base + o_slw);
        int64_t* d_slo = (int64_t*)(base + o_slo);
        int32_t* d_srow = (int32_t*)(base + o_srow);
        int32_t* d_len = (int32_t*)(base + o_len);
        int64_t* d_rb = (int64_t*)(base + o_rb);
        P.d_bad = (int*)(base + o_bad);
        P.d_zeta = (double*)(base + o_zeta);
        P.d_mu = (double*)(base + o_mu);
        P.d_maxabs = (double*)(base + o_max);
        P.d_entries = nullptr;
        P.d_e0 = P.d_e1 = nullptr;
        P.d_partial = P.d_chunk = P.d_dots = nullptr;
        P.nentries = 0;
        std::vector<SellMatDev> hm(nmat);
        for (int m = 0; m < nmat; ++m) {
            hm[m].rp = D[m].rp;
            hm[m].ci = D[m].ci;
            hm[m].val = D[m].val;
            hm[m].sell = nullptr;
            hm[m].slw = d_slw + slice_base[m];
            hm[m].slo = d_slo + slice_base[m];
            hm[m].srow = d_srow + slice_base[m] * C;
            hm[m].n = D[m].n;
            hm[m].nsl = (int)(slice_base[m + 1] - slice_base[m]);
        }
        // row lengths to the host, in one copy
        KPM_HIP(ctx, hipMemcpyAsync(P.d_mats, hm.data(), hm.size() * sizeof(SellMatDev), hipMemcpyHostToDevice,
                                    P.gstream));
        KPM_HIP(ctx, hipMemcpyAsync(d_rb, row_base.data(), (size_t)nmat * 8, hipMemcpyHostToDevice, P.gstream));
        row_length_kernel<<<dim3((unsigned)((nmax + 255) / 256), nmat), 256, 0, P.gstream>>>(P.d_mats, d_rb, d_len);
        KPM_HIP(ctx, hipGetLastError());
        std::vector<int32_t> len(row_base[nmat]);
        KPM_HIP(ctx, hipMemcpyAsync(len.data(), d_len, len.size() * 4, hipMemcpyDeviceToHost, P.gstream));
        KPM_HIP(ctx, hipStreamSynchronize(P.gstream));
        // per matrix: rows by decreasing length (counting sort, ties by
        // index), slices of C, each slice's width = its first row's length
        std::vector<int32_t> srow((size_t)nslices * C, -1), w(nslices);
        std::vector<int64_t> so(nslices);
        std::vector<int32_t> cnt;
        int64_t slots = 0;
        for (int m = 0; m < nmat; ++m) {
            const int n = D[m].n;
            const int32_t* L = len.data() + row_base[m];
            int lmax = 0;
            for (int r = 0; r < n; ++r) lmax = std::max(lmax, L[r]);
            cnt.assign((size_t)lmax + 2, 0);
            for (int r = 0; r < n; ++r) ++cnt[(size_t)(lmax - L[r]) + 1];  // key lmax - len: longest first
            for (int v = 1; v <= lmax + 1; ++v) cnt[v] += cnt[v - 1];
            int32_t* out = srow.data() + slice_base[m] * C;
            for (int r = 0; r < n; ++r) out[cnt[(size_t)(lmax - L[r])]++] = r;
            for (int64_t sl = 0; sl < slice_base[m + 1] - slice_base[m]; ++sl) {
                const int64_t g = slice_base[m] + sl;
                w[g] = L[out[sl * C]];
                so[g] = slots;
                slots += (int64_t)((w[g] + 1) & ~1) * C;
            }
        }
        const size_t pair_bytes = P.val_f64 ? 16 : 8;
        if (!plan_malloc(&P.sell_mem, std::max<size_t>(256, (size_t)slots * pair_bytes))) {
            P.sell_mem = nullptr;
            return kpm_fail(ctx, KPM_ERR_ALLOC, "hipMalloc for the sliced matrices failed");
        }
        for (int m = 0; m < nmat; ++m) hm[m].sell = P.sell_mem;
        KPM_HIP(ctx, hipMemcpyAsync(d_slw, w.data(), (size_t)nslices * 4, hipMemcpyHostToDevice, P.gstream));
        KPM_HIP(ctx, hipMemcpyAsync(d_slo, so.data(), (size_t)nslices * 8, hipMemcpyHostToDevice, P.gstream));
        KPM_HIP(ctx, hipMemcpyAsync(d_srow, srow.data(), srow.size() * 4, hipMemcpyHostToDevice, P.gstream));
        KPM_HIP(ctx, hipMemcpyAsync(P.d_mats, hm.data(), hm.size() * sizeof(SellMatDev), hipMemcpyHostToDevice,
                                    P.gstream));
        P.mvs.assign(P.nmv, BatchMvDev());
        for (int m = 0; m < nmat; ++m)
            for (int vb = 0; vb < nvb; ++vb) {
                BatchMvDev& d = P.mvs[m * nvb + vb];
                d.rp = D[m].rp;
                d.ci = D[m].ci;
                d.val = D[m].val;
                d.X0 = d.X1 = nullptr;
                d.n = D[m].n;
                d.ncols = std::min(b, nvec - vb * b);
                d.mat = m;
                d.vec0 = vb * b;
            }
        KPM_HIP(ctx, hipStreamSynchronize(P.gstream));
    } else if (!reuse) {
        // work table: workgroups per mv proportional to its bytes of work,
        // and at least kMinEntriesPerMv (or one per panel) for every mv
        const int resident_wg = o->precision == KPM_FP64
                                    ? (P.val_f64 ? batched_resident<double, double>() : batched_resident<float, double>())
                                    : batched_resident<float, float>();
        const int target = std::max(resident_wg, 256);
        std::vector<double> work(P.nmv);
        double wsum = 0.0;
        for (int m = 0; m < nmat; ++m)
            for (int vb = 0; vb < nvb; ++vb) {
                const double w = (double)(esz + 4) * D[m].nnz + 3.0 * esz * D[m].n * g.ld;
                work[m * nvb + vb] = w;
                wsum += w;
            }
        // Workgroup b runs entry xcd_panel(b, nentries): XCD x runs the x-th
        // contiguous run of entries.  The entries of one mv that fall on one
        // XCD share a contiguous panel range (its share in proportion) and
        // stride through it.
        int64_t total_entries = 0;
        std::vector<int> gws(P.nmv);
        const int minw = P.nmv > target ? kMinEntriesPerMv : 1;
        for (int m = 0; m < nmat; ++m)
            for (int vb = 0; vb < nvb; ++vb) {
                const int mv = m * nvb + vb;
                const int panels = (int)((D[m].n + P.rows - 1) / P.rows);
                const int gw = (int)std::lround(target * work[mv] / wsum);
                gws[mv] = std::max(std::min(panels, minw), std::min(gw, panels));
                total_entries += gws[mv];
            }
        const int nb = (int)total_entries;
        auto xcd_of = [&](int e) {  // XCD that runs entry e (inverse of xcd_panel)
            if (nb < 8) return e;
            const int q = nb / 8, r = nb % 8;
            int x = 0;
            while (x < 7 && e >= (x + 1) * q + std::min(x + 1, r)) ++x;
            return x;
        };
        std::vector<BatchEntryDev> entries;
        std::vector<int32_t> e0(P.nmv), e1(P.nmv);
        for (int m = 0; m < nmat; ++m)
            for (int vb = 0; vb < nvb; ++vb) {
                const int mv = m * nvb + vb;
                const int panels = (int)((D[m].n + P.rows - 1) / P.rows);
                const int gw = gws[mv];
                const int a0 = (int)entries.size();
                e0[mv] = a0;
                int i = 0;
                while (i < gw) {  // runs of consecutive entries on one XCD
                    int j = i + 1;
                    while (j < gw && xcd_of(a0 + j) == xcd_of(a0 + i)) ++j;
                    const int P0 = (int)((int64_t)panels * i / gw), P1 = (int)((int64_t)panels * j / gw);
                    for (int u = i; u < j; ++u) {
                        BatchEntryDev e = {};
                        e.mv = mv;
                        e.first = P0 + (u - i);
                        e.end = P1;
                        e.stride = j - i;
                        e.base = P0;
                        entries.push_back(e);
                    }
                    i = j;
                }
                e1[mv] = (int32_t)entries.size();
            }
        P.nentries = (int)entries.size();
        // one device allocation: vectors, tables, partials, outputs
        size_t off = 0;
        std::vector<size_t> xoff(P.nmv);
        for (int mv = 0; mv < P.nmv; ++mv) {
            xoff[mv] = off;
            off += 2 * align256((size_t)D[mv / nvb].n * g.ld * esz);
        }
        const size_t o_entries = off;
        off += align256(entries.size() * sizeof(BatchEntryDev));
        const size_t o_mvs = off;
        off += align256((size_t)P.nmv * sizeof(BatchMvDev));
        const size_t o_e0 = off;
        off += align256((size_t)P.nmv * 4);
        const size_t o_e1 = off;
        off += align256((size_t)P.nmv * 4);
        const size_t o_part = off;
        off += align256((size_t)std::min(std::max(P.K, 1), 2) * P.nentries * 2 * g.ld * 8);
        const size_t o_chunk = off;
        off += align256((size_t)2 * P.nentries * 2 * g.ld * 8);
        const size_t o_dots = off;
        off += align256((size_t)std::max(P.K, 1) * P.nmv * 2 * g.ld * 8);
        const size_t o_zeta = off;
        off += align256((size_t)nmat * nvec * (M + 1) * 8);
        const size_t o_mu = off;
        off += align256((size_t)nmat * (M + 1) * 8);
        const size_t o_max = off;
        off += align256((size_t)nmat * 8);
        if (!plan_malloc(&P.mem, off)) {
            P.mem = nullptr;
            return kpm_fail(ctx, KPM_ERR_ALLOC, "hipMalloc for the batched plan failed");
        }
        P.mem_bytes = off;
        char* base = (char*)P.mem;
        P.d_entries = (BatchEntryDev*)(base + o_entries);
        P.d_mvs = (BatchMvDev*)(base + o_mvs);
        P.d_e0 = (int32_t*)(base + o_e0);
        P.d_e1 = (int32_t*)(base + o_e1);
        P.d_partial = (double*)(base + o_part);
        P.d_chunk = (double*)(base + o_chunk);
        P.d_dots = (double*)(base + o_dots);
        P.d_zeta = (double*)(base + o_zeta);
        P.d_mu = (double*)(base + o_mu);
        P.d_maxabs = (double*)(base + o_max);
        P.mvs.assign(P.nmv, BatchMvDev());
        for (int m = 0; m < nmat; ++m)
            for (int vb = 0; vb < nvb; ++vb) {
                BatchMvDev& d = P.mvs[m * nvb + vb];
                d.rp = D[m].rp;
                d.ci = D[m].ci;
                d.val = D[m].val;
                d.X0 = base + xoff[m * nvb + vb];
                d.X1 = d.X0 + align256((size_t)D[m].n * g.ld * esz);
                d.n = D[m].n;
                d.ncols = std::min(b, nvec - vb * b);
                d.mat = m;
                d.vec0 = vb * b;
            }
        KPM_HIP(ctx, hipMemcpyAsync(P.d_entries, entries.data(), entries.size() * sizeof(BatchEntryDev),
                                    hipMemcpyHostToDevice, P.gstream));
        KPM_HIP(ctx, hipMemcpyAsync(P.d_e0, e0.data(), (size_t)P.nmv * 4, hipMemcpyHostToDevice, P.gstream));
        KPM_HIP(ctx, hipMemcpyAsync(P.d_e1, e1.data(), (size_t)P.nmv * 4, hipMemcpyHostToDevice, P.gstream));
        KPM_HIP(ctx, hipStreamSynchronize(P.gstream));
    }
    // the plan is complete: later calls of the same shape reuse it (a build
    // that failed part way left the shape empty, so it is rebuilt)
    if (!reuse) P.shape = shape;
    // per-call scalars
    for (int m = 0; m < nmat; ++m) {
        const double c = 0.5 * (lb[m] + ub[m]), d = 0.5 * (ub[m] - lb[m]);
        for (int vb = 0; vb < nvb; ++vb) {
            BatchMvDev& x = P.mvs[m * nvb + vb];
            x.alpha = 2.0 / d;
            x.beta = -2.0 * c / d;
            x.seed = seeds ? seeds[m] : o->seed + (uint64_t)m;
        }
    }
    // order after the caller's stream (the matrices may have been written there)
    hipEvent_t ev;
    KPM_HIP(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipEventRecord(ev, ctx->stream);
    hipStreamWaitEvent(P.gstream, ev, 0);
    hipEventDestroy(ev);
    KPM_HIP(ctx, hipMemcpyAsync(P.d_mvs, P.mvs.data(), P.mvs.size() * sizeof(BatchMvDev), hipMemcpyHostToDevice,
                                P.gstream));
    const bool use_graph = (o->flags & KPM_FLAG_NO_GRAPH) == 0;
    kpm_prof_begin_on(ctx, "batched", P.gstream);
    if (use_graph) {
        if (!P.exec) {
            if (P.graph) {  // left by an instantiation that failed
                hipGraphDestroy(P.graph);
                P.graph = nullptr;
            }
            KPM_HIP(ctx, hipStreamBeginCapture(P.gstream, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_plan(P.gstream, P);
            hipGraph_t gr = nullptr;
            hipError_t e2 = hipStreamEndCapture(P.gstream, &gr);
            if (e != hipSuccess) return kpm_hip_fail(ctx, e, "batched launch sequence (capture)");
            if (e2 != hipSuccess) return kpm_hip_fail(ctx, e2, "hipStreamEndCapture");
            P.graph = gr;
            KPM_HIP(ctx, hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0));
        }
        KPM_HIP(ctx, hipGraphLaunch(P.exec, P.gstream));
    } else {
        KPM_HIP(ctx, enqueue_plan(P.gstream, P));
    }
    kpm_prof_end_on(ctx, "batched", P.gstream, 1);
    std::vector<double> maxabs(nmat);
    int bad = 0;
    KPM_HIP(ctx, hipMemcpyAsync(mu, P.d_mu, (size_t)nmat * (M + 1) * 8, hipMemcpyDeviceToHost, P.gstream));
    KPM_HIP(ctx, hipMemcpyAsync(maxabs.data(), P.d_maxabs, (size_t)nmat * 8, hipMemcpyDeviceToHost, P.gstream));
    if (P.resident) KPM_HIP(ctx, hipMemcpyAsync(&bad, P.d_bad, 4, hipMemcpyDeviceToHost, P.gstream));
    KPM_HIP(ctx, hipStreamSynchronize(P.gstream));
    if (bad) {
        free_plan(P);  // rebuilt from the current structure on the next call
        return kpm_fail(ctx, KPM_ERR_ARG,
                        "a matrix's sparsity structure changed since its batched plan was built (same addresses and "
                        "sizes): call again to rebuild the plan");
    }
    kpm_prof_collect(ctx);
    if (max_abs_mu) memcpy(max_abs_mu, maxabs.data(), (size_t)nmat * 8);
    const double tol = o->precision == KPM_FP64 ? 1e-9 : 1e-4;
    for (int m = 0; m < nmat; ++m)
        if (!(maxabs[m] <= 1.0 + tol)) {
            char msg[160];
            snprintf(msg, sizeof msg, "spectrum of matrix %d escaped [lb, ub]: max |mu_k| over probes = %g", m,
                     maxabs[m]);
            return kpm_fail(ctx, KPM_ERR_SPECTRUM, msg);
        }
    return KPM_OK;
}

extern "C" kpm_status kpm_moments_batched(kpm_ctx* ctx, int nmat, const kpm_csr* A, const double* lb,
                                          const double* ub, const kpm_moment_opts* o, double* mu,
                                          double* max_abs_mu) {
    return kpm_moments_batched_seeded(ctx, nmat, A, lb, ub, o, nullptr, mu, max_abs_mu);
}

// ---------------------------------------------------------------- autotuner
// Times kpm_moments_batched for candidate (probe-block width, row-panel
// height) pairs: per candidate one call to build and capture the plan, then
// two calls each of degree 15 and 47 (8 and 24 steps); the difference of the
// faster device times over the 16 extra steps is the time per step, free of
// the fixed costs.
extern "C" kpm_status kpm_autotune_batched(kpm_ctx* ctx, int nmat, const kpm_csr* A, const double* lb,
                                           const double* ub, const kpm_moment_opts* o, kpm_moment_opts* best,
                                           double* us_per_step) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!o || !best || nmat < 1 || !A) return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (o->precision != KPM_FP32 && o->precision != KPM_FP64)
        return kpm_fail(ctx, KPM_ERR_ARG, "precision must be KPM_FP32 or KPM_FP64");
    const int maxb = o->precision == KPM_FP64 ? 128 : 256;
    if (o->nvec < 1 || o->block < 0 || o->block > maxb || o->rows_per_block < 0 || o->rows_per_block > (1 << 20))
        return kpm_fail(ctx, KPM_ERR_ARG, "nvec, block or rows_per_block out of range");
    int64_t nmax = 0;
    for (int m = 0; m < nmat; ++m) nmax = std::max<int64_t>(nmax, A[m].n);
    std::vector<int> blocks;
    if (o->block > 0) {
        blocks.push_back(std::min(o->block, o->nvec));
    } else {
        const int c32[] = {16, 32, 64}, c64[] = {8, 16, 32};
        for (int c : (o->precision == KPM_FP64 ? c64 : c32))
            if (c <= o->nvec) blocks.push_back(c);
        if (blocks.empty()) blocks.push_back(o->nvec);
    }
    std::vector<double> mu;
    // device time of one call, from the event pair the call records around
    // its launch sequence when profiling is on
    const bool prof_was = ctx->prof;
    ctx->prof = true;
    auto timed = [&](kpm_moment_opts t, int M, double* sec) -> kpm_status {
        t.M = M;
        mu.resize((size_t)nmat * (M + 1));
        kpm_prof_entry& pe = ctx->prof_map["batched"];
        const double before = pe.total_ms;
        const kpm_status r = kpm_moments_batched(ctx, nmat, A, lb, ub, &t, mu.data(), nullptr);
        *sec = (ctx->prof_map["batched"].total_ms - before) * 1e-3;
        return r == KPM_ERR_SPECTRUM ? KPM_OK : r;  // values do not matter here
    };
    double best_t = 1e300;
    kpm_moment_opts bo = *o;
    for (int b : blocks) {
        const int r0 = make_geom(nmax, b, o->precision, o->rows_per_block).rows_per_block;
        std::vector<int> rows;
        if (o->rows_per_block > 0) rows.push_back(r0);
        else rows = {std::max(1, r0 / 2), r0, 2 * r0};
        for (int r : rows) {
            kpm_moment_opts t = *o;
            t.block = b;
            t.rows_per_block = r;
            t.validate = 0;
            double s0, s1, s2, s3, s4;
            kpm_status st = timed(t, 47, &s0);  // plan and graph for this shape
            if (st == KPM_OK) st = timed(t, 15, &s1);
            if (st == KPM_OK) st = timed(t, 47, &s2);
            if (st == KPM_OK) st = timed(t, 15, &s3);
            if (st == KPM_OK) st = timed(t, 47, &s4);
            if (st != KPM_OK) {
                ctx->prof = prof_was;
                return st;
            }
            (void)s0;
            const double per_step = std::max(1e-12, (std::min(s2, s4) - std::min(s1, s3)) / 16.0) / b;
            if (per_step < best_t) {
                best_t = per_step;
                bo.block = b;
                bo.rows_per_block = make_geom(nmax, b, o->precision, r).rows_per_block;
            }
        }
    }
    ctx->prof = prof_was;
    *best = bo;
    if (us_per_step) *us_per_step = best_t * 1e6 * o->nvec;
    return KPM_OK;
}
