// Device code shared by the single-matrix and the batched step kernels:
// probe signs, the XCD-aware workgroup map, vector packs, and the fused
// per-row / per-panel Chebyshev step (Lin, Saad & Yang, eq. (3term) with
// the product identity of Appendix A; the Legendre recurrence of Algorithm
// DGL as a variant).  Included by .hip sources only.
#pragma once

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
    __device__ static __forceinline__ void load_nt(const float* p, float (&v)[4]) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 t = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p));
        v[0] = t[0]; v[1] = t[1]; v[2] = t[2]; v[3] = t[3];
    }
    __device__ static __forceinline__ void store(float* p, const float (&v)[4]) {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    }
    __device__ static __forceinline__ void store_nt(float* p, const float (&v)[4]) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        f4 t = {v[0], v[1], v[2], v[3]};
        __builtin_nontemporal_store(t, reinterpret_cast<f4*>(p));
    }
};
template <>
struct Pack<double> {
    static constexpr int N = 2;
    __device__ static __forceinline__ void load(const double* p, double (&v)[2]) {
        const double2 t = *reinterpret_cast<const double2*>(p);
        v[0] = t.x; v[1] = t.y;
    }
    __device__ static __forceinline__ void load_nt(const double* p, double (&v)[2]) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 t = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
        v[0] = t[0]; v[1] = t[1];
    }
    __device__ static __forceinline__ void store(double* p, const double (&v)[2]) {
        *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    }
    __device__ static __forceinline__ void store_nt(double* p, const double (&v)[2]) {
        typedef double d2 __attribute__((ext_vector_type(2)));
        d2 t = {v[0], v[1]};
        __builtin_nontemporal_store(t, reinterpret_cast<d2*>(p));
    }
};

// Byte offset of element (row, column group) in a vector block.  With
// OFF32 the block is known to be smaller than 4 GiB and the offset is an
// unsigned 32-bit value added to a uniform base (one address register per
// load instead of two).
template <bool OFF32>
__device__ __forceinline__ uint64_t voff(uint32_t row, uint32_t ldb, uint32_t coffb) {
    if (OFF32) return (uint32_t)(row * ldb + coffb);
    return (uint64_t)row * ldb + coffb;
}

// Readers of a row's CSR entries (column index, value) at position k:
// the two global arrays, or the panel's (index, value) pairs staged in LDS
// (one 8- or 16-byte LDS read per entry).
template <typename TA>
struct CsrArrays {
    const int32_t* __restrict__ ci;
    const TA* __restrict__ val;
    __device__ __forceinline__ void get(int k, int& j, TA& a) const {
        j = ci[k];
        a = val[k];
    }
};
template <typename TA>
struct CsrPair;
template <>
struct CsrPair<float> {
    int32_t c;
    float v;
};
template <>
struct __align__(16) CsrPair<double> {
    double v;
    int32_t c, pad;
};
template <typename TA>
struct CsrPairs {
    const CsrPair<TA>* e;
    __device__ __forceinline__ void get(int k, int& j, TA& a) const {
        const CsrPair<TA> t = e[k];
        j = t.c;
        a = t.v;
    }
};

// Extra arguments of the Legendre step (Algorithm DGL's recurrence
// v_{k+1} = alpha A v_k + beta v_k + gam v_{k-1}): the coefficient of
// v_{k-1} and the sign bits of the probe block v_0 ([n][sw] 32-bit words,
// bit j of word w set when column 32 w + j of the row is -1), against which
// the moment v_0^T v_{k+1} is accumulated.
struct LegArgs {
    const uint32_t* __restrict__ sgn;
    int sw, sword, sshift;
    double gam;
};

// One matrix row of the fused step for the lanes of one row group: gather
// the CSR row in batches of G entries (one memory round trip for rows of up
// to G entries), combine, store, and accumulate the two dot products.
//
// A batch first reads its G (index, value) pairs, then issues its G gathers
// back to back; slots past the end of the row take value 0 and gather the
// row's own entry (already being loaded, so it costs no extra DRAM traffic),
// which keeps the loads unconditional instead of behind one branch and one
// index wait each.
//
// With `ntu` set the U row (read once here, then overwritten) is loaded
// non-temporally: for probe blocks larger than the 256 MB MALL this leaves
// the cache to the gathered rows (large workload: 3 % faster; on a 67 MB
// block it cost 25 %, so the caller sets it by block size).
//
// EARLY (indices in LDS): the own-row and U loads go out first and overlap
// the gathers.  Without staging the index loads share the in-order vector
// memory counter with them, so the own-row and U loads are issued after the
// gathers instead.
//
// LEG (not FIRST): the Legendre step; the first dot is then taken against
// v_0 (from its sign bits) instead of v_k.
template <typename TA, typename TV, bool FIRST, bool EARLY, bool OFF32, int G, typename E, bool LEG = false>
__device__ __forceinline__ void step_row(int row, int kb, int ke, const E& csr, const char* __restrict__ Vb,
                                         char* __restrict__ Ub, uint32_t ldb, uint32_t coffb,
                                         double alpha, double beta, double (&sx)[Pack<TV>::N],
                                         double (&ss)[Pack<TV>::N], const LegArgs* leg = nullptr,
                                         int ntu = 0) {
    constexpr int N = Pack<TV>::N;
    const uint64_t orow = voff<OFF32>(row, ldb, coffb);
    TV own[N], u[N];
    uint32_t bits = 0;
    if (EARLY) {
        Pack<TV>::load(reinterpret_cast<const TV*>(Vb + orow), own);
        if (!FIRST) {
            if (ntu)
                Pack<TV>::load_nt(reinterpret_cast<const TV*>(Ub + orow), u);
            else
                Pack<TV>::load(reinterpret_cast<const TV*>(Ub + orow), u);
        }
        if (LEG) bits = leg->sgn[(int64_t)row * leg->sw + leg->sword] >> leg->sshift;
    }
    TV acc[N];
#pragma unroll
    for (int e = 0; e < N; ++e) acc[e] = (TV)0;
    for (int k = kb; k < ke; k += G) {
        int j[G];
        TV a[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const bool on = k + i < ke;
            const int ks = on ? k + i : k;  // k < ke: always a valid entry
            int jj;
            TA vv;
            csr.get(ks, jj, vv);
            j[i] = on ? jj : row;
            a[i] = on ? (TV)vv : (TV)0;
        }
        TV x[G][N];
#pragma unroll
        for (int i = 0; i < G; ++i)
            Pack<TV>::load(reinterpret_cast<const TV*>(Vb + voff<OFF32>(j[i], ldb, coffb)), x[i]);
#pragma unroll
        for (int i = 0; i < G; ++i)
#pragma unroll
            for (int e = 0; e < N; ++e) acc[e] = fma(a[i], x[i][e], acc[e]);
    }
    if (!EARLY) {
        Pack<TV>::load(reinterpret_cast<const TV*>(Vb + orow), own);
        if (!FIRST) Pack<TV>::load(reinterpret_cast<const TV*>(Ub + orow), u);
        if (LEG) bits = leg->sgn[(int64_t)row * leg->sw + leg->sword] >> leg->sshift;
    }
    TV out[N];
    if (FIRST) {
        // v1 = B v0 = (alpha/2) A v0 + (beta/2) v0
#pragma unroll
        for (int e = 0; e < N; ++e)
            out[e] = (TV)fma(0.5 * alpha, (double)acc[e], 0.5 * beta * (double)own[e]);
    } else if (LEG) {
#pragma unroll
        for (int e = 0; e < N; ++e)
            out[e] = (TV)fma(alpha, (double)acc[e], fma(beta, (double)own[e], leg->gam * (double)u[e]));
    } else {
#pragma unroll
        for (int e = 0; e < N; ++e)
            out[e] = (TV)fma(alpha, (double)acc[e], fma(beta, (double)own[e], -(double)u[e]));
    }
    // U_new is not read again in this step: a non-temporal store leaves the
    // L2 to the gathered V rows (measured faster than a cached store).
    Pack<TV>::store_nt(reinterpret_cast<TV*>(Ub + orow), out);
#pragma unroll
    for (int e = 0; e < N; ++e) {
        const double o = (double)out[e];
        if (LEG)
            sx[e] += ((bits >> e) & 1u) ? -o : o;
        else
            sx[e] = fma(o, (double)own[e], sx[e]);
        ss[e] = fma(o, o, ss[e]);
    }
}

// One row panel [r0, r1) of the fused step for one workgroup.  With `stage`
// set and when it fits, the panel's slice of the CSR arrays (row offsets,
// and the column indices and values as interleaved pairs) is first copied
// to LDS with coalesced loads, so each row costs one round of independent
// gathers.  The dots are added to the caller's per-lane accumulators sx/ss.
template <typename TA, typename TV, bool FIRST, bool OFF32, int G, int LDS_DOUBLES, bool LEG = false>
__device__ __forceinline__ void process_panel(int r0, int r1, const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ ci, const TA* __restrict__ val,
                                              const char* __restrict__ Vb, char* __restrict__ Ub, uint32_t ldb,
                                              uint32_t coffb, double alpha, double beta, int stage,
                                              double (&smem)[LDS_DOUBLES], bool lane_on, int wave, int rw,
                                              int rpw, double (&sx)[Pack<TV>::N],
                                              double (&ss)[Pack<TV>::N], const LegArgs* leg = nullptr,
                                              int ntu = 0) {
    const int pass_rows = kWaves * rpw;
    // Staging layout in LDS: [row offsets (R+1) x 4 bytes, padded to 16]
    // [(index, value) pairs pnnz x sizeof(CsrPair<TA>)].
    const int R = r1 - r0;
    const int kbase = rp[r0];
    const int pnnz = rp[r1] - kbase;
    const int off_e = ((R + 1) * 4 + 15) & ~15;
    const bool staged = stage && off_e + pnnz * (int)sizeof(CsrPair<TA>) <= (int)sizeof(smem);
    if (staged) {
        char* base = reinterpret_cast<char*>(smem);
        int32_t* s_rp = reinterpret_cast<int32_t*>(base);
        CsrPair<TA>* s_e = reinterpret_cast<CsrPair<TA>*>(base + off_e);
        for (int t = threadIdx.x; t <= R; t += kThreads) s_rp[t] = rp[r0 + t] - kbase;
        for (int t = threadIdx.x; t < pnnz; t += kThreads) {
            s_e[t].c = ci[kbase + t];
            s_e[t].v = val[kbase + t];
        }
        __syncthreads();
        if (lane_on) {
            const CsrPairs<TA> csr{s_e};
            for (int row = r0 + wave * rpw + rw; row < r1; row += pass_rows) {
                const int lr = row - r0;
                step_row<TA, TV, FIRST, true, OFF32, G, CsrPairs<TA>, LEG>(row, s_rp[lr], s_rp[lr + 1], csr, Vb, Ub,
                                                                           ldb, coffb, alpha, beta, sx, ss, leg, ntu);
            }
        }
        __syncthreads();  // before the LDS is restaged or reused
    } else if (lane_on) {
        const CsrArrays<TA> csr{ci, val};
        for (int row = r0 + wave * rpw + rw; row < r1; row += pass_rows)
            step_row<TA, TV, FIRST, false, OFF32, G, CsrArrays<TA>, LEG>(row, rp[row], rp[row + 1], csr, Vb, Ub,
                                                                         ldb, coffb, alpha, beta, sx, ss, leg);
    }
}

}  // namespace kpm
