// Locality renumbering of structured-grid matrices for the single-matrix
// moment path (KPM_FLAG_LOCALITY).
//
// A matrix from a d-dimensional grid numbered lexicographically (x fastest)
// has its off-diagonal entries on a few dominant column offsets, 1, nx and
// nx * ny.  With that numbering the neighbours one plane apart (nx * ny rows
// later) are far in the probe block: on a 128^3 grid with 64 FP32 probes a
// plane is 4 MB, the size of an XCD's L2, so every plane-apart gather
// misses it.  Renumbering the rows along a Morton (Z-order) curve of the
// grid coordinates keeps all neighbours of a row within a small block of
// rows.  The moments do not depend on the numbering: with P the
// permutation, v^T T_k(A) v = (P v)^T T_k(P A P^T) (P v), and the probes of
// the renumbered matrix are generated at the original row indices, so the
// same probes enter and the per-probe moments agree up to rounding.
//
// kpm_locality_order finds the grid from the offsets of the entries (the
// two or three offsets that each occur in at least 40 % of the rows, the
// smallest being 1) and returns the permutation; random long-range entries
// have offsets that repeat rarely and do not disturb it.  The context caches
// the renumbered structure per matrix (row offsets, columns, the source
// index of each entry, the original index of each row) and gathers the
// values at every call, so values may change between calls; the structure
// at a given address may not.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <unordered_map>
#include <vector>

#include "kpm_internal.h"

using namespace kpm;

namespace {

// Interleave the bits of x, y, z (z most significant of each triple).
uint64_t morton3(uint64_t x, uint64_t y, uint64_t z) {
    uint64_t key = 0;
    for (int b = 0; b < 21; ++b)
        key |= ((x >> b) & 1ull) << (3 * b) | ((y >> b) & 1ull) << (3 * b + 1) | ((z >> b) & 1ull) << (3 * b + 2);
    return key;
}

// Order-free checksum of a CSR structure (row offsets and columns): a
// wrapping sum of SplitMix64-finalised (index, entry) words, the same on
// the host and the device.
__host__ __device__ inline uint64_t structure_word(uint64_t tag, uint64_t idx, uint32_t v) {
    uint64_t z = tag + ((idx << 32) ^ (uint64_t)v) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
constexpr uint64_t kTagRp = 0x1, kTagCi = 0x2;

uint64_t structure_sum_host(const int32_t* rp, int64_t n, const int32_t* ci, int64_t nnz) {
    uint64_t s = 0;
    for (int64_t i = 0; i <= n; ++i) s += structure_word(kTagRp, (uint64_t)i, (uint32_t)rp[i]);
    for (int64_t k = 0; k < nnz; ++k) s += structure_word(kTagCi, (uint64_t)k, (uint32_t)ci[k]);
    return s;
}

__global__ void clear_sum_kernel(unsigned long long* out) { out[0] = 0ull; }

__global__ __launch_bounds__(256) void structure_sum_kernel(const int32_t* __restrict__ rp, int64_t n,
                                                            const int32_t* __restrict__ ci, int64_t nnz,
                                                            unsigned long long* out) {
    __shared__ unsigned long long sh[256];
    uint64_t s = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride)
        s += structure_word(kTagRp, (uint64_t)i, (uint32_t)rp[i]);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride)
        s += structure_word(kTagCi, (uint64_t)k, (uint32_t)ci[k]);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, sh[0]);
}

template <typename T>
__global__ void gather_values_kernel(const T* __restrict__ src_val, const int32_t* __restrict__ src,
                                     int64_t nnz, T* __restrict__ out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = src_val[src[k]];
}

}  // namespace

extern "C" kpm_status kpm_locality_order(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                                         int32_t* perm, int32_t* dims) {
    if (n < 1 || n >= ((int64_t)1 << 31) || nnz < 0 || !row_ptr || (nnz > 0 && !col_idx) || !perm || !dims)
        return KPM_ERR_ARG;
    if (row_ptr[0] != 0 || row_ptr[n] != nnz) return KPM_ERR_ARG;
    dims[0] = dims[1] = dims[2] = 0;
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    // offsets of the entries above the diagonal, over a sample of at most
    // 2^18 evenly spaced rows
    const int64_t step = std::max<int64_t>(1, n >> 18);
    std::unordered_map<int64_t, int64_t> count;
    int64_t rows = 0;
    for (int64_t i = 0; i < n; i += step, ++rows) {
        const int32_t kb = row_ptr[i], ke = row_ptr[i + 1];
        if (kb > ke || kb < 0 || ke > nnz) return KPM_ERR_ARG;
        for (int32_t k = kb; k < ke; ++k)
            if (col_idx[k] > i) ++count[col_idx[k] - i];
    }
    std::vector<int64_t> off;
    for (const auto& kv : count)
        if (kv.second * 5 >= rows * 2) off.push_back(kv.first);
    std::sort(off.begin(), off.end());
    int64_t nx = 0, ny = 1, nz = 1;
    if (off.size() == 2 && off[0] == 1 && n % off[1] == 0) {
        nx = off[1];
        ny = n / nx;
    } else if (off.size() == 3 && off[0] == 1 && off[2] % off[1] == 0 && n % off[2] == 0) {
        nx = off[1];
        ny = off[2] / off[1];
        nz = n / off[2];
    } else {
        return KPM_OK;  // no grid found: the identity
    }
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
        key[(size_t)i] = {morton3((uint64_t)x, (uint64_t)y, (uint64_t)z), (int32_t)i};
    }
    std::sort(key.begin(), key.end());
    for (int64_t r = 0; r < n; ++r) perm[r] = key[(size_t)r].second;
    dims[0] = (int32_t)nx;
    dims[1] = (int32_t)ny;
    dims[2] = (int32_t)nz;
    return KPM_OK;
}

struct kpm_locality_state {
    const int32_t* rp = nullptr;  // the matrix the plan belongs to
    const int32_t* ci = nullptr;
    int64_t n = 0, nnz = 0;
    bool val_f64 = false;  // the values' type the value buffer is sized for
    bool structured = false;
    uint64_t sum = 0;     // structure checksum when the plan was built
    void* mem = nullptr;  // rp2 | ci2 | src | orig | val2 | sum
    int32_t *rp2 = nullptr, *ci2 = nullptr, *src = nullptr, *orig = nullptr;
    void* val2 = nullptr;
    unsigned long long* d_sum = nullptr;  // checksum of the current call's structure
    unsigned long long* h_sum = nullptr;  // its copy in page-locked host memory
    bool check_pending = false;
};

void kpm_locality_free(kpm_ctx* ctx) {
    if (!ctx->loc) return;
    if (ctx->loc->mem || ctx->loc->h_sum) hipStreamSynchronize(ctx->stream);  // a pending copy may target h_sum
    if (ctx->loc->mem) hipFree(ctx->loc->mem);
    if (ctx->loc->h_sum) hipHostFree(ctx->loc->h_sum);
    delete ctx->loc;
    ctx->loc = nullptr;
}

kpm_status kpm_locality_view(kpm_ctx* ctx, const CsrDev& A, CsrDev* out, const int32_t** orig, bool refresh) {
    *out = A;
    *orig = nullptr;
    kpm_locality_state*& L = ctx->loc;
    if (!L || L->rp != A.rp || L->ci != A.ci || L->n != A.n || L->nnz != A.nnz || L->val_f64 != A.val_f64) {
        KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
        kpm_locality_free(ctx);
        L = new kpm_locality_state();
        L->rp = A.rp;
        L->ci = A.ci;
        L->n = -1;  // matches no matrix until the build below has completed
        L->nnz = A.nnz;
        L->val_f64 = A.val_f64;
        std::vector<int32_t> rp((size_t)A.n + 1), ci((size_t)A.nnz), perm((size_t)A.n);
        KPM_HIP(ctx, hipMemcpyAsync(rp.data(), A.rp, rp.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
        if (A.nnz > 0) KPM_HIP(ctx, hipMemcpyAsync(ci.data(), A.ci, ci.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
        KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
        // the whole structure is read on the host below: check it first
        bool ok = rp[0] == 0 && rp[(size_t)A.n] == A.nnz;
        for (int64_t i = 0; ok && i < A.n; ++i) ok = rp[(size_t)i] <= rp[(size_t)i + 1];
        for (int64_t k = 0; ok && k < A.nnz; ++k) ok = ci[(size_t)k] >= 0 && ci[(size_t)k] < A.n;
        int32_t dims[3];
        const kpm_status st = ok ? kpm_locality_order(A.n, A.nnz, rp.data(), ci.data(), perm.data(), dims)
                                 : KPM_ERR_ARG;
        if (st != KPM_OK) {
            kpm_locality_free(ctx);
            return kpm_fail(ctx, st, "locality renumbering: malformed CSR (row offsets or column indices)");
        }
        L->structured = dims[0] > 0;
        if (!L->structured) {
            L->n = A.n;
            return KPM_OK;
        }
        L->sum = structure_sum_host(rp.data(), A.n, ci.data(), A.nnz);
        // the renumbered structure: row r is row perm[r] of A, its columns
        // renumbered and sorted, src[k] the entry of A it came from
        std::vector<int32_t> inv((size_t)A.n), rp2((size_t)A.n + 1), ci2((size_t)A.nnz), src((size_t)A.nnz);
        for (int64_t r = 0; r < A.n; ++r) inv[(size_t)perm[(size_t)r]] = (int32_t)r;
        std::vector<std::pair<int32_t, int32_t>> row;
        rp2[0] = 0;
        for (int64_t r = 0; r < A.n; ++r) {
            const int32_t o = perm[(size_t)r];
            row.clear();
            for (int32_t k = rp[(size_t)o]; k < rp[(size_t)o + 1]; ++k) row.push_back({inv[(size_t)ci[(size_t)k]], k});
            std::sort(row.begin(), row.end());
            int32_t at = rp2[(size_t)r];
            for (const auto& e : row) {
                ci2[(size_t)at] = e.first;
                src[(size_t)at] = e.second;
                ++at;
            }
            rp2[(size_t)r + 1] = at;
        }
        const size_t vsz = A.val_f64 ? 8 : 4;
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        const size_t b_rp = al((size_t)(A.n + 1) * 4), b_ci = al((size_t)A.nnz * 4 + 4), b_or = al((size_t)A.n * 4);
        const size_t b_val = al((size_t)A.nnz * vsz + vsz);
        const size_t total = b_rp + 2 * b_ci + b_or + b_val + 256;
        if (hipMalloc(&L->mem, total) != hipSuccess) {
            L->mem = nullptr;
            kpm_locality_free(ctx);
            return kpm_fail(ctx, KPM_ERR_ALLOC, "hipMalloc for the renumbered matrix failed");
        }
        if (hipHostMalloc((void**)&L->h_sum, sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
            L->h_sum = nullptr;
            kpm_locality_free(ctx);
            return kpm_fail(ctx, KPM_ERR_ALLOC, "hipHostMalloc for the structure checksum failed");
        }
        char* p = static_cast<char*>(L->mem);
        L->rp2 = reinterpret_cast<int32_t*>(p);
        L->ci2 = reinterpret_cast<int32_t*>(p + b_rp);
        L->src = reinterpret_cast<int32_t*>(p + b_rp + b_ci);
        L->orig = reinterpret_cast<int32_t*>(p + b_rp + 2 * b_ci);
        L->val2 = p + b_rp + 2 * b_ci + b_or;
        L->d_sum = reinterpret_cast<unsigned long long*>(p + b_rp + 2 * b_ci + b_or + b_val);
        KPM_HIP(ctx, hipMemcpyAsync(L->rp2, rp2.data(), rp2.size() * 4, hipMemcpyHostToDevice, ctx->stream));
        if (A.nnz > 0) {
            KPM_HIP(ctx, hipMemcpyAsync(L->ci2, ci2.data(), ci2.size() * 4, hipMemcpyHostToDevice, ctx->stream));
            KPM_HIP(ctx, hipMemcpyAsync(L->src, src.data(), src.size() * 4, hipMemcpyHostToDevice, ctx->stream));
        }
        KPM_HIP(ctx, hipMemcpyAsync(L->orig, perm.data(), perm.size() * 4, hipMemcpyHostToDevice, ctx->stream));
        const hipError_t e = hipStreamSynchronize(ctx->stream);  // the host arrays go out of scope
        if (e != hipSuccess) {
            kpm_locality_free(ctx);
            return kpm_hip_fail(ctx, e, "renumbered matrix upload");
        }
        L->n = A.n;
    }
    if (!L->structured) return KPM_OK;
    if (!refresh && L->check_pending) {
        // refreshed earlier in the same call (checksum and values enqueued)
        out->rp = L->rp2;
        out->ci = L->ci2;
        out->val = L->val2;
        *orig = L->orig;
        return KPM_OK;
    }
    // the checksum of the current structure, copied to page-locked host
    // memory behind it and compared with the plan's once the caller has
    // waited for its results (kpm_locality_check)
    clear_sum_kernel<<<1, 1, 0, ctx->stream>>>(L->d_sum);
    structure_sum_kernel<<<(int)std::min<int64_t>(2048, (A.nnz + A.n + 256) / 256), 256, 0, ctx->stream>>>(
        A.rp, A.n, A.ci, A.nnz, L->d_sum);
    KPM_HIP(ctx, hipGetLastError());
    KPM_HIP(ctx, hipMemcpyAsync(L->h_sum, L->d_sum, sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream));
    L->check_pending = true;
    // the current values, in the renumbered order
    if (A.nnz > 0) {
        const int64_t blocks = std::min<int64_t>(8192, (A.nnz + 255) / 256);
        if (A.val_f64)
            gather_values_kernel<double><<<(int)blocks, 256, 0, ctx->stream>>>(
                static_cast<const double*>(A.val), L->src, A.nnz, static_cast<double*>(L->val2));
        else
            gather_values_kernel<float><<<(int)blocks, 256, 0, ctx->stream>>>(
                static_cast<const float*>(A.val), L->src, A.nnz, static_cast<float*>(L->val2));
        KPM_HIP(ctx, hipGetLastError());
    }
    out->rp = L->rp2;
    out->ci = L->ci2;
    out->val = L->val2;
    *orig = L->orig;
    return KPM_OK;
}

kpm_status kpm_locality_check(kpm_ctx* ctx) {
    kpm_locality_state* L = ctx->loc;
    if (!L || !L->check_pending) return KPM_OK;
    L->check_pending = false;
    // the caller has waited for its stream, and so for the checksum's copy
    if ((uint64_t)*L->h_sum != L->sum) {
        kpm_locality_free(ctx);  // rebuilt from the current structure on the next call
        return kpm_fail(ctx, KPM_ERR_ARG,
                        "the matrix's sparsity structure changed since its renumbered copy was built (same address "
                        "and sizes): call again to rebuild it");
    }
    return KPM_OK;
}
