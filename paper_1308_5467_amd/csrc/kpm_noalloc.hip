// kpm_moments_noalloc: the Chebyshev moments of kpm_moments (section 3.1.1,
// Algorithm 1, with the product identity of Appendix A) for callers that
// cannot allocate device memory (code under HIP graph capture, serving
// loops that forbid hipMalloc).  The probe blocks, dot partials, reduced
// dots and (when the caller passes no per-probe output) per-probe moments
// live in one file-scope device array, `scratch`, of
// KPM_NOALLOC_SCRATCH_BYTES.
//
// A file-scope __device__ array has one instance per device the code object
// is loaded on, at an address that differs per device, and its host-side
// name is only a handle: it is resolved with hipGetSymbolAddress once per
// device (kpm_create calls kpm_noalloc_attach with the device current) and
// only the resolved pointer is passed to kernels.
//
// The launches are those of kpm_moments with the same geometry (probe
// block width, panel height, gather batch, grid, walk direction), so the
// results are bitwise those of kpm_moments for the same options.  Nothing
// needs clearing between calls: the probe fill writes every entry of the
// first block (padding columns included), each step writes every row of
// the other block and one partial per workgroup, and each reduction writes
// every dot it covers.  Calls that overlap on one device race on the array.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <mutex>

#include "kpm_internal.h"

using namespace kpm;

static __device__ __align__(256) unsigned char scratch[KPM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

struct ScratchTable {
    std::mutex mu;
    bool tried[kMaxDevices] = {};
    void* ptr[kMaxDevices] = {};
    hipError_t err[kMaxDevices] = {};
};
ScratchTable& table() {
    static ScratchTable t;
    return t;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Resolves this device's instance of `scratch` (the caller has made
// `device` current).  Idempotent per device; the outcome is recorded and
// reported by kpm_moments_noalloc.
void kpm_noalloc_attach(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    ScratchTable& t = table();
    std::lock_guard<std::mutex> lock(t.mu);
    if (t.tried[device]) return;
    t.tried[device] = true;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    t.err[device] = e;
    t.ptr[device] = e == hipSuccess ? p : nullptr;
}

static kpm_status scratch_of(kpm_ctx* ctx, void** out) {
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "device ordinal beyond the scratch table");
    ScratchTable& t = table();
    std::lock_guard<std::mutex> lock(t.mu);
    if (!t.tried[ctx->device])
        return kpm_fail(ctx, KPM_ERR_HIP, "scratch array not resolved for this device (context not made by kpm_create)");
    if (t.err[ctx->device] != hipSuccess || !t.ptr[ctx->device])
        return kpm_hip_fail(ctx, t.err[ctx->device] != hipSuccess ? t.err[ctx->device] : hipErrorInvalidSymbol,
                            "hipGetSymbolAddress(scratch)");
    *out = t.ptr[ctx->device];
    return KPM_OK;
}

extern "C" kpm_status kpm_moments_noalloc(kpm_ctx* ctx, const kpm_csr* Ain, double lb, double ub,
                                          const kpm_moment_opts* o, double* mu, double* mu_per_vec) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!o || !mu) return kpm_fail(ctx, KPM_ERR_ARG, "opts or mu is NULL");
    if (!Ain) return kpm_fail(ctx, KPM_ERR_ARG, "matrix is NULL");
    if (!Ain->on_device) return kpm_fail(ctx, KPM_ERR_ARG, "the matrix must be in device memory (on_device = 1)");
    if (Ain->n < 1 || Ain->n >= ((int64_t)1 << 31)) return kpm_fail(ctx, KPM_ERR_ARG, "n must be in [1, 2^31)");
    if (Ain->nnz < 0 || Ain->nnz >= ((int64_t)1 << 31)) return kpm_fail(ctx, KPM_ERR_ARG, "nnz must be in [0, 2^31)");
    if (!Ain->row_ptr || (Ain->nnz > 0 && (!Ain->col_idx || !Ain->val)))
        return kpm_fail(ctx, KPM_ERR_ARG, "CSR array pointer is NULL");
    if (o->M < 0 || o->M > (1 << 20)) return kpm_fail(ctx, KPM_ERR_ARG, "M must be in [0, 2^20]");
    if (o->nvec < 1 || o->nvec > (1 << 24)) return kpm_fail(ctx, KPM_ERR_ARG, "nvec must be in [1, 2^24]");
    if (o->precision != KPM_FP32 && o->precision != KPM_FP64)
        return kpm_fail(ctx, KPM_ERR_ARG, "precision must be KPM_FP32 or KPM_FP64");
    if (o->precision == KPM_FP32 && Ain->val_is_f64)
        return kpm_fail(ctx, KPM_ERR_ARG, "the FP32 path needs FP32 values here (no conversion buffer)");
    const int maxb = o->precision == KPM_FP64 ? 128 : 256;
    if (o->block < 0 || o->block > maxb) return kpm_fail(ctx, KPM_ERR_ARG, "block out of range");
    if (o->rows_per_block < 0 || o->rows_per_block > (1 << 20))
        return kpm_fail(ctx, KPM_ERR_ARG, "rows_per_block out of range");
    if (o->validate) return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "validate must be 0 (validation waits on the host)");
    if (o->flags & KPM_FLAG_LOCALITY)
        return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "KPM_FLAG_LOCALITY allocates its renumbered copy of the matrix");
    if (!(isfinite(lb) && isfinite(ub) && ub > lb)) return kpm_fail(ctx, KPM_ERR_ARG, "need finite lb < ub");
    void* base;
    kpm_status st = scratch_of(ctx, &base);
    if (st != KPM_OK) return st;
    KPM_HIP(ctx, hipSetDevice(ctx->device));

    CsrDev A;
    A.rp = Ain->row_ptr;
    A.ci = Ain->col_idx;
    A.val = Ain->val;
    A.val_f64 = Ain->val_is_f64 ? 1 : 0;
    A.n = (int32_t)Ain->n;
    A.nnz = (int32_t)Ain->nnz;

    const double c = 0.5 * (lb + ub), d = 0.5 * (ub - lb);
    const double alpha = 2.0 / d, beta = -2.0 * c / d;
    const int M = o->M, nvec = o->nvec;
    const int b = o->block > 0 ? std::min(o->block, nvec) : kpm_default_block(nvec, o->precision);
    const int K = (M + 1) / 2;
    const int esz = o->precision == KPM_FP64 ? 8 : 4;
    BlockGeom g = make_geom(A.n, b, o->precision, o->rows_per_block);
    if (o->flags & KPM_FLAG_GATHER4) g.gather = 4;
    if (o->flags & KPM_FLAG_GATHER7) g.gather = 7;
    if (o->flags & KPM_FLAG_GATHER8) g.gather = 8;
    const int grid = cheb_step_grid(A, o->precision, g);
    BlockGeom gr = g;
    int gridr = grid;
    if (nvec % b != 0) {
        gr = make_geom(A.n, nvec % b, o->precision, o->rows_per_block);
        gr.gather = g.gather;
        gridr = cheb_step_grid(A, o->precision, gr);
    }
    if (grid <= 0 || gridr <= 0) return kpm_fail(ctx, KPM_ERR_HIP, "could not size the step grid");

    // Scratch layout: X0 | X1 | dots | zeta (when mu_per_vec is NULL) |
    // partials of R steps.  The partial ring takes what is left, at most K
    // steps: the reduction of each step is the same fixed-order sum for any R.
    const size_t vbytes = align256((size_t)A.n * g.ld * esz);
    const size_t dbytes = align256((size_t)std::max(K, 1) * 2 * g.ld * 8);
    const size_t zbytes = mu_per_vec ? 0 : align256((size_t)nvec * (M + 1) * 8);
    const size_t step_part = std::max((size_t)grid * 2 * g.ld * 8, (size_t)gridr * 2 * gr.ld * 8);
    const size_t fixed = 2 * vbytes + dbytes + zbytes;
    const size_t cap = (size_t)KPM_NOALLOC_SCRATCH_BYTES;
    if (fixed + step_part > cap) {
        char msg[256];
        snprintf(msg, sizeof msg,
                 "problem needs %zu bytes of scratch (two probe blocks of n x %d values, dots%s and one step of "
                 "partials); the maximum is %zu",
                 fixed + step_part, g.ld, mu_per_vec ? "" : ", per-probe moments", cap);
        return kpm_fail(ctx, KPM_ERR_ARG, msg);
    }
    const int R = (int)std::max<size_t>(1, std::min<size_t>((size_t)std::max(K, 1), (cap - fixed) / step_part));
    char* p = static_cast<char*>(base);
    void* X0 = p;
    void* X1 = p + vbytes;
    double* dots = reinterpret_cast<double*>(p + 2 * vbytes);
    double* zeta = mu_per_vec ? mu_per_vec : reinterpret_cast<double*>(p + 2 * vbytes + dbytes);
    double* part = reinterpret_cast<double*>(p + fixed);

    const int nblk_vec = (nvec + b - 1) / b;
    for (int blk = 0; blk < nblk_vec; ++blk) {
        const int ncols = std::min(b, nvec - blk * b);
        const BlockGeom& gb = ncols == b ? g : gr;
        const int gridb = ncols == b ? grid : gridr;
        const int64_t vec0 = (int64_t)blk * b;
        KPM_HIP(ctx, launch_rademacher(ctx->stream, o->seed, vec0, ncols, gb.ld, A.n, o->precision, 1, X0));
        void* X[2] = {X0, X1};
        for (int s = 0; s < K; ++s) {
            double* ps = part + (size_t)(s % R) * gridb * 2 * gb.ld;
            KPM_HIP(ctx, launch_cheb_step(ctx->stream, A, o->precision, s == 0, gb, gridb, X[s & 1], X[(s + 1) & 1],
                                          alpha, beta, ps, (s & 1) != 0));
            if ((s + 1) % R == 0 || s == K - 1) {
                const int s0 = s - s % R;
                KPM_HIP(ctx, launch_reduce_partials(ctx->stream, part, gridb, 2 * gb.ld, s - s0 + 1,
                                                    dots + (size_t)s0 * 2 * gb.ld));
            }
        }
        KPM_HIP(ctx, launch_assemble(ctx->stream, dots, K, gb.ld, ncols, M, (double)A.n, vec0, zeta));
    }
    KPM_HIP(ctx, launch_mean_moments(ctx->stream, zeta, nvec, M, mu));
    return KPM_OK;
}
