// C ABI of the KPM library: context, workspace, argument checking and the
// host side of each entry point.  Every numerical step runs in the device
// kernels of this library; the host only orders launches, moves small
// arrays and solves the Lanczos tridiagonal eigenproblem (at most 32 x 32).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <string>
#include <thread>
#include <vector>

#include "kpm_internal.h"

using namespace kpm;

// ---------------------------------------------------------------- context helpers
kpm_status kpm_fail(kpm_ctx* ctx, kpm_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return st;
}

kpm_status kpm_hip_fail(kpm_ctx* ctx, hipError_t e, const char* what) {
    std::string m = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
    return kpm_fail(ctx, KPM_ERR_HIP, m);
}

kpm_status kpm_ws(kpm_ctx* ctx, const char* role, size_t bytes, void** out) {
    kpm_dev_buf& b = ctx->bufs[role];
    if (bytes == 0) bytes = 256;
    if (b.cap < bytes) {
        if (b.p) {
            hipError_t e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) return kpm_hip_fail(ctx, e, "hipStreamSynchronize (workspace)");
            hipFree(b.p);
            b.p = nullptr;
            b.cap = 0;
        }
        size_t cap = (bytes + 4095) / 4096 * 4096;
        hipError_t e = hipMalloc(&b.p, cap);
        if (e != hipSuccess) {
            b.p = nullptr;
            return kpm_fail(ctx, KPM_ERR_ALLOC,
                            std::string("hipMalloc of ") + std::to_string(cap) + " bytes for " + role + " failed");
        }
        b.cap = cap;
    }
    *out = b.p;
    return KPM_OK;
}

kpm_status kpm_pinned(kpm_ctx* ctx, size_t bytes, void** out) {
    if (bytes == 0) bytes = 256;
    if (ctx->pinned_cap < bytes) {
        if (ctx->pinned) {
            hipError_t e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) return kpm_hip_fail(ctx, e, "hipStreamSynchronize (pinned staging)");
            hipHostFree(ctx->pinned);
            ctx->pinned = nullptr;
            ctx->pinned_cap = 0;
        }
        const size_t cap = (bytes + 65535) / 65536 * 65536;
        hipError_t e = hipHostMalloc(&ctx->pinned, cap, hipHostMallocDefault);
        if (e != hipSuccess) {
            ctx->pinned = nullptr;
            return kpm_fail(ctx, KPM_ERR_ALLOC, "hipHostMalloc of the host staging buffer failed");
        }
        ctx->pinned_cap = cap;
    }
    *out = ctx->pinned;
    return KPM_OK;
}

void kpm_prof_begin(kpm_ctx* ctx, const char* kernel) { kpm_prof_begin_on(ctx, kernel, ctx->stream); }
void kpm_prof_end(kpm_ctx* ctx, const char* kernel, int launches) {
    kpm_prof_end_on(ctx, kernel, ctx->stream, launches);
}

void kpm_prof_begin_on(kpm_ctx* ctx, const char* kernel, hipStream_t stream) {
    if (!ctx->prof) return;
    kpm_prof_entry& e = ctx->prof_map[kernel];
    if (e.used + 2 > e.ev.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess) return;
            e.ev.push_back(ev);
        }
    }
    hipEventRecord(e.ev[e.used], stream);
}

void kpm_prof_end_on(kpm_ctx* ctx, const char* kernel, hipStream_t stream, int launches) {
    if (!ctx->prof) return;
    kpm_prof_entry& e = ctx->prof_map[kernel];
    if (e.used + 2 > e.ev.size()) return;
    hipEventRecord(e.ev[e.used + 1], stream);
    e.counts.push_back(launches);
    e.used += 2;
}

void kpm_prof_collect(kpm_ctx* ctx) {
    for (auto& kv : ctx->prof_map) {
        kpm_prof_entry& e = kv.second;
        for (size_t i = 0; i + 1 < e.used; i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e.ev[i], e.ev[i + 1]) == hipSuccess) {
                e.total_ms += ms;
                e.launches += e.counts[i / 2];
            }
        }
        e.used = 0;
        e.counts.clear();
    }
}

static kpm_status sync(kpm_ctx* ctx) {
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    kpm_prof_collect(ctx);
    return KPM_OK;
}

// ---------------------------------------------------------------- CSR intake
static kpm_status check_csr_args(kpm_ctx* ctx, const kpm_csr* A) {
    if (!A) return kpm_fail(ctx, KPM_ERR_ARG, "matrix is NULL");
    if (A->n < 1 || A->n >= ((int64_t)1 << 31))
        return kpm_fail(ctx, KPM_ERR_ARG, "n must be in [1, 2^31)");
    if (A->nnz < 0 || A->nnz >= ((int64_t)1 << 31))
        return kpm_fail(ctx, KPM_ERR_ARG, "nnz must be in [0, 2^31)");
    if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
        return kpm_fail(ctx, KPM_ERR_ARG, "CSR array pointer is NULL");
    return KPM_OK;
}

// Device view of A; host arrays are copied into the context, FP64 values are
// rounded to FP32 when the FP32 path is requested.
kpm_status kpm_prepare_csr(kpm_ctx* ctx, const kpm_csr* A, int precision, CsrDev* out, const char* tag) {
    kpm_status st = check_csr_args(ctx, A);
    if (st != KPM_OK) return st;
    CsrDev D;
    D.n = (int32_t)A->n;
    D.nnz = (int32_t)A->nnz;
    D.val_f64 = A->val_is_f64 ? 1 : 0;
    const size_t vbytes = (size_t)A->nnz * (A->val_is_f64 ? 8 : 4);
    if (A->on_device) {
        D.rp = A->row_ptr;
        D.ci = A->col_idx;
        D.val = A->val;
    } else {
        void *rp, *ci, *va;
        std::string t(tag);
        if ((st = kpm_ws(ctx, ("csr_rp" + t).c_str(), (size_t)(A->n + 1) * 4, &rp)) != KPM_OK) return st;
        if ((st = kpm_ws(ctx, ("csr_ci" + t).c_str(), (size_t)A->nnz * 4, &ci)) != KPM_OK) return st;
        if ((st = kpm_ws(ctx, ("csr_val" + t).c_str(), vbytes, &va)) != KPM_OK) return st;
        KPM_HIP(ctx, hipMemcpyAsync(rp, A->row_ptr, (size_t)(A->n + 1) * 4, hipMemcpyHostToDevice, ctx->stream));
        if (A->nnz > 0) {
            KPM_HIP(ctx, hipMemcpyAsync(ci, A->col_idx, (size_t)A->nnz * 4, hipMemcpyHostToDevice, ctx->stream));
            KPM_HIP(ctx, hipMemcpyAsync(va, A->val, vbytes, hipMemcpyHostToDevice, ctx->stream));
        }
        D.rp = (const int32_t*)rp;
        D.ci = (const int32_t*)ci;
        D.val = va;
    }
    if (precision == KPM_FP32 && D.val_f64) {
        void* v32;
        if ((st = kpm_ws(ctx, (std::string("csr_val32") + tag).c_str(), (size_t)A->nnz * 4, &v32)) != KPM_OK)
            return st;
        if (A->nnz > 0) KPM_HIP(ctx, launch_convert_f64_to_f32(ctx->stream, (const double*)D.val, (float*)v32, A->nnz));
        D.val = v32;
        D.val_f64 = 0;
    }
    *out = D;
    return KPM_OK;
}

kpm_status kpm_validate_csr(kpm_ctx* ctx, const CsrDev& D) {
    void* f;
    kpm_status st = kpm_ws(ctx, "flags", 64, &f);
    if (st != KPM_OK) return st;
    KPM_HIP(ctx, hipMemsetAsync(f, 0, 16, ctx->stream));
    KPM_HIP(ctx, launch_validate_csr(ctx->stream, D, (int*)f));
    int flags[4] = {0, 0, 0, 0};
    KPM_HIP(ctx, hipMemcpyAsync(flags, f, 16, hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync(ctx)) != KPM_OK) return st;
    if (flags[0]) return kpm_fail(ctx, KPM_ERR_ARG, "row_ptr is not a valid CSR row pointer");
    if (flags[1]) return kpm_fail(ctx, KPM_ERR_ARG, "col_idx out of range or not strictly increasing within a row");
    if (flags[2]) return kpm_fail(ctx, KPM_ERR_ARG, "matrix values are not all finite");
    return KPM_OK;
}

// ---------------------------------------------------------------- create / destroy
extern "C" kpm_status kpm_create(int device, void* hip_stream, kpm_ctx** out) {
    if (!out) return KPM_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return KPM_ERR_HIP;
    if (device < 0 || device >= count) return KPM_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return KPM_ERR_HIP;
    kpm_noalloc_attach(device);
    kpm_ctx* ctx = new kpm_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    *out = ctx;
    return KPM_OK;
}

extern "C" kpm_status kpm_destroy(kpm_ctx* ctx) {
    if (!ctx) return KPM_ERR_ARG;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    kpm_batch_free(ctx);
    kpm_locality_free(ctx);
    for (auto& kv : ctx->bufs)
        if (kv.second.p) hipFree(kv.second.p);
    if (ctx->mlp_params.p) hipFree(ctx->mlp_params.p);
    for (auto& kv : ctx->prof_map)
        for (hipEvent_t e : kv.second.ev) hipEventDestroy(e);
    if (ctx->pinned) hipHostFree(ctx->pinned);
    if (ctx->copy_done) hipEventDestroy(ctx->copy_done);
    if (ctx->aux) {
        hipStreamSynchronize(ctx->aux);
        hipStreamDestroy(ctx->aux);
    }
    if (ctx->aux_fork) hipEventDestroy(ctx->aux_fork);
    if (ctx->aux_join) hipEventDestroy(ctx->aux_join);
    delete ctx;
    return KPM_OK;
}

extern "C" kpm_status kpm_set_stream(kpm_ctx* ctx, void* hip_stream) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return KPM_OK;
}

extern "C" const char* kpm_last_error(const kpm_ctx* ctx) {
    if (!ctx) return "context is NULL";
    return ctx->err.c_str();
}

// ---------------------------------------------------------------- bounds
// The bounds of kpm_bounds.  `overlap` (nullable) enqueues more work on the
// context's stream after the Lanczos coefficients' copy; the host then waits
// for the copy alone, so that work runs while the host finishes the bounds.
// [lb0, ub0] from the coefficients of an m-step Lanczos run (hc: alpha at
// 0, beta at 64): the extreme Ritz values widened by their residual norms
// (section 3.1.1).  *breakdown: the run stopped early on a vanishing
// residual, after which the caller merges the Gershgorin hull.  Touches no
// context (the many-matrix form runs it on several host threads); on error
// *msg names the failure.
static kpm_status lanczos_interval(const double* hc, int m, double* lb0, double* ub0, bool* breakdown,
                                   const char** msg) {
    // Breakdown test in step order: stop at the first residual below 1e-12 of
    // the largest coefficient seen so far.
    double scale = 0.0, beta_last = 0.0;
    int k = m;
    *breakdown = false;
    for (int j = 0; j < m; ++j) {
        const double a = hc[j], b = hc[64 + j];
        if (!isfinite(a) || !isfinite(b)) {
            *msg = "non-finite Lanczos coefficient (matrix values not finite?)";
            return KPM_ERR_ARG;
        }
        scale = std::max(scale, std::max(fabs(a), b));
        if (j == m - 1) {
            beta_last = b;
            break;
        }
        if (b <= 1e-12 * scale) {
            *breakdown = true;
            beta_last = b;
            k = j + 1;
            break;
        }
    }
    // Ritz values and the last components s_k of the Ritz vectors: the last
    // components of T's eigenvectors are the first components of those of
    // the flipped matrix J T J (J the reversal), which the implicit QR solver
    // accumulates in O(k^2) without forming eigenvectors.
    std::vector<double> fa(k), fb(std::max(k - 1, 1), 0.0), theta(k), s2(k);
    for (int j = 0; j < k; ++j) fa[j] = hc[k - 1 - j];
    for (int j = 0; j + 1 < k; ++j) fb[j] = hc[64 + k - 2 - j];
    const kpm_status es = kpm_tridiag_eig(k, fa.data(), fb.data(), theta.data(), s2.data());
    if (es == KPM_ERR_NOCONV) {
        *msg = "QR iteration on the Lanczos matrix did not converge";
        return es;
    }
    if (es != KPM_OK) {
        *msg = "Lanczos matrix eigenproblem failed";
        return es;
    }
    // residual norms beta_k |s_k| of the extreme Ritz pairs
    const double rlo = beta_last * sqrt(s2[0]);
    const double rhi = beta_last * sqrt(s2[k - 1]);
    *lb0 = theta[0] - rlo;
    *ub0 = theta[k - 1] + rhi;
    return KPM_OK;
}

// The margin: [lb0, ub0] maps into [-(1 - margin), 1 - margin], with a
// half-width of at least margin * max(|c|, 1); a zero half-width (margin 0
// on a 1 x 1 matrix) becomes 1, so that no rescaling divides by zero.
static void widen_interval(double lb0, double ub0, double margin, double* lb, double* ub) {
    const double c = 0.5 * (lb0 + ub0);
    double d = 0.5 * (ub0 - lb0) / (1.0 - margin);
    d = std::max(d, margin * std::max(fabs(c), 1.0));
    if (!(d > 0.0)) d = 1e-300 > d ? 1.0 : d;
    *lb = c - d;
    *ub = c + d;
}

static kpm_status bounds_impl(kpm_ctx* ctx, const kpm_csr* Ain, int steps, uint64_t seed, double margin,
                              double* lb, double* ub, const std::function<kpm_status()>& overlap) {
    if (!lb || !ub) return kpm_fail(ctx, KPM_ERR_ARG, "lb/ub output is NULL");
    if (steps < 1 || steps > 32) return kpm_fail(ctx, KPM_ERR_ARG, "steps must be in [1, 32]");
    if (!(margin >= 0.0 && margin < 0.5)) return kpm_fail(ctx, KPM_ERR_ARG, "margin must be in [0, 0.5)");
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    CsrDev A;
    kpm_status st = kpm_prepare_csr(ctx, Ain, KPM_FP64, &A, "");
    if (st != KPM_OK) return st;
    const int n = A.n;
    const int m = std::min(steps, n);
    LanczosWork W;
    W.chunk = 256 * lanczos_rows_per_thread(n);
    W.nblk = (int)(((int64_t)n + W.chunk - 1) / W.chunk);
    void *Q, *w, *coef, *part;
    if ((st = kpm_ws(ctx, "lz_Q", (size_t)m * n * 8, &Q)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "lz_w", (size_t)2 * n * 8, &w)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "lz_coef", 256 * 8, &coef)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "lz_part", (size_t)3 * 32 * W.nblk * 8 + (size_t)2 * 8 * W.nblk, &part)) != KPM_OK)
        return st;
    W.Q = (double*)Q;
    W.w = (double*)w;
    W.coef = (double*)coef;
    W.partial = (double*)part;
    kpm_prof_begin(ctx, "lanczos");
    KPM_HIP(ctx, launch_lanczos(ctx->stream, A, m, seed, W));
    kpm_prof_end(ctx, "lanczos", 1);
    void* stage;
    if ((st = kpm_pinned(ctx, 256 * 8, &stage)) != KPM_OK) return st;
    KPM_HIP(ctx, hipMemcpyAsync(stage, coef, 256 * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (overlap) {
        if (!ctx->copy_done) KPM_HIP(ctx, hipEventCreateWithFlags(&ctx->copy_done, hipEventDisableTiming));
        KPM_HIP(ctx, hipEventRecord(ctx->copy_done, ctx->stream));
        if ((st = overlap()) != KPM_OK) return st;
        KPM_HIP(ctx, hipEventSynchronize(ctx->copy_done));
    } else if ((st = sync(ctx)) != KPM_OK) {
        return st;
    }
    const double* hc = (const double*)stage;
    double lb0, ub0;
    bool breakdown;
    const char* msg = nullptr;
    if ((st = lanczos_interval(hc, m, &lb0, &ub0, &breakdown, &msg)) != KPM_OK) return kpm_fail(ctx, st, msg);
    if (breakdown) {
        const int gb = W.nblk;
        double* gout = (double*)part + (size_t)3 * 32 * W.nblk;
        KPM_HIP(ctx, launch_gershgorin(ctx->stream, A, gout, gb));
        std::vector<double> hg(2 * gb);
        KPM_HIP(ctx, hipMemcpyAsync(hg.data(), gout, 2 * gb * 8, hipMemcpyDeviceToHost, ctx->stream));
        if ((st = sync(ctx)) != KPM_OK) return st;
        for (int b = 0; b < gb; ++b) {
            lb0 = std::min(lb0, hg[2 * b]);
            ub0 = std::max(ub0, hg[2 * b + 1]);
        }
    }
    widen_interval(lb0, ub0, margin, lb, ub);
    return KPM_OK;
}

extern "C" kpm_status kpm_bounds(kpm_ctx* ctx, const kpm_csr* Ain, int steps, uint64_t seed,
                                 double margin, double* lb, double* ub) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    return bounds_impl(ctx, Ain, steps, seed, margin, lb, ub, nullptr);
}

extern "C" kpm_status kpm_bounds_batched(kpm_ctx* ctx, int nmat, const kpm_csr* Ain, int steps, uint64_t seed,
                                         double margin, double* lb, double* ub) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!Ain || !lb || !ub) return kpm_fail(ctx, KPM_ERR_ARG, "A, lb or ub is NULL");
    if (nmat < 1 || nmat > (1 << 20)) return kpm_fail(ctx, KPM_ERR_ARG, "nmat must be in [1, 2^20]");
    if (steps < 1 || steps > 32) return kpm_fail(ctx, KPM_ERR_ARG, "steps must be in [1, 32]");
    if (!(margin >= 0.0 && margin < 0.5)) return kpm_fail(ctx, KPM_ERR_ARG, "margin must be in [0, 0.5)");
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    std::vector<CsrDev> A(nmat);
    kpm_status st;
    for (int m = 0; m < nmat; ++m) {
        if (!Ain[m].on_device)
            return kpm_fail(ctx, KPM_ERR_ARG, "matrix " + std::to_string(m) + ": on_device must be 1");
        if ((st = kpm_prepare_csr(ctx, &Ain[m], KPM_FP64, &A[m], "")) != KPM_OK) return st;
    }
    LanczosBatchLayout L;
    lanczos_batch_layout(nmat, A.data(), steps, &L);
    void *Q, *w, *coef, *part, *tab, *stage;
    if ((st = kpm_ws(ctx, "lzb_Q", (size_t)L.q_total * 8, &Q)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "lzb_w", (size_t)L.w_total * 8, &w)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "lzb_coef", (size_t)nmat * 256 * 8, &coef)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "lzb_part", (size_t)L.part_total * 8, &part)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "lzb_tab", L.table_bytes, &tab)) != KPM_OK) return st;
    // one staging buffer for the tables' upload and the coefficients' copy
    // back (ordered on the stream)
    if ((st = kpm_pinned(ctx, std::max(L.table_bytes, (size_t)nmat * 256 * 8), &stage)) != KPM_OK) return st;
    if (!ctx->aux) {
        KPM_HIP(ctx, hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
        KPM_HIP(ctx, hipEventCreateWithFlags(&ctx->aux_fork, hipEventDisableTiming));
        KPM_HIP(ctx, hipEventCreateWithFlags(&ctx->aux_join, hipEventDisableTiming));
    }
    kpm_prof_begin(ctx, "lanczos_batched");
    KPM_HIP(ctx, launch_lanczos_batched(ctx->stream, nmat, A.data(), seed, L, (double*)Q, (double*)w,
                                        (double*)coef, (double*)part, tab, stage, nullptr, ctx->aux, ctx->aux_fork,
                                        ctx->aux_join));
    kpm_prof_end(ctx, "lanczos_batched", 1);
    KPM_HIP(ctx, hipMemcpyAsync(stage, coef, (size_t)nmat * 256 * 8, hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync(ctx)) != KPM_OK) return st;
    // the small tridiagonal problems, on up to 16 host threads
    const double* hc = (const double*)stage;
    std::vector<double> lb0(nmat), ub0(nmat);
    std::vector<char> brk(nmat, 0);
    std::vector<kpm_status> mst(nmat, KPM_OK);
    std::vector<const char*> msg(nmat, nullptr);
    auto solve = [&](int t0, int T) {
        for (int m = t0; m < nmat; m += T) {
            bool b = false;
            mst[m] = lanczos_interval(hc + (size_t)256 * m, L.m[m], &lb0[m], &ub0[m], &b, &msg[m]);
            brk[m] = b ? 1 : 0;
        }
    };
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int T = std::max(1, std::min(std::min((int)hw, 16), (nmat + 63) / 64));
    if (T == 1) {
        solve(0, 1);
    } else {
        std::vector<std::thread> pool;
        pool.reserve(T - 1);
        for (int t = 1; t < T; ++t) pool.emplace_back(solve, t, T);
        solve(0, T);
        for (std::thread& th : pool) th.join();
    }
    for (int m = 0; m < nmat; ++m)
        if (mst[m] != KPM_OK) return kpm_fail(ctx, mst[m], "matrix " + std::to_string(m) + ": " + msg[m]);
    // Gershgorin hulls of the matrices whose run broke down
    std::vector<int> bm;
    int64_t gtot = 0;
    for (int m = 0; m < nmat; ++m)
        if (brk[m]) {
            bm.push_back(m);
            gtot += 2 * L.nblk[m];
        }
    if (!bm.empty()) {
        std::vector<double> hg((size_t)gtot);
        int64_t o = 0;
        for (int m : bm) {
            double* gout = (double*)part + lanczos_batch_gershgorin_off(L, m);
            KPM_HIP(ctx, launch_gershgorin(ctx->stream, A[m], gout, L.nblk[m]));
            KPM_HIP(ctx, hipMemcpyAsync(hg.data() + o, gout, (size_t)2 * L.nblk[m] * 8, hipMemcpyDeviceToHost,
                                        ctx->stream));
            o += 2 * L.nblk[m];
        }
        if ((st = sync(ctx)) != KPM_OK) return st;
        o = 0;
        for (int m : bm) {
            for (int b = 0; b < L.nblk[m]; ++b) {
                lb0[m] = std::min(lb0[m], hg[o + 2 * b]);
                ub0[m] = std::max(ub0[m], hg[o + 2 * b + 1]);
            }
            o += 2 * L.nblk[m];
        }
    }
    for (int m = 0; m < nmat; ++m) widen_interval(lb0[m], ub0[m], margin, &lb[m], &ub[m]);
    return KPM_OK;
}

extern "C" kpm_status kpm_gershgorin(kpm_ctx* ctx, const kpm_csr* Ain, double* lo, double* hi) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!lo || !hi) return kpm_fail(ctx, KPM_ERR_ARG, "lo/hi output is NULL");
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    CsrDev A;
    kpm_status st = kpm_prepare_csr(ctx, Ain, KPM_FP64, &A, "");
    if (st != KPM_OK) return st;
    const int nblk = (int)std::min<int64_t>(1024, ((int64_t)A.n + 255) / 256);
    void* g;
    if ((st = kpm_ws(ctx, "gersh", (size_t)2 * nblk * 8, &g)) != KPM_OK) return st;
    KPM_HIP(ctx, launch_gershgorin(ctx->stream, A, (double*)g, nblk));
    std::vector<double> hg(2 * nblk);
    KPM_HIP(ctx, hipMemcpyAsync(hg.data(), g, hg.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync(ctx)) != KPM_OK) return st;
    double a = hg[0], b = hg[1];
    for (int i = 1; i < nblk; ++i) {
        a = std::min(a, hg[2 * i]);
        b = std::max(b, hg[2 * i + 1]);
    }
    if (!isfinite(a) || !isfinite(b)) return kpm_fail(ctx, KPM_ERR_ARG, "matrix values are not all finite");
    *lo = a;
    *hi = b;
    return KPM_OK;
}

// ---------------------------------------------------------------- moments
// Default probe-block width: 256-byte probe rows (64 FP32 or 32 FP64
// probes), so the gathered rows of a 3D stencil's neighbouring planes stay
// in an XCD's L2.  64 FP64 probes (512-byte rows) overflow it: on a 64^3
// stencil, 64 probes took 94.9 us per step as one block and 2 x 38.5 us as
// two blocks of 32 (degree 256: 12.3 vs 10.0 ms per call).
int kpm::kpm_default_block(int nvec, int precision) {
    return std::min(nvec, precision == KPM_FP64 ? 32 : 64);
}
static int default_block(int nvec, int precision) { return kpm::kpm_default_block(nvec, precision); }

// Device results of a moment computation still in flight on the context's
// stream: mean moments mud [M+1] and per-probe normalised moments zout
// [nvec x (M+1)].
struct MomentsPending {
    void* mud = nullptr;
    void* zout = nullptr;
    int M = 0, nvec = 0, precision = KPM_FP32;
};

// Copies the moments to the host (mu nullable, mu_per_vec nullable), waits
// for the stream and checks |mu_k| <= 1 per probe.
// Copies go through the context's page-locked staging buffer; `extra`
// (nullable) is one more device array of extra_n doubles copied to
// extra_host in the same wait.
static kpm_status moments_collect(kpm_ctx* ctx, const MomentsPending& P, double* mu, double* mu_per_vec,
                                  const double* extra = nullptr, size_t extra_n = 0, double* extra_host = nullptr) {
    const int M = P.M, nvec = P.nvec;
    const size_t nm = (size_t)M + 1, nz = (size_t)nvec * (M + 1);
    void* stage;
    kpm_status st;
    if ((st = kpm_pinned(ctx, (nm + nz + extra_n) * 8, &stage)) != KPM_OK) return st;
    double* sm = (double*)stage;
    double* sz = sm + nm;
    double* sx = sz + nz;
    KPM_HIP(ctx, hipMemcpyAsync(sm, P.mud, nm * 8, hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(sz, P.zout, nz * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (extra && extra_n) KPM_HIP(ctx, hipMemcpyAsync(sx, extra, extra_n * 8, hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync(ctx)) != KPM_OK) return st;
    if ((st = kpm_locality_check(ctx)) != KPM_OK) return st;
    if (mu) memcpy(mu, sm, nm * 8);
    if (extra && extra_n) memcpy(extra_host, sx, extra_n * 8);
    std::vector<double>& hz = ctx->host_scratch;
    hz.assign(sz, sz + nz);
    if (mu_per_vec) memcpy(mu_per_vec, hz.data(), hz.size() * 8);
    // |v^T T_k(B) v| <= v^T v = n when the spectrum of B lies in [-1, 1]
    // (and so |v^T L_k(B) v| <= n, a convex combination of those).
    const double tol = P.precision == KPM_FP64 ? 1e-9 : 1e-4;
    for (size_t i = 0; i < hz.size(); ++i) {
        if (!isfinite(hz[i]) || fabs(hz[i]) > 1.0 + tol) {
            char msg[200];
            snprintf(msg, sizeof msg,
                     "spectrum escaped [lb, ub]: probe %zu moment %zu = %g (|mu_k| must stay <= 1)",
                     i / (M + 1), i % (M + 1), hz[i]);
            return kpm_fail(ctx, KPM_ERR_SPECTRUM, msg);
        }
    }
    return KPM_OK;
}

// Chebyshev moments, or (legendre) the Legendre moments obtained from them
// by the non-negative Chebyshev-to-Legendre weights on the device.  With
// `pending` the work is only enqueued (Chebyshev moments only) and the
// device results are described there; finish with moments_collect.
static kpm_status moments_impl(kpm_ctx* ctx, const kpm_csr* Ain, double lb, double ub,
                               const kpm_moment_opts* o, double* mu, double* mu_per_vec, bool legendre,
                               MomentsPending* pending = nullptr, bool block0_filled = false) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!o || (!mu && !pending)) return kpm_fail(ctx, KPM_ERR_ARG, "opts or mu is NULL");
    if (pending && legendre) return kpm_fail(ctx, KPM_ERR_ARG, "internal: pending Legendre moments");
    if (o->M < 0 || o->M > (1 << 20)) return kpm_fail(ctx, KPM_ERR_ARG, "M must be in [0, 2^20]");
    if (o->nvec < 1 || o->nvec > (1 << 24)) return kpm_fail(ctx, KPM_ERR_ARG, "nvec must be in [1, 2^24]");
    if (o->precision != KPM_FP32 && o->precision != KPM_FP64)
        return kpm_fail(ctx, KPM_ERR_ARG, "precision must be KPM_FP32 or KPM_FP64");
    const int maxb = o->precision == KPM_FP64 ? 128 : 256;
    if (o->block < 0 || o->block > maxb) return kpm_fail(ctx, KPM_ERR_ARG, "block out of range");
    if (o->rows_per_block < 0 || o->rows_per_block > (1 << 20))
        return kpm_fail(ctx, KPM_ERR_ARG, "rows_per_block out of range");
    if (!(isfinite(lb) && isfinite(ub) && ub > lb)) return kpm_fail(ctx, KPM_ERR_ARG, "need finite lb < ub");
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    CsrDev A;
    kpm_status st = kpm_prepare_csr(ctx, Ain, o->precision, &A, "");
    if (st != KPM_OK) return st;
    if (o->validate && (st = kpm_validate_csr(ctx, A)) != KPM_OK) return st;
    // KPM_FLAG_LOCALITY: the same moments on the matrix renumbered along its
    // grid's Morton curve, probes generated at the original row indices
    const int32_t* rows = nullptr;
    if (o->flags & KPM_FLAG_LOCALITY) {
        if (legendre && (o->flags & KPM_FLAG_LEGENDRE_RECURRENCE))
            return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "KPM_FLAG_LOCALITY with the Legendre recurrence");
        // a host matrix lives in reused workspace: its cached structure is
        // not trusted across calls
        if (!Ain->on_device) kpm_locality_free(ctx);
        CsrDev R;
        // the pipeline's prefill of the first block refreshed the view already
        if ((st = kpm_locality_view(ctx, A, &R, &rows, !block0_filled)) != KPM_OK) return st;
        A = R;
    }

    const double c = 0.5 * (lb + ub), d = 0.5 * (ub - lb);
    const double alpha = 2.0 / d, beta = -2.0 * c / d;
    const int M = o->M, nvec = o->nvec;
    const int b = o->block > 0 ? std::min(o->block, nvec) : default_block(nvec, o->precision);
    // ceil(M/2) sparse products per block with the product identity; M for
    // the Legendre recurrence, which has none.
    const bool leg_rec = legendre && (o->flags & KPM_FLAG_LEGENDRE_RECURRENCE);
    const int K = leg_rec ? M : (M + 1) / 2;
    const int esz = o->precision == KPM_FP64 ? 8 : 4;
    BlockGeom g = make_geom(A.n, b, o->precision, o->rows_per_block);
    if (o->flags & KPM_FLAG_GATHER4) g.gather = 4;
    if (o->flags & KPM_FLAG_GATHER7) g.gather = 7;
    if (o->flags & KPM_FLAG_GATHER8) g.gather = 8;

    void *X0, *X1, *part, *dots, *zeta, *mud;
    const int grid = cheb_step_grid(A, o->precision, g);
    const size_t vbytes = (size_t)A.n * g.ld * esz;
    if ((st = kpm_ws(ctx, "X0", vbytes, &X0)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "X1", vbytes, &X1)) != KPM_OK) return st;
    // Per-workgroup dot partials are kept for a ring of R steps and reduced
    // every R steps (and after the last), so this buffer is bounded (about
    // 64 MiB) whatever the degree; storing all K steps grew with the degree
    // (K x grid x 2 x ld x 8 bytes: 0.5 GB at degree 1000 and 64 FP32 probes).
    // The reduction of each step is the same fixed-order sum either way.
    size_t step_part = (size_t)grid * 2 * g.ld * 8;
    if (nvec % b != 0) {
        BlockGeom gr = make_geom(A.n, nvec % b, o->precision, o->rows_per_block);
        gr.gather = g.gather;
        step_part = std::max(step_part, (size_t)cheb_step_grid(A, o->precision, gr) * 2 * gr.ld * 8);
    }
    const int R = (int)std::max<size_t>(1, std::min<size_t>((size_t)std::max(K, 1), ((size_t)64 << 20) / step_part));
    if ((st = kpm_ws(ctx, "partial", (size_t)R * step_part, &part)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dots", (size_t)std::max(K, 1) * 2 * g.ld * 8, &dots)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "zeta", (size_t)nvec * (M + 1) * 8, &zeta)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "mu", (size_t)(M + 1) * 8, &mud)) != KPM_OK) return st;
    void* sgn = nullptr;
    const int sw = (g.ld + 31) / 32;
    if (leg_rec && (st = kpm_ws(ctx, "sign_bits", (size_t)A.n * sw * 4, &sgn)) != KPM_OK) return st;

    const int nblk_vec = (nvec + b - 1) / b;
    for (int blk = 0; blk < nblk_vec; ++blk) {
        const int ncols = std::min(b, nvec - blk * b);
        BlockGeom gb = g;
        if (ncols != b) {
            gb = make_geom(A.n, ncols, o->precision, o->rows_per_block);
            gb.gather = g.gather;
        }
        const int gridb = ncols == b ? grid : cheb_step_grid(A, o->precision, gb);
        const int64_t vec0 = (int64_t)blk * b;
        if (!(blk == 0 && block0_filled))
            KPM_HIP(ctx, launch_rademacher(ctx->stream, o->seed, vec0, ncols, gb.ld, A.n, o->precision, 1, X0, rows));
        const int swb = (gb.ld + 31) / 32;
        if (leg_rec)
            KPM_HIP(ctx, launch_sign_bits(ctx->stream, o->seed, vec0, ncols, A.n, swb, (uint32_t*)sgn));
        void* X[2] = {X0, X1};
        for (int s = 0; s < K; ++s) {
            double* ps = (double*)part + (size_t)(s % R) * gridb * 2 * gb.ld;
            // One event pair brackets the first step and one the run of the
            // remaining steps (events between launches would add gaps).
            if (s == 0) kpm_prof_begin(ctx, "cheb_first");
            if (s == 1) kpm_prof_begin(ctx, "cheb_step");
            // Odd steps walk the panels backwards: they start on the rows
            // the previous step finished with, still in the XCD's L2.
            if (leg_rec && s > 0) {
                // v_{s+1} = (2s+1)/(s+1) B v_s - s/(s+1) v_{s-1}, B = (A - cI)/d
                const double r = (double)(2 * s + 1) / (double)(s + 1);
                const LegStep ls{-(double)s / (double)(s + 1), (const uint32_t*)sgn, swb};
                KPM_HIP(ctx, launch_cheb_step(ctx->stream, A, o->precision, false, gb, gridb, X[s & 1],
                                              X[(s + 1) & 1], r / d, -r * c / d, ps, (s & 1) != 0, &ls));
            } else {
                KPM_HIP(ctx, launch_cheb_step(ctx->stream, A, o->precision, s == 0, gb, gridb, X[s & 1],
                                              X[(s + 1) & 1], alpha, beta, ps, (s & 1) != 0));
            }
            if (s == 0) kpm_prof_end(ctx, "cheb_first", 1);
            if (s == K - 1 && K > 1) kpm_prof_end(ctx, "cheb_step", K - 1);
            if ((s + 1) % R == 0 || s == K - 1) {
                const int s0 = s - s % R;
                KPM_HIP(ctx, launch_reduce_partials(ctx->stream, (double*)part, gridb, 2 * gb.ld, s - s0 + 1,
                                                    (double*)dots + (size_t)s0 * 2 * gb.ld));
            }
        }
        if (leg_rec)
            KPM_HIP(ctx, launch_legendre_assemble(ctx->stream, (double*)dots, gb.ld, ncols, M, (double)A.n, vec0,
                                                  (double*)zeta));
        else
            KPM_HIP(ctx, launch_assemble(ctx->stream, (double*)dots, K, gb.ld, ncols, M, (double)A.n, vec0,
                                         (double*)zeta));
    }
    void* zout = zeta;
    std::vector<double> aw;
    if (legendre && !leg_rec) {
        void *zl, *ad;
        if ((st = kpm_ws(ctx, "zeta_leg", (size_t)nvec * (M + 1) * 8, &zl)) != KPM_OK) return st;
        if ((st = kpm_ws(ctx, "leg_a", (size_t)(M + 1) * 8, &ad)) != KPM_OK) return st;
        aw.resize((size_t)M + 1);
        legendre_connection_weights(M, aw.data());
        KPM_HIP(ctx, hipMemcpyAsync(ad, aw.data(), aw.size() * 8, hipMemcpyHostToDevice, ctx->stream));
        KPM_HIP(ctx, launch_cheb_to_legendre(ctx->stream, (const double*)zeta, nvec, M, (const double*)ad,
                                             (double*)zl));
        zout = zl;
    }
    KPM_HIP(ctx, launch_mean_moments(ctx->stream, (double*)zout, nvec, M, (double*)mud));
    MomentsPending P;
    P.mud = mud;
    P.zout = zout;
    P.M = M;
    P.nvec = nvec;
    P.precision = o->precision;
    if (pending) {
        *pending = P;
        return KPM_OK;
    }
    return moments_collect(ctx, P, mu, mu_per_vec);
}

extern "C" kpm_status kpm_moments(kpm_ctx* ctx, const kpm_csr* A, double lb, double ub,
                                  const kpm_moment_opts* o, double* mu, double* mu_per_vec) {
    return moments_impl(ctx, A, lb, ub, o, mu, mu_per_vec, false);
}

extern "C" kpm_status kpm_legendre_moments(kpm_ctx* ctx, const kpm_csr* A, double lb, double ub,
                                           const kpm_moment_opts* o, double* mu, double* mu_per_vec) {
    return moments_impl(ctx, A, lb, ub, o, mu, mu_per_vec, true);
}

// ---------------------------------------------------------------- autotuner
// Times the fused step on A for candidate (probe-block width, row-panel
// height, gather batch) triples and returns the fastest per probe.  Each
// candidate runs the first step and kTuneWarm - 1 warm-up steps, then
// kTuneSteps timed steps between two events on the context's stream.  With
// KPM_FLAG_LOCALITY the steps run on the renumbered matrix kpm_moments would
// use, and the flag stays set in the returned options.
extern "C" kpm_status kpm_autotune(kpm_ctx* ctx, const kpm_csr* Ain, double lb, double ub,
                                   const kpm_moment_opts* o, kpm_moment_opts* best, double* us_per_step) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!o || !best) return kpm_fail(ctx, KPM_ERR_ARG, "opts or best is NULL");
    if (o->nvec < 1 || o->nvec > (1 << 24)) return kpm_fail(ctx, KPM_ERR_ARG, "nvec must be in [1, 2^24]");
    if (o->precision != KPM_FP32 && o->precision != KPM_FP64)
        return kpm_fail(ctx, KPM_ERR_ARG, "precision must be KPM_FP32 or KPM_FP64");
    const int maxb = o->precision == KPM_FP64 ? 128 : 256;
    if (o->block < 0 || o->block > maxb) return kpm_fail(ctx, KPM_ERR_ARG, "block out of range");
    if (o->rows_per_block < 0 || o->rows_per_block > (1 << 20))
        return kpm_fail(ctx, KPM_ERR_ARG, "rows_per_block out of range");
    if (!(isfinite(lb) && isfinite(ub) && ub > lb)) return kpm_fail(ctx, KPM_ERR_ARG, "need finite lb < ub");
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    CsrDev A;
    kpm_status st = kpm_prepare_csr(ctx, Ain, o->precision, &A, "");
    if (st != KPM_OK) return st;
    if (o->validate && (st = kpm_validate_csr(ctx, A)) != KPM_OK) return st;
    const int32_t* orig_rows = nullptr;  // original index of each renumbered row
    if (o->flags & KPM_FLAG_LOCALITY) {
        if (!Ain->on_device) kpm_locality_free(ctx);  // host matrices live in reused workspace
        CsrDev R;
        if ((st = kpm_locality_view(ctx, A, &R, &orig_rows)) != KPM_OK) return st;
        A = R;
    }

    const int nvec = o->nvec;
    std::vector<int> blocks;
    if (o->block > 0) {
        blocks.push_back(std::min(o->block, nvec));
    } else {
        const int cand32[] = {32, 64, 128}, cand64[] = {16, 32, 64};
        for (int c : (o->precision == KPM_FP64 ? cand64 : cand32))
            if (c <= nvec) blocks.push_back(c);
        if (blocks.empty()) blocks.push_back(nvec);
    }
    const int esz = o->precision == KPM_FP64 ? 8 : 4;
    int ldmax = 0;
    for (int b : blocks) ldmax = std::max(ldmax, make_geom(A.n, b, o->precision, 0).ld);
    constexpr int kTuneWarm = 8, kTuneSteps = 16;
    void *X0, *X1, *part;
    if ((st = kpm_ws(ctx, "X0", (size_t)A.n * ldmax * esz, &X0)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "X1", (size_t)A.n * ldmax * esz, &X1)) != KPM_OK) return st;
    hipEvent_t e0, e1;
    KPM_HIP(ctx, hipEventCreate(&e0));
    KPM_HIP(ctx, hipEventCreate(&e1));
    const double c = 0.5 * (lb + ub), d = 0.5 * (ub - lb);
    const double alpha = 2.0 / d, beta = -2.0 * c / d;
    double best_t = 1e300;
    kpm_moment_opts bo = *o;
    kpm_status rs = KPM_OK;
    for (int b : blocks) {
        const BlockGeom g0 = make_geom(A.n, b, o->precision, o->rows_per_block);
        std::vector<int> rows;
        if (o->rows_per_block > 0) rows.push_back(g0.rows_per_block);
        else rows = {std::max(1, g0.rows_per_block / 2), g0.rows_per_block, 2 * g0.rows_per_block};
        for (int r : rows)
            for (int G : {4, 7, 8}) {
                BlockGeom g = make_geom(A.n, b, o->precision, r);
                g.gather = G;
                const int grid = cheb_step_grid(A, o->precision, g);
                if ((rs = kpm_ws(ctx, "partial", (size_t)grid * 2 * g.ld * 8, &part)) != KPM_OK) break;
                hipError_t he =
                    launch_rademacher(ctx->stream, o->seed, 0, b, g.ld, A.n, o->precision, 1, X0, orig_rows);
                void* X[2] = {X0, X1};
                for (int k = 0; he == hipSuccess && k < kTuneWarm + kTuneSteps; ++k) {
                    if (k == kTuneWarm) he = hipEventRecord(e0, ctx->stream);
                    if (he == hipSuccess)
                        he = launch_cheb_step(ctx->stream, A, o->precision, k == 0, g, grid, X[k & 1], X[(k + 1) & 1],
                                              alpha, beta, (double*)part, (k & 1) != 0);
                }
                if (he == hipSuccess) he = hipEventRecord(e1, ctx->stream);
                if (he == hipSuccess) he = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
                if (he != hipSuccess) {
                    rs = kpm_hip_fail(ctx, he, "autotune candidate");
                    break;
                }
                const double t = (double)ms / kTuneSteps / b;  // per step and probe
                if (t < best_t) {
                    best_t = t;
                    bo.block = b;
                    bo.rows_per_block = g.rows_per_block;
                    bo.flags = (o->flags & ~(KPM_FLAG_GATHER4 | KPM_FLAG_GATHER7 | KPM_FLAG_GATHER8)) |
                               (G == 4 ? KPM_FLAG_GATHER4 : (G == 7 ? KPM_FLAG_GATHER7 : KPM_FLAG_GATHER8));
                }
            }
        if (rs != KPM_OK) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rs != KPM_OK) return rs;
    if ((st = kpm_locality_check(ctx)) != KPM_OK) return st;
    *best = bo;
    if (us_per_step) *us_per_step = best_t * 1000.0 * nvec;
    return KPM_OK;
}

extern "C" kpm_status kpm_moments_robust(kpm_ctx* ctx, const kpm_csr* A, int steps, uint64_t lanczos_seed,
                                         double margin, const kpm_moment_opts* o, double* mu,
                                         double* mu_per_vec, double* lb, double* ub, int* attempts) {
    if (!ctx) return KPM_ERR_ARG;
    if (!lb || !ub) return kpm_fail(ctx, KPM_ERR_ARG, "lb/ub output is NULL");
    double l, u;
    kpm_status st = kpm_bounds(ctx, A, steps, lanczos_seed, margin, &l, &u);
    if (st != KPM_OK) return st;
    for (int attempt = 1; attempt <= 3; ++attempt) {
        if (attempt == 2) {
            if ((st = kpm_bounds(ctx, A, steps, lanczos_seed, std::min(4.0 * margin, 0.4), &l, &u)) != KPM_OK)
                return st;
        } else if (attempt == 3) {
            double glo, ghi;
            if ((st = kpm_gershgorin(ctx, A, &glo, &ghi)) != KPM_OK) return st;
            const double c = 0.5 * (glo + ghi);
            double d = 0.5 * (ghi - glo) / (1.0 - margin);
            d = std::max(d, std::max(margin, 1e-3) * std::max(fabs(c), 1.0));
            l = c - d;
            u = c + d;
        }
        *lb = l;
        *ub = u;
        if (attempts) *attempts = attempt;
        st = kpm_moments(ctx, A, l, u, o, mu, mu_per_vec);
        if (st != KPM_ERR_SPECTRUM) return st;
    }
    return st;
}

// ---------------------------------------------------------------- damping / density
extern "C" kpm_status kpm_damping_factors(kpm_ctx* ctx, kpm_damping kind, int M, const double* mu,
                                          double* g) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!g || M < 0 || M > (1 << 20)) return kpm_fail(ctx, KPM_ERR_ARG, "bad M or g is NULL");
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    void* gd;
    kpm_status st = kpm_ws(ctx, "damp_g", (size_t)(M + 1) * 8, &gd);
    if (st != KPM_OK) return st;
    if (kind == KPM_DAMP_NONE) {
        for (int k = 0; k <= M; ++k) g[k] = 1.0;
        return KPM_OK;
    } else if (kind == KPM_DAMP_JACKSON) {
        KPM_HIP(ctx, launch_jackson(ctx->stream, M, (double*)gd));
    } else if (kind == KPM_DAMP_LEARNED) {
        if (!mu) return kpm_fail(ctx, KPM_ERR_ARG, "learned damping needs the moments");
        return kpm_learned_damping(ctx, M, mu, g);
    } else {
        return kpm_fail(ctx, KPM_ERR_ARG, "unknown damping kind");
    }
    KPM_HIP(ctx, hipMemcpyAsync(g, gd, (size_t)(M + 1) * 8, hipMemcpyDeviceToHost, ctx->stream));
    return sync(ctx);
}

static kpm_status upload_series(kpm_ctx* ctx, const double* mu, const double* g, int M, void** mud,
                                void** gd) {
    kpm_status st;
    if ((st = kpm_ws(ctx, "dos_mu", (size_t)(M + 1) * 8, mud)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dos_g", (size_t)(M + 1) * 8, gd)) != KPM_OK) return st;
    KPM_HIP(ctx, hipMemcpyAsync(*mud, mu, (size_t)(M + 1) * 8, hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(*gd, g, (size_t)(M + 1) * 8, hipMemcpyHostToDevice, ctx->stream));
    return KPM_OK;
}

extern "C" kpm_status kpm_dos(kpm_ctx* ctx, const double* mu, const double* g, int M, double lb,
                              double ub, const double* x, int npts, double* phi) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!mu || !g || !x || !phi || M < 0 || npts < 0) return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (!(isfinite(lb) && isfinite(ub) && ub > lb)) return kpm_fail(ctx, KPM_ERR_ARG, "need finite lb < ub");
    if (npts == 0) return KPM_OK;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    void *mud, *gd, *xd, *pd;
    kpm_status st = upload_series(ctx, mu, g, M, &mud, &gd);
    if (st != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dos_x", (size_t)npts * 8, &xd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dos_phi", (size_t)npts * 8, &pd)) != KPM_OK) return st;
    KPM_HIP(ctx, hipMemcpyAsync(xd, x, (size_t)npts * 8, hipMemcpyHostToDevice, ctx->stream));
    const double c = 0.5 * (lb + ub), d = 0.5 * (ub - lb);
    KPM_HIP(ctx, launch_dos(ctx->stream, (double*)mud, (double*)gd, M, c, d, (double*)xd, npts, (double*)pd));
    KPM_HIP(ctx, hipMemcpyAsync(phi, pd, (size_t)npts * 8, hipMemcpyDeviceToHost, ctx->stream));
    return sync(ctx);
}

extern "C" kpm_status kpm_dos_batched(kpm_ctx* ctx, int nmat, const double* mu, const double* g, int g_per_matrix,
                                      int M, const double* lb, const double* ub, const double* x, int npts,
                                      double* phi) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!mu || !g || !lb || !ub || !x || !phi || M < 0 || M > (1 << 20) || npts < 0 || nmat < 1 || nmat > 65535)
        return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    for (int m = 0; m < nmat; ++m)
        if (!(isfinite(lb[m]) && isfinite(ub[m]) && ub[m] > lb[m]))
            return kpm_fail(ctx, KPM_ERR_ARG, "matrix " + std::to_string(m) + ": need finite lb < ub");
    if (npts == 0) return KPM_OK;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    const size_t nm = (size_t)nmat * (M + 1), ng = g_per_matrix ? nm : (size_t)M + 1;
    const size_t np = (size_t)nmat * npts;
    void *mud, *gd, *bd, *xd, *pd;
    kpm_status st;
    if ((st = kpm_ws(ctx, "dosb_mu", nm * 8, &mud)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dosb_g", ng * 8, &gd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dosb_b", (size_t)2 * nmat * 8, &bd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dosb_x", np * 8, &xd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dosb_phi", np * 8, &pd)) != KPM_OK) return st;
    double* dlb = (double*)bd;
    double* dub = dlb + nmat;
    KPM_HIP(ctx, hipMemcpyAsync(mud, mu, nm * 8, hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(gd, g, ng * 8, hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(dlb, lb, (size_t)nmat * 8, hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(dub, ub, (size_t)nmat * 8, hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(xd, x, np * 8, hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, launch_dos_batched(ctx->stream, nmat, (const double*)mud, (const double*)gd,
                                    g_per_matrix ? (int64_t)M + 1 : 0, M, dlb, dub, (const double*)xd, npts,
                                    (double*)pd));
    KPM_HIP(ctx, hipMemcpyAsync(phi, pd, np * 8, hipMemcpyDeviceToHost, ctx->stream));
    return sync(ctx);
}

// Escaping matrices are recovered as one sub-batch from this many on, when
// none has more rows than kMaxRecoveryBatchRows.  Measured on 16 copies of
// one matrix (degree 200, 32 FP32 probes), one batched call against 16
// single-matrix calls: 0.9 against 12.8 ms at n = 4,096, 7.5 against
// 14.8 ms at 65,536, 16.0 against 19.6 ms at 110,592; eight copies of a
// 262,144-row matrix ran slower batched (55.1 against 39.4 ms).
constexpr int kMinRecoveryBatch = 16;
constexpr int64_t kMaxRecoveryBatchRows = 131072;

extern "C" kpm_status kpm_dos_pipeline_batched(kpm_ctx* ctx, int nmat, const kpm_csr* A, int lanczos_steps,
                                               uint64_t lanczos_seed, double margin, const kpm_moment_opts* o,
                                               kpm_damping damping, const double* x, int npts, double* phi,
                                               double* mu, double* lb, double* ub, int* attempts) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!A || !o || !x || !phi || !lb || !ub || npts < 0 || nmat < 1 || nmat > 65535)
        return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (damping != KPM_DAMP_NONE && damping != KPM_DAMP_JACKSON && damping != KPM_DAMP_LEARNED)
        return kpm_fail(ctx, KPM_ERR_ARG, "unknown damping kind");
    if (o->M < 0 || o->M > (1 << 20)) return kpm_fail(ctx, KPM_ERR_ARG, "bad M");
    if (damping == KPM_DAMP_LEARNED && o->M > 127)
        return kpm_fail(ctx, KPM_ERR_ARG, "learned damping is defined for M <= 127");
    const int M = o->M;
    kpm_status st = kpm_bounds_batched(ctx, nmat, A, lanczos_steps, lanczos_seed, margin, lb, ub);
    if (st != KPM_OK) return st;
    std::vector<int> tries((size_t)nmat, 1);
    std::vector<double> hmu;
    double* mup = mu;
    if (!mup) {
        hmu.assign((size_t)nmat * (M + 1), 0.0);
        mup = hmu.data();
    }
    std::vector<double> mx((size_t)nmat);
    st = kpm_moments_batched(ctx, nmat, A, lb, ub, o, mup, mx.data());
    if (st == KPM_ERR_SPECTRUM) {
        // Escape recovery as in kpm_moments_robust, for the escaping matrices
        // only, each with its own probes (seed opts->seed + m): first their
        // bounds with margin 4x (one batched call) and their moments, as one
        // sub-batch when enough of them escape and none is large (a few
        // large matrices run faster on the single-matrix path), else one by
        // one;
        // then, for any that still escape, the Gershgorin interval and the
        // single-matrix path.
        const double tol = o->precision == KPM_FP64 ? 1e-9 : 1e-4;
        std::vector<int> bad;
        for (int m = 0; m < nmat; ++m)
            if (!(mx[m] <= 1.0 + tol)) bad.push_back(m);
        const int nb = (int)bad.size();
        std::vector<kpm_csr> sub(nb);
        std::vector<uint64_t> seeds(nb);
        std::vector<double> l2(nb), u2(nb), mu2((size_t)nb * (M + 1)), mx2(nb);
        for (int i = 0; i < nb; ++i) {
            sub[i] = A[bad[i]];
            seeds[i] = o->seed + (uint64_t)bad[i];
        }
        if ((st = kpm_bounds_batched(ctx, nb, sub.data(), lanczos_steps, lanczos_seed, std::min(4.0 * margin, 0.4),
                                     l2.data(), u2.data())) != KPM_OK)
            return st;
        auto single_opts = [&](int m) {
            kpm_moment_opts om = *o;
            om.seed = o->seed + (uint64_t)m;
            om.block = 0;
            om.rows_per_block = 0;
            om.flags = 0;
            return om;
        };
        int64_t nmax_bad = 0;
        for (int m : bad) nmax_bad = std::max<int64_t>(nmax_bad, A[m].n);
        if (nb >= kMinRecoveryBatch && nmax_bad <= kMaxRecoveryBatchRows) {
            st = kpm_moments_batched_seeded(ctx, nb, sub.data(), l2.data(), u2.data(), o, seeds.data(), mu2.data(),
                                            mx2.data());
            if (st != KPM_OK && st != KPM_ERR_SPECTRUM) return st;
            for (int i = 0; i < nb; ++i)
                memcpy(mup + (size_t)bad[i] * (M + 1), mu2.data() + (size_t)i * (M + 1), (size_t)(M + 1) * 8);
        } else {
            for (int i = 0; i < nb; ++i) {
                const kpm_moment_opts om = single_opts(bad[i]);
                st = kpm_moments(ctx, &A[bad[i]], l2[i], u2[i], &om, mup + (size_t)bad[i] * (M + 1), nullptr);
                if (st != KPM_OK && st != KPM_ERR_SPECTRUM) return st;
                mx2[i] = st == KPM_OK ? 0.0 : HUGE_VAL;
            }
        }
        for (int i = 0; i < nb; ++i) {
            lb[bad[i]] = l2[i];
            ub[bad[i]] = u2[i];
            tries[bad[i]] = 2;
        }
        st = KPM_OK;
        for (int i = 0; i < nb && st == KPM_OK; ++i) {
            if (mx2[i] <= 1.0 + tol) continue;
            const int m = bad[i];
            double glo, ghi;
            if ((st = kpm_gershgorin(ctx, &A[m], &glo, &ghi)) != KPM_OK) return st;
            const double c = 0.5 * (glo + ghi);
            double d = 0.5 * (ghi - glo) / (1.0 - margin);
            d = std::max(d, std::max(margin, 1e-3) * std::max(fabs(c), 1.0));
            lb[m] = c - d;
            ub[m] = c + d;
            tries[m] = 3;
            const kpm_moment_opts om = single_opts(m);
            st = kpm_moments(ctx, &A[m], lb[m], ub[m], &om, mup + (size_t)m * (M + 1), nullptr);
        }
    }
    if (attempts) memcpy(attempts, tries.data(), (size_t)nmat * sizeof(int));
    if (st != KPM_OK) return st;
    // damping factors: one shared row, or one per matrix for the network
    std::vector<double> g;
    if (damping == KPM_DAMP_LEARNED) {
        constexpr int kIn = 128;
        std::vector<float> xin((size_t)nmat * kIn, 0.0f), gf((size_t)nmat * kIn);
        for (int m = 0; m < nmat; ++m)
            for (int k = 0; k <= M; ++k) xin[(size_t)m * kIn + k] = (float)mup[(size_t)m * (M + 1) + k];
        if ((st = kpm_mlp_forward(ctx, nmat, xin.data(), gf.data())) != KPM_OK) return st;
        g.resize((size_t)nmat * (M + 1));
        for (int m = 0; m < nmat; ++m) {
            for (int k = 0; k <= M; ++k) g[(size_t)m * (M + 1) + k] = gf[(size_t)m * kIn + k];
            g[(size_t)m * (M + 1)] = 1.0;
        }
    } else {
        g.resize((size_t)M + 1);
        if ((st = kpm_damping_factors(ctx, damping, M, nullptr, g.data())) != KPM_OK) return st;
    }
    return kpm_dos_batched(ctx, nmat, mup, g.data(), damping == KPM_DAMP_LEARNED ? 1 : 0, M, lb, ub, x, npts, phi);
}

extern "C" kpm_status kpm_dos_bins(kpm_ctx* ctx, const double* mu, const double* g, int M, double lb,
                                   double ub, const double* edges, int nbins, double* mass) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!mu || !g || !edges || !mass || M < 0 || nbins < 0) return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (!(isfinite(lb) && isfinite(ub) && ub > lb)) return kpm_fail(ctx, KPM_ERR_ARG, "need finite lb < ub");
    for (int i = 0; i < nbins; ++i)
        if (!(edges[i + 1] >= edges[i])) return kpm_fail(ctx, KPM_ERR_ARG, "edges must be non-decreasing");
    if (nbins == 0) return KPM_OK;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    void *mud, *gd, *ed, *md;
    kpm_status st = upload_series(ctx, mu, g, M, &mud, &gd);
    if (st != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "bins_e", (size_t)(nbins + 1) * 8, &ed)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "bins_m", (size_t)nbins * 8, &md)) != KPM_OK) return st;
    KPM_HIP(ctx, hipMemcpyAsync(ed, edges, (size_t)(nbins + 1) * 8, hipMemcpyHostToDevice, ctx->stream));
    const double c = 0.5 * (lb + ub), d = 0.5 * (ub - lb);
    KPM_HIP(ctx, launch_dos_bins(ctx->stream, (double*)mud, (double*)gd, M, c, d, (double*)ed, nbins, (double*)md));
    KPM_HIP(ctx, hipMemcpyAsync(mass, md, (size_t)nbins * 8, hipMemcpyDeviceToHost, ctx->stream));
    return sync(ctx);
}

extern "C" kpm_status kpm_rademacher(kpm_ctx* ctx, uint64_t seed, int64_t vec0, int nvec, int64_t n,
                                     int64_t ld, int precision, void* out_device) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!out_device || nvec < 0 || n < 0 || ld < nvec || vec0 < 0 || vec0 + nvec > ((int64_t)1 << 32) ||
        n > ((int64_t)1 << 32) || (precision != KPM_FP32 && precision != KPM_FP64))
        return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (n == 0 || nvec == 0) return KPM_OK;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    KPM_HIP(ctx, launch_rademacher(ctx->stream, seed, vec0, nvec, ld, n, precision, 0, out_device));
    return sync(ctx);
}

// ---------------------------------------------------------------- whole path
// Bounds, moments, damping and density in one call: the Lanczos bounds need
// one wait (their Ritz values are found on the host); everything after them
// -- the learned damping network included -- is enqueued back to back and
// waited for once.
extern "C" kpm_status kpm_dos_pipeline(kpm_ctx* ctx, const kpm_csr* A, int lanczos_steps, uint64_t lanczos_seed,
                                       double margin, const kpm_moment_opts* o, kpm_damping damping,
                                       const double* x, int npts, double* phi, double* mu, double* lb,
                                       double* ub) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!o || !x || !phi || !lb || !ub || npts < 0) return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    if (damping != KPM_DAMP_NONE && damping != KPM_DAMP_JACKSON && damping != KPM_DAMP_LEARNED)
        return kpm_fail(ctx, KPM_ERR_ARG, "unknown damping kind");
    // The first probe block does not depend on the bounds: it is filled while
    // the host waits for the Lanczos coefficients (same arguments, hence the
    // same block, as the fill moments_impl would otherwise launch).
    bool prefilled = false;
    auto prefill = [&]() -> kpm_status {
        const int maxb = o->precision == KPM_FP64 ? 128 : 256;
        if (o->nvec < 1 || o->nvec > (1 << 24) || o->block < 0 || o->block > maxb ||
            (o->precision != KPM_FP32 && o->precision != KPM_FP64) || o->rows_per_block < 0 ||
            o->rows_per_block > (1 << 20) || o->M < 0 || o->M > (1 << 20))
            return KPM_OK;  // moments_impl reports the bad argument
        const int b = o->block > 0 ? std::min(o->block, o->nvec) : default_block(o->nvec, o->precision);
        const BlockGeom g = make_geom(A->n, b, o->precision, o->rows_per_block);
        const int esz = o->precision == KPM_FP64 ? 8 : 4;
        // with KPM_FLAG_LOCALITY the block is that of the renumbered matrix
        const int32_t* rows = nullptr;
        if (o->flags & KPM_FLAG_LOCALITY) {
            if (!A->on_device) return KPM_OK;  // moments_impl fills it
            CsrDev D, R;
            kpm_status s1 = kpm_prepare_csr(ctx, A, o->precision, &D, "");
            if (s1 != KPM_OK) return KPM_OK;  // moments_impl reports it
            if ((s1 = kpm_locality_view(ctx, D, &R, &rows)) != KPM_OK) return s1;
        }
        void* X0;
        kpm_status s2 = kpm_ws(ctx, "X0", (size_t)A->n * g.ld * esz, &X0);
        if (s2 != KPM_OK) return s2;
        KPM_HIP(ctx, launch_rademacher(ctx->stream, o->seed, 0, b, g.ld, A->n, o->precision, 1, X0, rows));
        prefilled = true;
        return KPM_OK;
    };
    kpm_status st = bounds_impl(ctx, A, lanczos_steps, lanczos_seed, margin, lb, ub, prefill);
    if (st != KPM_OK) return st;
    MomentsPending P;
    if ((st = moments_impl(ctx, A, *lb, *ub, o, nullptr, nullptr, false, &P, prefilled)) != KPM_OK) return st;
    const int M = P.M;
    void *gd, *xd, *pd;
    if ((st = kpm_ws(ctx, "pipe_g", (size_t)(M + 1) * 8, &gd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dos_x", (size_t)std::max(npts, 1) * 8, &xd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "dos_phi", (size_t)std::max(npts, 1) * 8, &pd)) != KPM_OK) return st;
    std::vector<double> hg;  // host damping factors (none); alive until the final wait
    if (damping == KPM_DAMP_JACKSON) {
        KPM_HIP(ctx, launch_jackson(ctx->stream, M, (double*)gd));
    } else if (damping == KPM_DAMP_LEARNED) {
        // the network reads the device moments directly
        if ((st = kpm_learned_damping_device(ctx, M, (const double*)P.mud, (double*)gd)) != KPM_OK) return st;
    } else {
        hg.assign((size_t)M + 1, 1.0);
        KPM_HIP(ctx, hipMemcpyAsync(gd, hg.data(), hg.size() * 8, hipMemcpyHostToDevice, ctx->stream));
    }
    const double c = 0.5 * (*lb + *ub), d = 0.5 * (*ub - *lb);
    if (npts > 0) {
        KPM_HIP(ctx, hipMemcpyAsync(xd, x, (size_t)npts * 8, hipMemcpyHostToDevice, ctx->stream));
        KPM_HIP(ctx, launch_dos(ctx->stream, (const double*)P.mud, (const double*)gd, M, c, d, (const double*)xd,
                                npts, (double*)pd));
    }
    return moments_collect(ctx, P, mu, nullptr, (const double*)pd, (size_t)npts, phi);
}

// ---------------------------------------------------------------- profiling
extern "C" kpm_status kpm_profile_enable(kpm_ctx* ctx, int enable) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->prof = enable != 0;
    return KPM_OK;
}

extern "C" kpm_status kpm_profile_query(kpm_ctx* ctx, const char* kernel, int64_t* launches, double* total_ms) {
    if (!ctx || !kernel || !launches || !total_ms) return KPM_ERR_ARG;
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    kpm_prof_collect(ctx);
    auto it = ctx->prof_map.find(kernel);
    *launches = it == ctx->prof_map.end() ? 0 : it->second.launches;
    *total_ms = it == ctx->prof_map.end() ? 0.0 : it->second.total_ms;
    return KPM_OK;
}

extern "C" kpm_status kpm_profile_reset(kpm_ctx* ctx) {
    if (!ctx) return KPM_ERR_ARG;
    hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->prof_map) {
        kv.second.used = 0;
        kv.second.counts.clear();
        kv.second.launches = 0;
        kv.second.total_ms = 0.0;
    }
    return KPM_OK;
}
