// Achievable-bandwidth probe: a plain streaming copy (16-byte non-temporal
// loads and stores) used as the practical denominator beside the HBM
// specification peak, and as the calibration kernel for the byte counters.
#include <hip/hip_runtime.h>

#include "kpm_internal.h"

namespace kpm {

// One 16-byte element per thread with non-temporal loads and stores, one
// workgroup per 4 KiB: the fastest plain copy measured on MI355X (6.6 TB/s
// read + write for 1 GiB, against 4.4-5.9 TB/s for grid-stride loops of 1-8
// elements per thread on 4-256 workgroups per CU, and 6.2 TB/s with cached
// stores).
typedef float probe_f4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy_probe_kernel(const probe_f4* __restrict__ src,
                                                         probe_f4* __restrict__ dst, int64_t n4) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n4) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace kpm

extern "C" kpm_status kpm_hbm_copy_probe(kpm_ctx* ctx, int64_t bytes, int iters, double* gbs) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!gbs || bytes < 4096 || iters < 1 || bytes > ((int64_t)1 << 36))
        return kpm_fail(ctx, KPM_ERR_ARG, "need bytes in [4 KiB, 64 GiB], iters >= 1");
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t n4 = bytes / 16;
    void *a, *b;
    kpm_status st;
    if ((st = kpm_ws(ctx, "probe_a", (size_t)n4 * 16, &a)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "probe_b", (size_t)n4 * 16, &b)) != KPM_OK) return st;
    KPM_HIP(ctx, hipMemsetAsync(a, 0, (size_t)n4 * 16, ctx->stream));
    const int64_t grid = (n4 + 255) / 256;  // <= 2^24 for 64 GiB
    kpm::copy_probe_kernel<<<(unsigned)grid, 256, 0, ctx->stream>>>((const kpm::probe_f4*)a, (kpm::probe_f4*)b,
                                                                   n4);  // warm-up
    KPM_HIP(ctx, hipGetLastError());
    hipEvent_t e0, e1;
    KPM_HIP(ctx, hipEventCreate(&e0));
    KPM_HIP(ctx, hipEventCreate(&e1));
    hipEventRecord(e0, ctx->stream);
    for (int i = 0; i < iters; ++i) {
        kpm_prof_begin(ctx, "copy_probe");
        kpm::copy_probe_kernel<<<(unsigned)grid, 256, 0, ctx->stream>>>(
            (const kpm::probe_f4*)(i & 1 ? b : a), (kpm::probe_f4*)(i & 1 ? a : b), n4);
        kpm_prof_end(ctx, "copy_probe", 1);
    }
    hipEventRecord(e1, ctx->stream);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return kpm_hip_fail(ctx, e, "copy probe timing");
    kpm_prof_collect(ctx);
    *gbs = 2.0 * (double)n4 * 16.0 * iters / (ms * 1e-3) / 1e9;
    return KPM_OK;
}
