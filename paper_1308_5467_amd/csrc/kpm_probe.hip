// Achievable-bandwidth probe: a plain streaming copy (16-byte loads and
// stores, grid-stride) used as the practical denominator beside the HBM
// specification peak, and as the calibration kernel for the byte counters.
#include <hip/hip_runtime.h>

#include "kpm_internal.h"

namespace kpm {

// Each thread moves four 16-byte elements per iteration (four loads in
// flight), strided by the grid so every wavefront access is contiguous.
__global__ __launch_bounds__(256) void copy_probe_kernel(const float4* __restrict__ src,
                                                         float4* __restrict__ dst, int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n4; i += stride) dst[i] = src[i];
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
    hipDeviceProp_t prop;
    KPM_HIP(ctx, hipGetDeviceProperties(&prop, ctx->device));
    const int grid = prop.multiProcessorCount * 8;
    kpm::copy_probe_kernel<<<grid, 256, 0, ctx->stream>>>((const float4*)a, (float4*)b, n4);  // warm-up
    KPM_HIP(ctx, hipGetLastError());
    hipEvent_t e0, e1;
    KPM_HIP(ctx, hipEventCreate(&e0));
    KPM_HIP(ctx, hipEventCreate(&e1));
    hipEventRecord(e0, ctx->stream);
    for (int i = 0; i < iters; ++i) {
        kpm_prof_begin(ctx, "copy_probe");
        kpm::copy_probe_kernel<<<grid, 256, 0, ctx->stream>>>((const float4*)(i & 1 ? b : a),
                                                              (float4*)(i & 1 ? a : b), n4);
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
