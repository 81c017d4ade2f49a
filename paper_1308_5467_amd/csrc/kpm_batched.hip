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

// Step k also finishes step k - 1's dots: the workgroup that runs an mv's
// first table entry adds that mv's partials of step k - 1 (`prev`, the other
// half of a two-step partial buffer) over its entries in order, with the
// compensated sum of batched_reduce_kernel, so only two steps of partials
// are ever stored whatever the number of table entries.
template <typename TA, typename TV, bool FIRST, int G>
__global__ __launch_bounds__(kThreads) void batched_step_kernel(const BatchEntryDev* __restrict__ entries,
                                                                const BatchMvDev* __restrict__ mvs, int parity,
                                                                int ld, int lpr, int rpw, int rows_per_panel,
                                                                int stage, double* __restrict__ partial,
                                                                const double* __restrict__ prev,
                                                                const int32_t* __restrict__ e0,
                                                                const int32_t* __restrict__ e1,
                                                                double* __restrict__ dots_prev) {
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
    if (!FIRST && e == e0[E.mv]) {
        // loads in groups of 16 (one memory round trip each), sums in order
        const int width = 2 * ld, f1 = e1[E.mv];
        for (int t = threadIdx.x; t < width; t += kThreads) {
            double s = 0.0, c = 0.0;
            for (int f = e; f < f1; f += 16) {
                double x[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) x[u] = f + u < f1 ? prev[(int64_t)(f + u) * width + t] : 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (f + u < f1) bneumaier(s, c, x[u]);
            }
            dots_prev[(int64_t)E.mv * width + t] = s + c;
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

// dots[k][mv][t] = sum over the mv's table entries of partial[k][e][t], in order
// (launched for the last step only; the step kernels reduce the others).
__global__ __launch_bounds__(64) void batched_reduce_kernel(const double* __restrict__ partial, int nentries,
                                                            int width, const int32_t* __restrict__ e0,
                                                            const int32_t* __restrict__ e1, int nmv,
                                                            double* __restrict__ dots) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    const int k = blockIdx.y, mv = blockIdx.z;
    if (t >= width) return;
    double s = 0.0, c = 0.0;
    const double* src = partial + (int64_t)k * nentries * width + t;
    for (int e = e0[mv]; e < e1[mv]; ++e) bneumaier(s, c, src[(int64_t)e * width]);
    dots[((int64_t)k * nmv + mv) * width + t] = s + c;
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
    std::vector<BatchMvDev> mvs;  // host copy (alpha/beta/seed refreshed per call)
    void* mem = nullptr;          // one device allocation for everything below
    size_t mem_bytes = 0;
    BatchEntryDev* d_entries = nullptr;
    BatchMvDev* d_mvs = nullptr;
    int32_t* d_e0 = nullptr;
    int32_t* d_e1 = nullptr;
    double* d_partial = nullptr;
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

template <typename TA, typename TV>
hipError_t enqueue_batched(hipStream_t s, const BatchPlan& P) {
    dim3 fill_grid(256, P.nmv);
    batched_fill_kernel<TV><<<fill_grid, 256, 0, s>>>(P.d_mvs, P.ld);
    const size_t width = 2 * (size_t)P.ld;
    // partials of step k go to half k & 1; step k reduces step k - 1's half
    for (int k = 0; k < P.K; ++k) {
        double* pk = P.d_partial + (size_t)(k & 1) * P.nentries * width;
        if (k == 0)
            batched_step_kernel<TA, TV, true, 7><<<P.nentries, kThreads, 0, s>>>(
                P.d_entries, P.d_mvs, 0, P.ld, P.lpr, P.rpw, P.rows, P.stage, pk, nullptr, P.d_e0, P.d_e1,
                nullptr);
        else
            batched_step_kernel<TA, TV, false, 7><<<P.nentries, kThreads, 0, s>>>(
                P.d_entries, P.d_mvs, k & 1, P.ld, P.lpr, P.rpw, P.rows, P.stage, pk,
                P.d_partial + (size_t)((k - 1) & 1) * P.nentries * width, P.d_e0, P.d_e1,
                P.d_dots + (size_t)(k - 1) * P.nmv * width);
    }
    if (P.K > 0) {  // the last step's dots
        dim3 rg((unsigned)((width + 63) / 64), 1, P.nmv);
        batched_reduce_kernel<<<rg, 64, 0, s>>>(P.d_partial + (size_t)((P.K - 1) & 1) * P.nentries * width,
                                                P.nentries, (int)width, P.d_e0, P.d_e1, P.nmv,
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
    P.exec = nullptr;
    P.graph = nullptr;
    P.mem = nullptr;
    P.mem_bytes = 0;
}

}  // namespace

struct kpm_batch_state {
    BatchPlan plan;
};

void kpm_batch_free(kpm_ctx* ctx) {
    if (!ctx->batch) return;
    hipStreamSynchronize(ctx->batch->plan.gstream ? ctx->batch->plan.gstream : ctx->stream);
    free_plan(ctx->batch->plan);
    if (ctx->batch->plan.gstream) hipStreamDestroy(ctx->batch->plan.gstream);
    delete ctx->batch;
    ctx->batch = nullptr;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

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

extern "C" kpm_status kpm_moments_batched(kpm_ctx* ctx, int nmat, const kpm_csr* A, const double* lb,
                                          const double* ub, const kpm_moment_opts* o, double* mu,
                                          double* max_abs_mu) {
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
    const int b = o->block > 0 ? std::min(o->block, nvec) : kpm_default_block(nvec, o->precision);
    int64_t nmax = 0;
    for (int m = 0; m < nmat; ++m) nmax = std::max<int64_t>(nmax, D[m].n);
    const BlockGeom g = make_geom(nmax, b, o->precision, o->rows_per_block);
    const int esz = o->precision == KPM_FP64 ? 8 : 4;
    if ((uint64_t)nmax * g.ld * esz >= (1ull << 32))
        return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "batched probe blocks must be smaller than 4 GiB");
    const int nvb = (nvec + b - 1) / b;
    if ((int64_t)nmat * nvb > 65535)
        return kpm_fail(ctx, KPM_ERR_UNSUPPORTED, "at most 65535 (matrix, probe block) pairs per batch");

    BatchShape shape;
    for (int m = 0; m < nmat; ++m) {
        shape.ptrs.push_back((uintptr_t)D[m].rp);
        shape.ptrs.push_back((uintptr_t)D[m].ci);
        shape.ptrs.push_back((uintptr_t)D[m].val);
        shape.dims.push_back(D[m].n);
        shape.dims.push_back(D[m].nnz);
    }
    const int64_t tail[] = {nmat, M, nvec, b, o->precision, D[0].val_f64, g.rows_per_block};
    shape.dims.insert(shape.dims.end(), tail, tail + 7);

    if (!ctx->batch) ctx->batch = new kpm_batch_state();
    BatchPlan& P = ctx->batch->plan;
    if (!P.gstream) KPM_HIP(ctx, hipStreamCreateWithFlags(&P.gstream, hipStreamNonBlocking));
    const bool reuse = P.mem && P.shape == shape;
    if (!reuse) {
        KPM_HIP(ctx, hipStreamSynchronize(P.gstream));
        free_plan(P);
        P.shape = shape;
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
        // work table: workgroups per mv proportional to its bytes of work,
        // and at least kMinEntriesPerMv (or one per panel) for every mv
        const int resident = o->precision == KPM_FP64
                                 ? (P.val_f64 ? batched_resident<double, double>() : batched_resident<float, double>())
                                 : batched_resident<float, float>();
        const int target = std::max(resident, 256);
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
        const size_t o_dots = off;
        off += align256((size_t)std::max(P.K, 1) * P.nmv * 2 * g.ld * 8);
        const size_t o_zeta = off;
        off += align256((size_t)nmat * nvec * (M + 1) * 8);
        const size_t o_mu = off;
        off += align256((size_t)nmat * (M + 1) * 8);
        const size_t o_max = off;
        off += align256((size_t)nmat * 8);
        if (hipMalloc(&P.mem, off) != hipSuccess) {
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
    // per-call scalars
    for (int m = 0; m < nmat; ++m) {
        const double c = 0.5 * (lb[m] + ub[m]), d = 0.5 * (ub[m] - lb[m]);
        for (int vb = 0; vb < nvb; ++vb) {
            BatchMvDev& x = P.mvs[m * nvb + vb];
            x.alpha = 2.0 / d;
            x.beta = -2.0 * c / d;
            x.seed = o->seed + (uint64_t)m;
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
    KPM_HIP(ctx, hipMemcpyAsync(mu, P.d_mu, (size_t)nmat * (M + 1) * 8, hipMemcpyDeviceToHost, P.gstream));
    KPM_HIP(ctx, hipMemcpyAsync(maxabs.data(), P.d_maxabs, (size_t)nmat * 8, hipMemcpyDeviceToHost, P.gstream));
    KPM_HIP(ctx, hipStreamSynchronize(P.gstream));
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
