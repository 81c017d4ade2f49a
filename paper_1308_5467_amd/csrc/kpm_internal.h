// Internal declarations of the KPM library: context, workspace and the
// launch wrappers of the device kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "kpm.h"

namespace kpm {

// Device view of a CSR matrix (int32 indices).
struct CsrDev {
    const int32_t* rp = nullptr;
    const int32_t* ci = nullptr;
    const void* val = nullptr;
    int val_f64 = 0;
    int32_t n = 0;
    int32_t nnz = 0;
};

// Geometry of one vector block on the device: `ld` values per row
// (a multiple of the per-lane pack width), `lpr` lanes per row, `rpw` rows
// per 64-wide wavefront, `rows_per_block` rows per workgroup (a multiple of
// the 4 * rpw rows one workgroup pass covers), `nblocks` workgroups.
struct BlockGeom {
    int ld = 0, lpr = 0, rpw = 0, rows_per_block = 0, nblocks = 0;
    int gather = 7;  // single-matrix step: CSR entries per gather batch (4, 7 or 8)
};

constexpr int kWaves = 4;        // wavefronts per workgroup of the step kernels
constexpr int kThreads = 64 * kWaves;

BlockGeom make_geom(int64_t n, int ncols, int precision, int rows_per_block_hint);
// Probe-block width used when the caller passes 0: min(nvec, 64) for FP32,
// min(nvec, 32) for FP64 (256-byte probe rows).
int kpm_default_block(int nvec, int precision);

// ---------------------------------------------------------------- moments
// rows (nullable): row i of the block takes entry rows[i] of each probe
// (a renumbered matrix's probes at the original indices).
hipError_t launch_rademacher(hipStream_t s, uint64_t seed, int64_t vec0, int ncols, int64_t ld,
                             int64_t n, int precision, int zero_pad, void* out, const int32_t* rows = nullptr);
// Workgroups every step launch of this geometry uses (= partial rows per step).
int cheb_step_grid(const CsrDev& A, int precision, const BlockGeom& g);
// Legendre moments from Chebyshev moments: a[0..M] connection weights
// (host), then per probe row zetaL[n] = sum_k (2 - [n = 2k]) a_k a_{n-k} zeta[n-2k].
void legendre_connection_weights(int M, double* a);
hipError_t launch_cheb_to_legendre(hipStream_t s, const double* zeta, int nvec, int M, const double* a,
                                   double* out);
// Sign bits of probes vec0 .. vec0+ncols-1 of `seed` into [n][sw] words
// (bit j of word w: entry of probe vec0 + 32 w + j is -1).
hipError_t launch_sign_bits(hipStream_t s, uint64_t seed, int64_t vec0, int ncols, int64_t n, int sw,
                            uint32_t* out);
// Per-probe normalised Legendre moments of one probe block from the reduced
// dots of the Legendre recurrence: zeta[(vec0 + j) * (M+1) + k] = 1 for
// k = 0, dots[(k-1) * 2 ld + j] / n for k = 1..M.
hipError_t launch_legendre_assemble(hipStream_t s, const double* dots, int ld, int ncols, int M, double n,
                                    int64_t vec0, double* zeta);
// Legendre step of Algorithm DGL (with a non-null LegStep and first ==
// false): U <- alpha A V + beta V + gam U, first dot against v_0 given by
// its sign bits sgn ([n][sw] words).
struct LegStep {
    double gam;
    const uint32_t* sgn;
    int sw;
};
hipError_t launch_cheb_step(hipStream_t s, const CsrDev& A, int precision, bool first,
                            const BlockGeom& g, int grid, const void* V, void* U, double alpha,
                            double beta, double* partial, bool reverse, const LegStep* leg = nullptr);
hipError_t launch_reduce_partials(hipStream_t s, const double* partial, int nblocks, int width,
                                  int K, double* dots);
hipError_t launch_assemble(hipStream_t s, const double* dots, int K, int ld, int ncols, int M,
                           double n, int64_t vec0, double* zeta_norm);
hipError_t launch_mean_moments(hipStream_t s, const double* zeta_norm, int nvec, int M, double* mu);
hipError_t launch_convert_f64_to_f32(hipStream_t s, const double* in, float* out, int64_t count);
hipError_t launch_validate_csr(hipStream_t s, const CsrDev& A, int* flags);

// ---------------------------------------------------------------- bounds
struct LanczosWork {
    double* Q = nullptr;        // [m x n] Lanczos vectors
    double* w = nullptr;        // [2 x n] residual ping-pong buffers
    double* coef = nullptr;     // alpha[64], beta[64], two projection vectors [32]
    double* partial = nullptr;  // [3 x 32 x nblk] per-workgroup partial sums
    int nblk = 0;               // workgroups
    int chunk = 0;              // rows per workgroup = 256 * rows per thread
};
int lanczos_rows_per_thread(int64_t n);
hipError_t launch_lanczos(hipStream_t s, const CsrDev& A, int m, uint64_t seed, LanczosWork& W);
hipError_t launch_gershgorin(hipStream_t s, const CsrDev& A, double* out /* [2 * nblk] */, int nblk);

// The same Lanczos run for many matrices (kpm_bounds_batched).  Per matrix:
// steps m = min(steps, n), row chunk and workgroup count as for one matrix,
// and the offsets (in doubles) of its Lanczos vectors (m x n), residual
// buffers (2 x n) and partials in buffers shared by all matrices; its
// coefficients go to coef + 256 * index, laid out as for one matrix.  The
// descriptor and work tables take table_bytes of device memory, built in a
// host staging buffer of the same size (page-locked: the upload is
// asynchronous).
struct LanczosBatchLayout {
    std::vector<int> m, nblk, chunk;
    std::vector<int64_t> q_off, w_off, part_off;
    int64_t q_total = 0, w_total = 0, part_total = 0;
    size_t desc_bytes = 0, tab_bytes = 0, table_bytes = 0;
};
void lanczos_batch_layout(int nmat, const CsrDev* A, int steps, LanczosBatchLayout* L);
// Offset in `part` of matrix m's free [2 x nblk] block (Gershgorin output).
int64_t lanczos_batch_gershgorin_off(const LanczosBatchLayout& L, int m);
// With s2 (and its fork / join events) the launch groups alternate between
// s and s2, whose chains are independent; s waits for s2 at the end.
hipError_t launch_lanczos_batched(hipStream_t s, int nmat, const CsrDev* A, uint64_t seed,
                                  const LanczosBatchLayout& L, double* Q, double* w, double* coef, double* part,
                                  void* dev_tables, void* host_stage, int* launches, hipStream_t s2 = nullptr,
                                  hipEvent_t fork = nullptr, hipEvent_t join = nullptr);

// ---------------------------------------------------------------- damping / density
hipError_t launch_jackson(hipStream_t s, int M, double* g);
hipError_t launch_dos(hipStream_t s, const double* mu, const double* g, int M, double c, double d,
                      const double* x, int npts, double* phi);
// Densities of nmat matrices: rows of mu [nmat][M+1], g (row stride
// g_stride, 0 for one shared row), x and phi [nmat][npts]; lb, ub [nmat].
hipError_t launch_dos_batched(hipStream_t s, int nmat, const double* mu, const double* g, int64_t g_stride, int M,
                              const double* lb, const double* ub, const double* x, int npts, double* phi);
hipError_t launch_dos_bins(hipStream_t s, const double* mu, const double* g, int M, double c,
                           double d, const double* edges, int nbins, double* mass);

}  // namespace kpm

// ---------------------------------------------------------------- context
struct kpm_dev_buf {
    void* p = nullptr;
    size_t cap = 0;
};

struct kpm_prof_entry {
    std::vector<hipEvent_t> ev;  // pairs (start, stop) recorded but not yet read
    size_t used = 0;             // number of events in use
    std::vector<int> counts;     // launches covered by each recorded pair
    int64_t launches = 0;
    double total_ms = 0.0;
};

struct kpm_batch_state;     // batched-moments plan and captured graph (kpm_batched.hip)
struct kpm_locality_state;  // renumbered structure of the last matrix (kpm_locality.hip)

struct kpm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::map<std::string, kpm_dev_buf> bufs;  // grow-only device workspace by role
    std::vector<double> host_scratch;
    void* pinned = nullptr;  // grow-only page-locked host staging for device-to-host copies
    size_t pinned_cap = 0;
    hipEvent_t copy_done = nullptr;  // marks a device-to-host copy the host waits for alone
    // a second stream (default priority) for independent launch chains of
    // one call, and the events that fork it from and join it to `stream`
    hipStream_t aux = nullptr;
    hipEvent_t aux_fork = nullptr, aux_join = nullptr;
    // damping network
    bool mlp_ready = false;
    kpm_dev_buf mlp_params;
    // the blur operator held in this context's "mlp_blur" workspace: the
    // sigma it was built for (< 0: not built) and the buffer it was built in
    float mlp_blur_sigma = -1.0f;
    const void* mlp_blur_buf = nullptr;
    kpm_batch_state* batch = nullptr;
    kpm_locality_state* loc = nullptr;
    // profiling
    bool prof = false;
    std::map<std::string, kpm_prof_entry> prof_map;
};

// Device view of a kpm_csr (host arrays copied into role-named workspace,
// FP64 values rounded to FP32 for the FP32 path) and its validation.
kpm_status kpm_prepare_csr(kpm_ctx* ctx, const kpm_csr* A, int precision, kpm::CsrDev* out, const char* tag);
kpm_status kpm_validate_csr(kpm_ctx* ctx, const kpm::CsrDev& D);
// kpm_moments_batched with matrix m's probes drawn from seeds[m] (host
// [nmat]) instead of opts->seed + m; seeds NULL gives the public call.
kpm_status kpm_moments_batched_seeded(kpm_ctx* ctx, int nmat, const kpm_csr* A, const double* lb, const double* ub,
                                     const kpm_moment_opts* o, const uint64_t* seeds, double* mu,
                                     double* max_abs_mu);
void kpm_batch_free(kpm_ctx* ctx);
// KPM_FLAG_LOCALITY: the matrix renumbered along a Morton curve of its grid
// when kpm_locality_order finds one (*out = the renumbered view, *orig = the
// original index of each of its rows), else *out = A and *orig = NULL.
// Each refresh enqueues a checksum of the current structure and gathers the
// current values; refresh = false returns the copy as refreshed earlier in
// the same call (nothing enqueued).
kpm_status kpm_locality_view(kpm_ctx* ctx, const kpm::CsrDev& A, kpm::CsrDev* out, const int32_t** orig,
                             bool refresh = true);
void kpm_locality_free(kpm_ctx* ctx);
// After a call that used kpm_locality_view has been waited for: KPM_ERR_ARG
// (and the cached copy dropped) when the matrix's structure at the cached
// address is not the one the copy was built from.
kpm_status kpm_locality_check(kpm_ctx* ctx);

// Learned damping (damping network on the device); host mu/g arrays.
kpm_status kpm_learned_damping(kpm_ctx* ctx, int M, const double* mu, double* g);
// The same from device moments into device factors, enqueued without a wait.
kpm_status kpm_learned_damping_device(kpm_ctx* ctx, int M, const double* mu_dev, double* g_dev);

// Resolves the no-allocation entry point's scratch array on `device` (which
// the caller has made current); called once per context creation.
void kpm_noalloc_attach(int device);

// Grow-only workspace allocation by role name.
kpm_status kpm_ws(kpm_ctx* ctx, const char* role, size_t bytes, void** out);
// Grow-only page-locked host buffer of at least `bytes` (waits for the
// context's stream before replacing a smaller one).
kpm_status kpm_pinned(kpm_ctx* ctx, size_t bytes, void** out);
kpm_status kpm_fail(kpm_ctx* ctx, kpm_status st, const std::string& msg);
kpm_status kpm_hip_fail(kpm_ctx* ctx, hipError_t e, const char* what);
// Profiling helpers: bracket a run of `launches` back-to-back launches of
// one kernel with an event pair when profiling is on.
void kpm_prof_begin(kpm_ctx* ctx, const char* kernel);
void kpm_prof_end(kpm_ctx* ctx, const char* kernel, int launches);
void kpm_prof_begin_on(kpm_ctx* ctx, const char* kernel, hipStream_t s);
void kpm_prof_end_on(kpm_ctx* ctx, const char* kernel, hipStream_t s, int launches);
// Fold recorded events into the totals (call after a stream sync).
void kpm_prof_collect(kpm_ctx* ctx);

#define KPM_HIP(ctx, call)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return kpm_hip_fail(ctx, e_, #call); \
    } while (0)
