/*
 * kpm.h -- C ABI of the MI355X (gfx950) kernel polynomial method library.
 *
 * The library estimates the density of states (DOS) of a real symmetric
 * sparse matrix A with the kernel polynomial method (KPM) as described by
 * Lin, Saad & Yang, "Approximating spectral densities of large matrices"
 * (SIAM Review 58(1), 2016; arXiv:1308.5467), section 3.1.1 and Appendix A.
 * The problem statement is that of Algorithm 1: given A, evaluation points
 * and a degree M, return the approximate DOS at those points.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - All functions return a kpm_status; nothing is thrown across the ABI.
 *    On failure a message is available from kpm_last_error(ctx).
 *  - Small arrays (moments, damping factors, points, outputs) are HOST
 *    pointers owned by the caller.  The call copies what it needs and has
 *    written every output when it returns (it synchronises its stream).
 *  - The sparse matrix is passed as a borrowed kpm_csr.  With on_device = 1
 *    its arrays are device pointers on the context's device and are used in
 *    place for the duration of the call; with on_device = 0 they are host
 *    pointers and are copied into context-owned device memory.
 *  - A context owns a HIP stream reference, grow-only device workspace and
 *    the damping network's weights.  One context must not be used from two
 *    threads at once.
 *  - Moments are normalised:  mu[k] = zeta_k / n  with
 *    zeta_k = (1/nvec) sum_l v_l^T T_k(B) v_l   (eqs. (nuk), (muEst)),
 *    B = (A - cI)/d, c = (lb+ub)/2, d = (ub-lb)/2  (eq. (cd)).  Hence
 *    mu[0] = 1, and the (2 - delta_k0)/pi factor of eq. (expmu) is applied
 *    inside kpm_dos / kpm_dos_bins.
 *  - Probe vectors are Rademacher vectors: entry i of probe vector l is -1
 *    when the top bit of output number ((l << 32) | i) + 1 of the SplitMix64
 *    sequence started from `seed` is set, +1 otherwise.  They satisfy the
 *    condition E[v] = 0, E[v v^T] = I of Theorem 1.
 */
#ifndef KPM_H
#define KPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KPM_OK = 0,
    KPM_ERR_ARG = -1,         /* invalid argument or malformed CSR            */
    KPM_ERR_ALLOC = -2,       /* device allocation failed                     */
    KPM_ERR_HIP = -3,         /* a HIP runtime call failed                    */
    KPM_ERR_SPECTRUM = -4,    /* spectrum escaped [lb, ub]: |zeta_k| > n or non-finite */
    KPM_ERR_NOCONV = -5,      /* eigen-solver of the Lanczos matrix did not converge */
    KPM_ERR_UNSUPPORTED = -6, /* option combination not supported             */
    KPM_ERR_NOMODEL = -7      /* learned damping requested but no weights set  */
} kpm_status;

typedef struct kpm_ctx kpm_ctx;

/* Borrowed CSR matrix.  Columns must be sorted and unique within a row;
 * the matrix must be symmetric (not checked on the hot path). */
typedef struct {
    int64_t n;               /* rows = columns, 1 <= n < 2^31                */
    int64_t nnz;             /* stored entries, row_ptr[n]                    */
    const int32_t* row_ptr;  /* [n + 1], row_ptr[0] = 0, non-decreasing       */
    const int32_t* col_idx;  /* [nnz], 0 <= col < n                           */
    const void* val;         /* [nnz] float (val_is_f64 = 0) or double (= 1) */
    int32_t val_is_f64;
    int32_t on_device;       /* 1: device pointers; 0: host pointers          */
} kpm_csr;

enum {
    KPM_FP32 = 0, /* FP32 matrix values and vectors, FP32 SpMM products,
                     FP64 recurrence combination and FP64 dot products      */
    KPM_FP64 = 1  /* FP64 everywhere                                       */
};

typedef struct {
    int32_t M;          /* degree: moments mu_0 .. mu_M are returned, M >= 0   */
    int32_t nvec;       /* number of probe vectors, >= 1                       */
    int32_t block;      /* probe vectors per device block, 0 = library choice
                           (64 FP32 or 32 FP64: 256-byte probe rows);
                           at most 256 (FP32) or 128 (FP64)                    */
    int32_t precision;  /* KPM_FP32 or KPM_FP64                                */
    uint64_t seed;      /* probe-vector seed                                   */
    int32_t validate;   /* 1: check the CSR structure and values first          */
    int32_t rows_per_block; /* row-panel height per workgroup, 0 = library choice */
    int32_t flags;      /* KPM_FLAG_* bits, 0 = defaults                        */
} kpm_moment_opts;

enum {
    KPM_FLAG_NO_GRAPH = 1, /* kpm_moments_batched: launch directly instead of
                              replaying the captured HIP graph                */
    KPM_FLAG_GATHER4 = 2,  /* kpm_moments: gather a row's CSR entries in
                              batches of 4 (fewest registers)                */
    KPM_FLAG_GATHER8 = 4,  /* kpm_moments: batches of 8                      */
    KPM_FLAG_GATHER7 = 8,  /* kpm_moments: batches of 7 (the default: one
                              round trip per 7-point stencil row at 5
                              wavefronts per SIMD); the GATHER flags override
                              the KPM_TUNE environment default               */
    KPM_FLAG_BATCH_STREAM = 32,   /* kpm_moments_batched: stream every probe
                              block through device memory (one launch per
                              step) even when the on-chip path applies     */
    KPM_FLAG_BATCH_RESIDENT = 64, /* kpm_moments_batched: the on-chip path
                              (KPM_ERR_UNSUPPORTED when a matrix is too
                              large for it)                                 */
    KPM_FLAG_LOCALITY = 128,      /* kpm_moments, kpm_legendre_moments,
                              kpm_dos_pipeline, kpm_slq (the Lanczos run on
                              P A P^T from P v has the same tridiagonal
                              matrix), kpm_autotune: when the matrix comes
                              from a 2D or 3D grid numbered lexicographically
                              (found by kpm_locality_order), run on it
                              renumbered along the grid's Morton curve,
                              probes at the original indices: the same
                              moments up to rounding, plane-apart neighbours
                              close in the probe block.  The renumbered
                              structure is built on the host (the whole CSR
                              is checked there first: KPM_ERR_ARG if
                              malformed) and cached in the context per
                              matrix address, sizes and value type; values
                              are re-read at every call.  A structure
                              rewritten in place at the same address is
                              detected by a checksum when the call's results
                              are collected (KPM_ERR_ARG) and the copy is
                              rebuilt on the next call.  Not accepted by
                              kpm_moments_noalloc (the copy is allocated) or
                              with KPM_FLAG_LEGENDRE_RECURRENCE              */
    KPM_FLAG_LEGENDRE_RECURRENCE = 16 /* kpm_legendre_moments: run the
                              Legendre three-term recurrence of Algorithm DGL
                              (M sparse products per block) instead of
                              converting Chebyshev moments                    */
};

typedef enum {
    KPM_DAMP_NONE = 0,    /* g_k = 1                                            */
    KPM_DAMP_JACKSON = 1, /* Jackson factors, Appendix A eq. (jackson)          */
    KPM_DAMP_LEARNED = 2  /* damping network (requires weights, M <= 127)       */
} kpm_damping;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the context. */
kpm_status kpm_create(int device, void* hip_stream, kpm_ctx** out);
kpm_status kpm_destroy(kpm_ctx* ctx);
/* Change the stream later calls enqueue on. */
kpm_status kpm_set_stream(kpm_ctx* ctx, void* hip_stream);
/* Message of the last failure on this context ("" if none); valid until the next call. */
const char* kpm_last_error(const kpm_ctx* ctx);

/*
 * kpm_bounds -- lower and upper bounds of the spectrum of A (section 3.1.1,
 * the paragraph after eq. (cd)).  Runs `steps` Lanczos steps in FP64 on the
 * device (start vector: probe vector 2^31 - 1 of `seed`, normalised; each
 * new vector orthogonalised against all previous ones by one classical
 * Gram-Schmidt pass), takes the extreme Ritz
 * values theta_1, theta_k of the tridiagonal matrix and widens each by its
 * residual norm beta_k |z_{k,j}|.  On breakdown the Gershgorin hull is merged
 * in.  The interval [lb0, ub0] is finally widened so that it maps into
 * [-(1 - margin), 1 - margin]:  c = (lb0+ub0)/2,  d = (ub0-lb0)/(2(1-margin)),
 * d >= margin * max(|c|, 1);  *lb = c - d,  *ub = c + d (with margin 0, an
 * interval of zero width -- a 1 x 1 matrix, say -- gets d = 1 instead).
 * steps in [1, 32] (capped at n); margin in [0, 0.5).
 */
kpm_status kpm_bounds(kpm_ctx* ctx, const kpm_csr* A, int steps, uint64_t seed,
                      double margin, double* lb, double* ub);

/*
 * kpm_bounds_batched -- kpm_bounds for nmat matrices in one launch sequence
 * (section 3.1.1, as for kpm_bounds): lb[m], ub[m] are bitwise the values
 * kpm_bounds(A[m], steps, seed, margin) returns (every matrix uses the same
 * start-vector seed; same per-matrix arithmetic and summation order).  Per
 * Lanczos step, one launch of each kind covers all matrices of like size
 * class and value type, instead of four launches per matrix; the m x m
 * tridiagonal problems are solved on up to 16 host threads.  A[m].on_device
 * must be 1 (value types may differ between matrices); lb, ub: host
 * [nmat].  nmat in [1, 2^20]; steps in [1, 32] (capped at each n); margin in
 * [0, 0.5).  Device memory kept by the context (grow-only): the Lanczos
 * vectors of all matrices, sum of min(steps, n_m) * n_m doubles (3 GB for
 * 9,216 matrices of n = 2,048 at 20 steps), plus 2 n_m doubles each.  Errors
 * as kpm_bounds, the message naming the first failing matrix; no output is
 * written then.
 */
kpm_status kpm_bounds_batched(kpm_ctx* ctx, int nmat, const kpm_csr* A, int steps, uint64_t seed,
                              double margin, double* lb, double* ub);

/*
 * kpm_gershgorin -- the Gershgorin hull [min_i a_ii - sum_j!=i |a_ij|,
 * max_i a_ii + sum_j!=i |a_ij|], which always contains the spectrum.
 */
kpm_status kpm_gershgorin(kpm_ctx* ctx, const kpm_csr* A, double* lo, double* hi);

/*
 * kpm_moments -- normalised stochastic Chebyshev moments mu[0..M] of
 * B = (A - cI)/d (Algorithm 1; eqs. (nuk), (3term), (muEst)), using the
 * product identity T_{p+q} = 2 T_p T_q - T_{|p-q|} (Appendix A) so that
 * ceil(M/2) sparse products per probe block give all M+1 moments:
 *   zeta_{2k}   = 2 v_k^T v_k     - zeta_0,
 *   zeta_{2k+1} = 2 v_{k+1}^T v_k - zeta_1.
 * mu:          host [M+1], written.
 * mu_per_vec:  host [nvec * (M+1)] or NULL; row l holds v_l^T T_k(B) v_l / n.
 * Returns KPM_ERR_SPECTRUM (after writing the outputs) when a per-vector
 * moment is non-finite or exceeds 1 in magnitude beyond rounding, i.e. the
 * spectrum of A is not inside [lb, ub].
 */
kpm_status kpm_moments(kpm_ctx* ctx, const kpm_csr* A, double lb, double ub,
                       const kpm_moment_opts* opts, double* mu, double* mu_per_vec);

/*
 * kpm_legendre_moments -- the stochastic Legendre moments of Algorithm DGL
 * (section 3.1.3) and of KPM with Legendre polynomials (Appendix A):
 *   mu[k] = (1/nvec) sum_l v_l^T L_k(B) v_l / n,   k = 0..M,
 * for the same probes, bounds, options, layouts and errors as kpm_moments
 * (mu_per_vec nullable, [nvec x (M+1)]).  They are computed from the
 * Chebyshev moments of the fused step (ceil(M/2) sparse products per
 * probe block) through L_n = sum_{k <= n/2} (2 - [n = 2k]) a_k a_{n-k} T_{n-2k},
 * a_m = (2m)!/(4^m (m!)^2): non-negative weights summing to 1, so the
 * result carries the Chebyshev moments' accuracy (FP32 path 1e-5, FP64 path
 * 1e-12).  The paper's Legendre recurrence, one sparse product per moment,
 * runs in the fused step instead with KPM_FLAG_LEGENDRE_RECURRENCE.
 */
kpm_status kpm_legendre_moments(kpm_ctx* ctx, const kpm_csr* A, double lb, double ub,
                                const kpm_moment_opts* opts, double* mu, double* mu_per_vec);

/*
 * kpm_moments_noalloc -- kpm_moments for callers that cannot allocate
 * device memory: code under HIP graph capture, serving loops and
 * harnesses that forbid hipMalloc.  It calls no allocating routine (device
 * or page-locked host) and does not wait: the launches are enqueued on the
 * context's stream and the outputs are complete when the stream reaches
 * the end of them.  Same moments as kpm_moments for the same opts (the same
 * launches and geometry, bitwise), with these differences:
 *  - A must be in device memory (on_device = 1); the FP32 path needs FP32
 *    values; opts->validate must be 0 and KPM_FLAG_LOCALITY unset
 *    (KPM_ERR_UNSUPPORTED otherwise).
 *  - mu: DEVICE [M+1] doubles; mu_per_vec: DEVICE [nvec * (M+1)] or NULL.
 *  - No escape check: the caller checks |mu_per_vec| <= 1 if it needs to.
 *  - Its work memory is one device array of KPM_NOALLOC_SCRATCH_BYTES per
 *    device, reserved when the library's code is loaded on that device and
 *    held until the process ends: two probe blocks of n x ld values (ld =
 *    the block width rounded up to 4 FP32 or 2 FP64 values), the reduced
 *    dots (ceil(M/2) x 2 x ld doubles), the per-probe moments when
 *    mu_per_vec is NULL (nvec x (M+1) doubles) and at least one step of
 *    per-workgroup dot partials (at most a few MiB).  A problem that does
 *    not fit returns KPM_ERR_ARG before anything is enqueued (the 64^3
 *    workload's 64 FP32 probes, 134 MB of probe blocks, fits).
 *  - Every call on a device shares that array and leaves its contents
 *    behind; calls that overlap on one device (two streams, two threads)
 *    race and must be serialised by the caller.
 * The context must come from kpm_create, which resolves the array's
 * address on its device.
 */
#define KPM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
kpm_status kpm_moments_noalloc(kpm_ctx* ctx, const kpm_csr* A, double lb, double ub,
                               const kpm_moment_opts* opts, double* mu, double* mu_per_vec);

/*
 * kpm_locality_order -- host-only: the row order KPM_FLAG_LOCALITY uses.
 * Finds a 2D or 3D grid behind a CSR matrix numbered lexicographically
 * (x fastest) from the offsets (column - row) of its entries above the
 * diagonal: the offsets occurring in at least 40 % of (a sample of at most
 * 2^18) rows must be {1, nx} (2D, n = nx ny) or {1, nx, nx ny} (3D, n = nx
 * ny nz).  perm (host [n]) receives the rows in the Morton (Z-order) of
 * their grid coordinates, perm[new] = old; dims (host [3]) the grid (nx,
 * ny, nz; nz = 1 in 2D) or zeros with perm the identity when no grid is
 * found.  KPM_ERR_ARG for bad sizes, NULL arrays or row_ptr[0] != 0,
 * row_ptr[n] != nnz.
 */
kpm_status kpm_locality_order(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                              int32_t* perm, int32_t* dims);

/*
 * kpm_autotune -- choose the device geometry of kpm_moments for A by
 * measurement: for each candidate probe-block width (opts->block if set,
 * else 32/64/128 for KPM_FP32, 16/32/64 for KPM_FP64, capped at nvec), row
 * panel height (opts->rows_per_block if set, else the library's choice and
 * half and twice it) and gather batch (4, 7 or 8 CSR entries), time 16 fused
 * recurrence steps (section 3.1.1, eq. (3term); after 8 untimed ones) on the
 * context's stream and
 * keep the fastest per probe.  *best = *opts with block, rows_per_block and
 * the KPM_FLAG_GATHER4 / 7 / 8 bit set to the winner (pass it to
 * kpm_moments; results depend on the geometry only through rounding, and are
 * bitwise reproducible for a fixed geometry).  *us_per_step (nullable): the
 * winner's time per recurrence step for all nvec probes, in microseconds.
 * The choice is a measurement: repeated calls may pick different winners
 * among near-equal candidates.  With KPM_FLAG_LOCALITY in opts->flags the
 * steps run on the renumbered matrix kpm_moments uses under that flag (the
 * flag stays set in *best); a structure changed since the renumbered copy
 * was built is reported as for kpm_moments (KPM_ERR_ARG).
 */
kpm_status kpm_autotune(kpm_ctx* ctx, const kpm_csr* A, double lb, double ub, const kpm_moment_opts* opts,
                        kpm_moment_opts* best, double* us_per_step);

/*
 * kpm_moments_robust -- bounds and moments with escape recovery.  The
 * Lanczos bound of kpm_bounds can miss an extreme eigenvalue whose
 * eigenvector barely overlaps the start vector (e.g. localised edge states
 * of strongly disordered models); the moments then grow exponentially
 * (section 3.1.1), which kpm_moments detects.  This entry point runs
 * kpm_bounds(steps, lanczos_seed, margin) and kpm_moments; on
 * KPM_ERR_SPECTRUM it retries with margin 4x (capped at 0.4), then with the
 * Gershgorin hull widened by `margin`.  *lb, *ub receive the interval the
 * returned moments belong to; *attempts (nullable) the number of moment
 * runs (1 to 3).
 */
kpm_status kpm_moments_robust(kpm_ctx* ctx, const kpm_csr* A, int steps, uint64_t lanczos_seed,
                              double margin, const kpm_moment_opts* opts, double* mu, double* mu_per_vec,
                              double* lb, double* ub, int* attempts);

/*
 * kpm_moments_batched -- the same moments for nmat independent matrices of
 * uneven size (it pays off for many (matrix, probe block) pairs; a few large
 * matrices run faster as kpm_moments calls).  Two device paths:
 *  - on-chip: when opts->block is 0 and two blocks of N, 2N or 4N probes
 *    (N = 4 FP32, 2 FP64) of the largest matrix fit one workgroup's LDS
 *    (160 KB: n up to 2,048 with 8 FP32 probes), one workgroup owns each
 *    (matrix, probe block) pair for all ceil(M/2) steps of eq. (3term) and
 *    the product identity, its vectors in LDS; one launch for all steps
 *    (KPM_FLAG_BATCH_RESIDENT asks for it with a given block width);
 *  - streaming (otherwise, or with KPM_FLAG_BATCH_STREAM): each recurrence
 *    step is one launch over every (matrix, probe block, row-panel range)
 *    of all matrices, the probe blocks in device memory.
 * The per-probe vectors of both paths are bitwise equal (same per-row
 * arithmetic); the dots are summed in different orders.  The launch
 * sequence is captured once per shape (matrix pointers and sizes, M, nvec,
 * block, precision, path) in a HIP graph on a context-owned stream and
 * replayed on later calls (KPM_FLAG_NO_GRAPH launches it directly).  lb, ub: host [nmat].
 * All matrices share opts (M, nvec, block, precision, seed); matrix m uses
 * probe vectors of seed opts->seed + m.  mu: host [nmat * (M+1)], mu[m*(M+1)+k].
 * A[m].on_device must be 1 and the value type common to all m; the FP32
 * path needs FP32 values.  max_abs_mu: host [nmat] or NULL; receives the
 * largest |v_l^T T_k(B) v_l| / n over probes and degrees of each matrix (at
 * most 1 when its spectrum lies in [lb, ub]; +inf if non-finite).  Returns
 * KPM_ERR_SPECTRUM (after writing every output) if a matrix's spectrum is
 * not inside its [lb, ub].  nmat <= 65535, and at most 65535 (matrix, probe
 * block) pairs on the streaming path (2^26 on the on-chip path).  Device
 * memory (one allocation per shape; the context keeps the plans of the two
 * most recently used shapes until kpm_destroy, and releases the older one
 * when a new plan does not fit beside it): on the streaming path two probe blocks of n_m x
 * ld values per pair, dot partials of two steps per workgroup (2 x 2 x ld
 * doubles each; a pair gets at least 16 workgroups when there are more
 * pairs than resident workgroups), K x 2 x ld doubles of dots per pair and
 * the per-probe moments -- about 45 GB for 9,216 matrices of n = 2,048 with
 * 256 FP32 probes each, of which the on-chip path needs only the per-probe
 * moments (nmat x nvec x (M+1) doubles, 2.4 GB there).  KPM_ERR_ALLOC if it
 * cannot be allocated.
 */
kpm_status kpm_moments_batched(kpm_ctx* ctx, int nmat, const kpm_csr* A, const double* lb,
                               const double* ub, const kpm_moment_opts* opts, double* mu,
                               double* max_abs_mu);

/*
 * kpm_autotune_batched -- the same measurement for kpm_moments_batched: for
 * each candidate probe-block width (opts->block if set, else 16/32/64 for
 * KPM_FP32, 8/16/32 for KPM_FP64, capped at nvec) and row-panel height
 * (opts->rows_per_block if set, else the library's choice for the largest
 * matrix and half and twice it), build and capture the plan, then take the
 * device time of the batched launch sequence at degrees 15 and 47 (best of
 * two each) and divide the difference by the 16 extra steps.  *best = *opts with block and rows_per_block of the fastest
 * per probe; *us_per_step (nullable): its time per step for all nvec probes
 * of all matrices, in microseconds.  Leaves the last candidate's plan
 * cached (the next call with *best builds its own).
 */
kpm_status kpm_autotune_batched(kpm_ctx* ctx, int nmat, const kpm_csr* A, const double* lb, const double* ub,
                                const kpm_moment_opts* opts, kpm_moment_opts* best, double* us_per_step);

/*
 * kpm_damping_factors -- damping factors g[0..M] (host, written).
 * KPM_DAMP_NONE: all ones.  KPM_DAMP_JACKSON: eq. (jackson) of Appendix A.
 * KPM_DAMP_LEARNED: the damping network applied to mu[0..M] (host, M <=
 * 127; the network reads zeros above degree M, the truncation it is trained
 * with); g[0] = 1.
 */
kpm_status kpm_damping_factors(kpm_ctx* ctx, kpm_damping kind, int M, const double* mu, double* g);

/*
 * kpm_dos -- approximate DOS of A at npts points x (host) into phi (host):
 *   phi(x) = [g_0 mu_0 + 2 sum_{k>=1} g_k mu_k T_k(t)] / (pi d sqrt(1 - t^2)),
 *   t = (x - c)/d   (eq. (tdosFinal) with eq. (expmu)'s factor and the damping
 * of Appendix A; the 1/d converts the density of B into that of A).
 * phi = 0 where |t| >= 1.
 */
kpm_status kpm_dos(kpm_ctx* ctx, const double* mu, const double* g, int M, double lb, double ub,
                   const double* x, int npts, double* phi);

/*
 * kpm_dos_bins -- mass of the same density over [edges[i], edges[i+1]],
 * i < nbins (edges host [nbins+1], increasing), integrated exactly term by
 * term in theta = arccos t.  A histogram estimate of eq. (DOS1) / n.
 */
kpm_status kpm_dos_bins(kpm_ctx* ctx, const double* mu, const double* g, int M, double lb,
                        double ub, const double* edges, int nbins, double* mass);

/*
 * kpm_dos_pipeline -- the whole path of section 3.1.1 in one call: the
 * Lanczos bounds of kpm_bounds (lanczos_steps, lanczos_seed, margin), the
 * moments of kpm_moments on [lb, ub] (opts), the damping factors of
 * kpm_damping_factors (damping; KPM_DAMP_LEARNED needs M <= 127 and a
 * loaded network) and the density of kpm_dos at the npts points x (host),
 * with the results of those calls: phi (host [npts]), mu (host [M+1],
 * nullable), lb, ub (host).  After the bounds (whose Ritz values are found
 * on the host) the work is enqueued back to back and waited for once.
 * Errors as for the four calls.
 */
kpm_status kpm_dos_pipeline(kpm_ctx* ctx, const kpm_csr* A, int lanczos_steps, uint64_t lanczos_seed,
                            double margin, const kpm_moment_opts* opts, kpm_damping damping, const double* x,
                            int npts, double* phi, double* mu, double* lb, double* ub);

/*
 * kpm_dos_batched -- kpm_dos for nmat matrices in one launch: row m of phi
 * (host [nmat * npts]) is the density of matrix m (series row m of mu, host
 * [nmat * (M+1)]; interval lb[m], ub[m], host [nmat]) at its own points, row
 * m of x (host [nmat * npts]).  g: host [M+1] shared by all matrices, or
 * [nmat * (M+1)] one row per matrix when g_per_matrix != 0.  Each row is
 * bitwise what kpm_dos returns for that matrix (same per-point arithmetic).
 * nmat in [1, 65535].
 */
kpm_status kpm_dos_batched(kpm_ctx* ctx, int nmat, const double* mu, const double* g, int g_per_matrix, int M,
                           const double* lb, const double* ub, const double* x, int npts, double* phi);

/*
 * kpm_dos_pipeline_batched -- the whole path of section 3.1.1 for nmat
 * matrices:
 *  - the bounds of kpm_bounds_batched (lanczos_steps, lanczos_seed, margin);
 *  - the moments of kpm_moments_batched (opts; matrix m's probes from seed
 *    opts->seed + m; A[m].on_device must be 1);
 *  - for the matrices whose moments escape, the recovery of
 *    kpm_moments_robust, each matrix keeping its probes: its bounds again
 *    with margin 4x (capped at 0.4; all of them in one batched bounds call)
 *    and its moments -- in one batched moment call when 16 or more escape
 *    and none has more than 131,072 rows, else one kpm_moments call each
 *    (same M, nvec and precision; the
 *    library's block and panel choice; seed opts->seed + m); then, for any
 *    that still escape, the Gershgorin hull widened by margin and
 *    kpm_moments.  Intervals and attempts are those kpm_moments_robust
 *    returns for that matrix;
 *  - the damping factors (KPM_DAMP_LEARNED: one network inference over all
 *    nmat moment vectors, M <= 127, each row bitwise what
 *    kpm_damping_factors returns for that matrix);
 *  - the density of every matrix at its own npts points, as
 *    kpm_dos_batched.
 * x, phi: host [nmat * npts]; mu: host [nmat * (M+1)] or NULL; lb, ub: host
 * [nmat], receive the interval each matrix's moments belong to; attempts:
 * host [nmat] or NULL, the bound estimates each matrix needed (1 to 3).
 * Returns KPM_ERR_SPECTRUM (with lb, ub, mu and attempts written) if a
 * matrix still escapes its Gershgorin interval; other errors as for the
 * calls it makes.
 */
kpm_status kpm_dos_pipeline_batched(kpm_ctx* ctx, int nmat, const kpm_csr* A, int lanczos_steps,
                                    uint64_t lanczos_seed, double margin, const kpm_moment_opts* opts,
                                    kpm_damping damping, const double* x, int npts, double* phi, double* mu,
                                    double* lb, double* ub, int* attempts);

/*
 * kpm_dgl_dos -- the Delta-Gauss-Legendre density (section 3.1.3, eq.
 * (dglexpansion)): at each point x_i (host, A's units),
 *   phi(x_i) = sum_{k <= m_i} (k + 1/2) gamma_k(t_i) mu_k / sqrt(2 pi s^2) / d,
 * t_i = (x_i - c)/d, s = sigma/d, with gamma_k(t) = int_{-1}^{1} L_k(u)
 * exp(-((u - t)/s)^2 / 2) du (eq. (DGLcoeff)) from the recurrence of eq.
 * (Leg3) started at gamma_0 of eq. (gam0), and m_i the first k >= 1 with
 * |gamma_{k-1}| + |gamma_k| <= k tol (eq. (StopRecur); the paper suggests
 * tol = 1e-6), at most M.  mu: host [M+1] Legendre moments from
 * kpm_legendre_moments; sigma: Gaussian width in A's units (the density
 * approximated is the Gaussian-regularised one of eq. (blurphi)); phi host
 * [npts]; degree_used (nullable) host int [npts] = m_i.  The recurrence
 * amplifies rounding noise once the coefficients have decayed; since
 * |gamma_k| <= gamma_0 holds exactly, a computed coefficient beyond it is
 * reported as KPM_ERR_NOCONV (tol too small).  KPM_ERR_ARG for sigma <= 0,
 * tol < 0, lb >= ub.
 */
kpm_status kpm_dgl_dos(kpm_ctx* ctx, const double* mu, int M, double lb, double ub, double sigma, double tol,
                       const double* x, int npts, double* phi, int* degree_used);

/*
 * kpm_legendre_dos -- KPM with Legendre polynomials (Appendix A): the
 * expansion of the density in the basis orthogonal for the unit weight,
 *   phi(x) = sum_{k <= M} (k + 1/2) g_k mu_k L_k(t) / d,   t = (x - c)/d,
 * 0 for |t| > 1.  mu: host [M+1] Legendre moments; g: host [M+1] damping
 * factors or NULL (none); x, phi host [npts], A's units.
 */
kpm_status kpm_legendre_dos(kpm_ctx* ctx, const double* mu, const double* g, int M, double lb, double ub,
                            const double* x, int npts, double* phi);

/*
 * kpm_slq -- the stochastic Lanczos method of section 3.2.1.  For every probe
 * vector v_l (l < nvec, the Rademacher vectors of opts->seed) an M-step
 * Lanczos factorisation A V_M = V_M T_M + f_M e_M^T (eq. (lanfact)) from
 * v_l / ||v_l|| by the plain three-term recurrence (no re-orthogonalisation),
 * in FP64 on B = (A - cI)/d, c = (lb+ub)/2, d = (ub-lb)/2 (lb < ub need not
 * enclose the spectrum; they only centre and scale the arithmetic).  The run
 * of a probe stops at the first step k whose residual norm beta_k is at most
 * 1e-12 of the largest |alpha_j|, beta_j so far (breakdown: an invariant
 * subspace was found).  Outputs, row l for probe l (host, nvec x M):
 *   theta:  Ritz values c + d theta_k of the probe's tridiagonal matrix,
 *           ascending (eq. (landist)); 0 past steps_used[l];
 *   tau2:   squared first components of its normalised eigenvectors, the
 *           node weights (sum 1 per probe: a Rademacher probe has ||v||^2 = n,
 *           which cancels the 1/n of eq. (lanapprox)); 0 past steps_used[l];
 *   steps_used (nullable, int [nvec]): size of the tridiagonal matrix;
 *   alpha, beta (nullable): T of B, alpha[l*M+k] = q_k.B q_k (diagonal),
 *           beta[l*M+k] = ||r_k|| (coupling of q_k and q_{k+1}; the last one
 *           is ||f_M||).
 * theta and tau2 may both be NULL when alpha and beta are given: the
 * coefficients (and steps_used) alone, without the eigenvalue problems
 * (Haydock's method, kpm_haydock_dos, needs no Ritz values).
 * opts: M = Lanczos steps in [1, 4096], nvec, block (probes per device
 * block, 0 = min(nvec, 16), <= 64; up to 8 blocks run concurrently, one
 * group of XCDs each), seed, validate, rows_per_block;
 * precision must be KPM_FP64
 * (KPM_ERR_UNSUPPORTED otherwise).  FP32 or FP64 matrix values.
 */
kpm_status kpm_slq(kpm_ctx* ctx, const kpm_csr* A, double lb, double ub, const kpm_moment_opts* opts,
                   double* theta, double* tau2, int* steps_used, double* alpha, double* beta);

/*
 * kpm_slq_dos -- eq. (landos): the Gaussian-blurred Lanczos density
 *   phi(x_i) = (1/nvec) sum_l sum_k tau2[l*M+k] g_sigma(x_i - theta[l*M+k]),
 * g_sigma(t) = exp(-t^2 / (2 sigma^2)) / sqrt(2 pi sigma^2) (eq. (gauss)),
 * at npts points x (host) into phi (host), all in A's units.  theta, tau2:
 * host [nvec * M] as written by kpm_slq.  Non-negative by construction.
 */
kpm_status kpm_slq_dos(kpm_ctx* ctx, const double* theta, const double* tau2, int nvec, int M, double sigma,
                       const double* x, int npts, double* phi);

/*
 * kpm_haydock_dos -- Haydock's method (section 3.2.2): the density
 * regularised by Lorentzians of half-width eta (eq. (lorentz)),
 *   phi(x_i) = (1/nvec) sum_l -(1/pi) Im e_1^T ((x_i + i eta) I - T_l)^{-1} e_1,
 * from the probes' Lanczos matrices without their eigenvalues: the (1,1)
 * resolvent entry is the continued fraction of eq. (cfHaydock), evaluated
 * from the bottom in FP64 on the device.  T_l = c I + d tridiag(beta, alpha,
 * beta) restricted to its first steps_used[l] rows, with alpha, beta the
 * coefficients of B written by kpm_slq (host, [nvec * M], row l for probe
 * l; beta[l*M+k] couples steps k and k+1) and c = (lb+ub)/2, d = (ub-lb)/2
 * the lb, ub given to kpm_slq.  x (host, npts points) and eta in A's units;
 * phi (host, npts) in A's units, non-negative, unit mass per probe (the
 * paper's second form of phi_eta writes +Im: the sign is taken so that the
 * density is that of its first form).  KPM_ERR_ARG for eta <= 0, lb >= ub,
 * a steps_used entry outside [1, M], a non-finite coefficient among those
 * used, or nvec outside [1, 65535].
 */
kpm_status kpm_haydock_dos(kpm_ctx* ctx, const double* alpha, const double* beta, const int* steps_used,
                           int nvec, int M, double lb, double ub, double eta, const double* x, int npts,
                           double* phi);

/*
 * kpm_functional -- <phi~, f> = int f(lambda) phi~(lambda) dlambda for the
 * KPM density of eq. (tdosFinal) with damping g (host [M+1] or NULL = none)
 * and normalised Chebyshev moments mu (host [M+1]), the quantity compared
 * in the functional error of eq. (errormetric_g).  The integral is taken
 * in theta = arccos t by Gauss-Chebyshev quadrature on Q nodes:
 *   out = (1/Q) sum_q fvals[q] D(theta_q),  theta_q = (q + 1/2) pi / Q,
 *   D(theta) = sum_k (2 - [k = 0]) g_k mu_k cos(k theta),
 * where fvals[q] = f(c + d cos theta_q) (host [Q], A's units, c = (lb+ub)/2,
 * d = (ub-lb)/2) are the caller's samples of f.  Exact for polynomial f of
 * degree < 2Q - M; geometric convergence in Q for f analytic on [lb, ub].
 * out: one double (host).
 */
kpm_status kpm_functional(kpm_ctx* ctx, const double* mu, const double* g, int M, double lb, double ub,
                          const double* fvals, int Q, double* out);

/*
 * kpm_functional_nodes -- the Q points of A's axis at which kpm_functional
 * takes the caller's samples of f: x[q] = c + d cos((q + 1/2) pi / Q),
 * c = (lb+ub)/2, d = (ub-lb)/2 (the Gauss-Chebyshev nodes of the theta =
 * arccos t integral above, mapped back by eq. (cd)).  Host-only, no
 * context; x: host [Q], caller-owned.  KPM_ERR_ARG for Q < 1, Q > 2^26,
 * lb >= ub, non-finite bounds or a NULL x.
 */
kpm_status kpm_functional_nodes(int Q, double lb, double ub, double* x);

/*
 * kpm_heat_capacity -- section 4.3: C_v(T_j) = <phi~, g_T> for the KPM
 * density as in kpm_functional, with g_T of eq. (gfunc) in units where
 * k_B = 1 and hbar c / k_B = 1, as a function of lambda = omega^2:
 *   g_T(lambda) = x^2 e^{-x} / (1 - e^{-x})^2 = (x / (2 sinh(x/2)))^2,
 *   x = sqrt(lambda) / T,   g_T = 1 for lambda <= 0,
 * evaluated on the device at the Q nodes (Q = 0: max(1024, 4(M+1))).
 * T host [nT] (> 0), cv host [nT].
 */
kpm_status kpm_heat_capacity(kpm_ctx* ctx, const double* mu, const double* g, int M, double lb, double ub,
                             const double* T, int nT, int Q, double* cv);

/*
 * kpm_slq_heat_capacity -- the same heat capacity for the Lanczos density,
 * with g_T in place of the Gaussian of eq. (landos) (section 4.3):
 *   cv[j] = (1/nvec) sum_l sum_k tau2[l*M+k] g_T(theta[l*M+k]),
 * theta, tau2 host [nvec * M] as written by kpm_slq.
 */
kpm_status kpm_slq_heat_capacity(kpm_ctx* ctx, const double* theta, const double* tau2, int nvec, int M,
                                 const double* T, int nT, double* cv);

/*
 * kpm_tridiag_eig -- host-only helper (no device work): eigenvalues theta
 * (ascending) and squared first eigenvector components tau2 of the
 * symmetric tridiagonal matrix with diagonal alpha[0..m-1] and off-diagonal
 * beta[0..m-2] (beta may be NULL when m = 1), i.e. the nodes and weights of
 * eq. (landist) (Gauss quadrature, eq. (tauexpand)).  KPM_ERR_ARG for m < 1
 * or non-finite input, KPM_ERR_NOCONV if the QR iteration does not converge.
 */
kpm_status kpm_tridiag_eig(int m, const double* alpha, const double* beta, double* theta, double* tau2);

/*
 * kpm_rademacher -- fill a device block out[i * ld + j] (i < n, j < nvec)
 * with probe vectors vec0 .. vec0+nvec-1 of `seed` as float (precision
 * KPM_FP32) or double (KPM_FP64).  Columns nvec .. ld-1 are left untouched.
 */
kpm_status kpm_rademacher(kpm_ctx* ctx, uint64_t seed, int64_t vec0, int nvec, int64_t n,
                          int64_t ld, int precision, void* out_device);

/* ---- learned damping network (128 -> 256 -> 256 -> 128, GELU, sigmoid) ----
 * Parameters are one FP32 array in the order W1[128x256], b1[256],
 * W2[256x256], b2[256], W3[256x128], b3[128] (row-major, input index first):
 * kpm_mlp_param_count() floats in total. */
int64_t kpm_mlp_param_count(void);
kpm_status kpm_mlp_set_params(kpm_ctx* ctx, const float* params);
kpm_status kpm_mlp_get_params(kpm_ctx* ctx, float* params);
/* Forward pass: x host [N x 128] (moments) -> g host [N x 128]. */
kpm_status kpm_mlp_forward(kpm_ctx* ctx, int N, const float* x, float* g);
/* Loss (mean over the batch of the L1 distance between the blurred damped
 * KPM density and `target` on npts = 200 midpoints of [-1, 1], Gaussian
 * width sigma in B's units) and its gradient with respect to every
 * parameter, in the parameter order above.  grads host [param_count]. */
kpm_status kpm_mlp_loss_grad(kpm_ctx* ctx, int N, const float* x, const float* target,
                             float sigma, float* loss, float* grads);
/* Train with Adam (beta1 0.9, beta2 0.999, eps 1e-8) for `epochs` passes of
 * minibatches of `batch` samples in a seeded order; loss_per_epoch host
 * [epochs] or NULL.  Starts from the current parameters (kpm_mlp_init first
 * for a fresh network). */
kpm_status kpm_mlp_train(kpm_ctx* ctx, int N, const float* x, const float* target, float sigma,
                         int epochs, int batch, float lr, uint64_t seed, float* loss_per_epoch);
/* Fresh parameters: fan-in scaled Rademacher-signed weights, zero biases. */
kpm_status kpm_mlp_init(kpm_ctx* ctx, uint64_t seed);
/* Save / load the parameters as raw little-endian FP32 behind a 16-byte header. */
kpm_status kpm_mlp_save(kpm_ctx* ctx, const char* path);
kpm_status kpm_mlp_load(kpm_ctx* ctx, const char* path);

/*
 * kpm_hbm_copy_probe -- achievable device-memory bandwidth: a plain
 * streaming copy of `bytes` bytes (one 16-byte non-temporal load and store
 * per thread, one workgroup per 4 KiB) run `iters` times
 * between two context-owned buffers; *gbs = 2 * bytes * iters / time / 1e9.
 * The practical denominator beside the HBM specification peak and the
 * calibration kernel for hardware byte counters.
 */
kpm_status kpm_hbm_copy_probe(kpm_ctx* ctx, int64_t bytes, int iters, double* gbs);

/* ---- device timing of the library's own kernels ----
 * When enabled, the launches of the listed kernels are bracketed by HIP
 * events on the stream they run on.  kernel: "cheb_step" (fused recurrence
 * steps, the dominant kernel: one record per run of steps, counting its
 * launches), "cheb_first" (first steps), "lanczos" (a bounds run),
 * "lanczos_batched" (a kpm_bounds_batched call's launch sequence, one
 * record per call),
 * "batched" (one batched call's launch sequence), "slq_step" (a stochastic
 * Lanczos run's steps), "copy_probe".  Query waits for the context's stream
 * and returns the launches and their total time since the last reset (a
 * name never timed reads 0 launches). */
kpm_status kpm_profile_enable(kpm_ctx* ctx, int enable);
kpm_status kpm_profile_query(kpm_ctx* ctx, const char* kernel, int64_t* launches, double* total_ms);
kpm_status kpm_profile_reset(kpm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* KPM_H */
