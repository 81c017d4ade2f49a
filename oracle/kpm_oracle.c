/*
 * CPU FP64 oracle for the KPM moment computation -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the slow, plain reference that the GPU library is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the library never links or calls it, and it
 * shares no code with the library.
 *
 * It follows Lin, Saad & Yang, "Approximating spectral densities of large
 * matrices", section 3.1.1 (Algorithm 1, the kernel polynomial method):
 *   - the matrix is used as B = (A - c I)/d  (rescaling, eq. (cd));
 *   - for every probe vector v0: v1 = B v0, v_{k+1} = 2 B v_k - v_{k-1}
 *     (three-term recurrence, eq. (3term));
 *   - zeta_k += v0^T v_k for k = 0..M  (stochastic trace, eqs. (nuk), (muEst)).
 * Dot products are accumulated in FP64 with Neumaier's compensated sum.
 *
 * Probe vectors are Rademacher (+/-1) vectors defined by a counter-based
 * generator (SplitMix64, Steele, Lea & Flood, OOPSLA 2014): entry i of probe
 * vector l is +1 or -1 according to the top bit of output number
 * ((l << 32) | i) + 1 of the SplitMix64 sequence started from `seed`.  Any
 * vector with E[v] = 0 and E[v v^T] = I satisfies Theorem 1 of the paper.
 *
 * A second routine computes the same moments with the product identity of
 * Appendix A (T_{p+q} = 2 T_p T_q - T_{|p-q|}, sign as in the standard
 * identity) as a self-check; it is not used to produce reference values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* SplitMix64 output function (published constants). */
static uint64_t splitmix64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Output number k (k >= 1) of the SplitMix64 sequence started from seed. */
static uint64_t splitmix64_nth(uint64_t seed, uint64_t k) {
    return splitmix64_mix(seed + k * 0x9e3779b97f4a7c15ULL);
}

double oracle_rademacher_entry(uint64_t seed, uint32_t l, uint32_t i) {
    uint64_t counter = (((uint64_t)l) << 32) | (uint64_t)i;
    uint64_t z = splitmix64_nth(seed, counter + 1);
    return (z >> 63) ? -1.0 : 1.0;
}

void oracle_rademacher(uint64_t seed, int64_t l, int64_t n, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_rademacher_entry(seed, (uint32_t)l, (uint32_t)i);
}

uint64_t oracle_splitmix64_nth(uint64_t seed, uint64_t k) { return splitmix64_nth(seed, k); }

/* Neumaier's compensated summation of a[i]*b[i]. */
static double dot_neumaier(const double* a, const double* b, int64_t n) {
    double s = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double x = a[i] * b[i];
        double t = s + x;
        if (fabs(s) >= fabs(x))
            comp += (s - t) + x;
        else
            comp += (x - t) + s;
        s = t;
    }
    return s + comp;
}

/* y = B x with B = (A - c I)/d, A in CSR. */
static void apply_B(int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                    double c, double d, const double* x, double* y) {
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += val[k] * x[ci[k]];
        y[i] = (s - c * x[i]) / d;
    }
}

/*
 * Per-vector raw moments zeta[l*(M+1) + k] = v0^T T_k(B) v0 for probe vectors
 * vec0 .. vec0+nvec-1, k = 0..M, by the plain recurrence (no doubling).
 * Returns 0 on success, -1 on allocation failure.
 */
int oracle_moments(int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                   double c, double d, int M, int nvec, uint64_t seed, int64_t vec0,
                   double* zeta, int nthreads) {
    int failed = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
#endif
    for (int l = 0; l < nvec; ++l) {
        double* v0 = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double* vprev = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double* vcur = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double* vnext = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double* z = zeta + (size_t)l * (size_t)(M + 1);
        if (!v0 || !vprev || !vcur || !vnext) {
            failed |= 1;
        } else {
            oracle_rademacher(seed, vec0 + l, n, v0);
            z[0] = dot_neumaier(v0, v0, n);
            if (M >= 1) {
                memcpy(vprev, v0, sizeof(double) * (size_t)n);
                apply_B(n, rp, ci, val, c, d, v0, vcur); /* v1 = B v0 */
                z[1] = dot_neumaier(v0, vcur, n);
                for (int k = 1; k < M; ++k) {
                    apply_B(n, rp, ci, val, c, d, vcur, vnext);
                    for (int64_t i = 0; i < n; ++i) vnext[i] = 2.0 * vnext[i] - vprev[i];
                    z[k + 1] = dot_neumaier(v0, vnext, n);
                    double* t = vprev;
                    vprev = vcur;
                    vcur = vnext;
                    vnext = t;
                }
            }
        }
        free(v0);
        free(vprev);
        free(vcur);
        free(vnext);
    }
    return failed ? -1 : 0;
}

/*
 * Same quantities via T_{p+q} = 2 T_p T_q - T_{|p-q|}:
 *   zeta_{2k}   = 2 v_k^T v_k     - zeta_0,
 *   zeta_{2k+1} = 2 v_{k+1}^T v_k - zeta_1.
 * Self-check only.
 */
int oracle_moments_doubling(int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                            double c, double d, int M, int nvec, uint64_t seed, int64_t vec0,
                            double* zeta, int nthreads) {
    int failed = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
#endif
    for (int l = 0; l < nvec; ++l) {
        size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
        double* v0 = (double*)malloc(bytes);
        double* vprev = (double*)malloc(bytes);
        double* vcur = (double*)malloc(bytes);
        double* vnext = (double*)malloc(bytes);
        double* z = zeta + (size_t)l * (size_t)(M + 1);
        if (!v0 || !vprev || !vcur || !vnext) {
            failed |= 1;
        } else {
            oracle_rademacher(seed, vec0 + l, n, v0);
            z[0] = dot_neumaier(v0, v0, n);
            if (M >= 1) {
                memcpy(vprev, v0, bytes);
                apply_B(n, rp, ci, val, c, d, v0, vcur);
                z[1] = dot_neumaier(v0, vcur, n);
                /* vprev = v_{k-1}, vcur = v_k */
                for (int k = 1; 2 * k <= M; ++k) {
                    z[2 * k] = 2.0 * dot_neumaier(vcur, vcur, n) - z[0];
                    if (2 * k + 1 <= M) {
                        apply_B(n, rp, ci, val, c, d, vcur, vnext);
                        for (int64_t i = 0; i < n; ++i) vnext[i] = 2.0 * vnext[i] - vprev[i];
                        z[2 * k + 1] = 2.0 * dot_neumaier(vnext, vcur, n) - z[1];
                        double* t = vprev;
                        vprev = vcur;
                        vcur = vnext;
                        vnext = t;
                    }
                }
            }
        }
        free(v0);
        free(vprev);
        free(vcur);
        free(vnext);
    }
    return failed ? -1 : 0;
}

/*
 * Column block of probe vectors, row-major [n x nvec]: out[i*nvec + l] =
 * entry i of probe vector vec0 + l.  Used by tests to compare generators.
 */
void oracle_rademacher_block(uint64_t seed, int64_t vec0, int nvec, int64_t n, double* out) {
    for (int64_t i = 0; i < n; ++i)
        for (int l = 0; l < nvec; ++l)
            out[i * nvec + l] = oracle_rademacher_entry(seed, (uint32_t)(vec0 + l), (uint32_t)i);
}
