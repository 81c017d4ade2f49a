"""Equal-accuracy comparison on the 64^3 Anderson workload and the large
workload: FP32 moments with the shipped learned damping, and with no
damping, against FP64 moments + Jackson damping (Appendix A), and the
stochastic Lanczos method (section 3.2.1) on the same probes.

Error metric: L1 distance (eq. (err2), p = 1) on 200 midpoints of [-1, 1]
between Gaussian-blurred densities (sigma = 0.02 in the scaled variable, as
the paper blurs KPM before comparing in section 4.1).  Reference: the FP64
oracle's undamped series of degree 512 with the same probes (its blurred
tail beyond degree 512 is below 1e-20), so the metric measures what the
degree, the damping and the arithmetic precision cost, not the shared
stochastic-trace noise.  Against that reference no damping is the best
possible choice at every degree it has reached: whatever the damping
removes is part of the reference.  The learned network's value is measured
where trace noise counts, against exact densities (test_gpu_damping.py).

The network is the one the library ships (trained by test_gpu_damping.py on
exact labels of the training family, with truncation augmentation, so it
serves any degree up to 127).  The degrees at which each form first reaches
L1 <= 1e-2 are the ones bench.py times; this test asserts they agree.
"""
import json
import os
import sys

import numpy as np
import pytest

import bench
import oracle
import paper_1308_5467_amd as kpm
import synth

pytestmark = pytest.mark.gpu

SIGMA = 0.02
DEGREES = (16, 20, 24, 28, 32, 40, 48, 56, 64, 80, 96, 127)
SLQ_STEPS = (40, 50, 60, 65, 70, 80, 100)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _save_study(name, data):
    """Write a study table as JSON into $KPM_STUDY_DIR (nothing when unset)."""
    out = os.environ.get("KPM_STUDY_DIR")
    if not out:
        return
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, name), "w") as f:
        json.dump(data, f, indent=1)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = kpm.Context(0)
    yield c
    c.close()


def _blur_l1(mu, g, ref):
    t = oracle.midpoints(200)
    return oracle.l1_error(ref, oracle.blurred_kpm(mu, g, t, SIGMA, Q=8192))


@pytest.fixture(scope="module")
def trained(ctx):
    """The shipped damping network."""
    if not os.path.exists(kpm.DAMPING_WEIGHTS):
        pytest.skip("no shipped damping weights")
    kpm.kpm_mlp_load(ctx, kpm.DAMPING_WEIGHTS)


def _degree_rows(ctx, mu32, mu64, ref):
    rows = []
    for M in DEGREES:
        x = np.zeros(128)
        x[:M + 1] = mu32[:M + 1]
        g_learned = kpm.kpm_mlp_forward(ctx, x[None, :])[0].astype(np.float64)[:M + 1]
        rows.append(dict(M=M,
                         fp64_jackson=_blur_l1(mu64[:M + 1], oracle.jackson(M), ref),
                         fp32_learned=_blur_l1(mu32[:M + 1], g_learned, ref),
                         fp32_none=_blur_l1(mu32[:M + 1], np.ones(M + 1), ref),
                         fp32_jackson=_blur_l1(mu32[:M + 1], oracle.jackson(M), ref)))
    for r in rows:
        _say("M=%3d  fp64+jackson %.4f  fp32+learned %.4f  fp32+none %.4f  fp32+jackson %.4f"
             % (r["M"], r["fp64_jackson"], r["fp32_learned"], r["fp32_none"], r["fp32_jackson"]))
    return rows


def _degrees(rows):
    """Lowest tabulated degree at which FP64 + Jackson, FP32 + learned and
    FP32 undamped first reach L1 <= 1e-2."""
    return tuple(min(r["M"] for r in rows if r[k] <= 1e-2) for k in ("fp64_jackson", "fp32_learned", "fp32_none"))


def test_fp32_learned_vs_fp64_jackson_on_anderson64(ctx, trained):
    _say("c2 workload")
    A = synth.config_matrix("c2")
    D32 = kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32), "f32")
    D64 = kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32).astype(np.float64), "f64")
    lb, ub = kpm.kpm_bounds(ctx, D32, 20, 3002, 0.01)
    mu32 = kpm.kpm_moments(ctx, D32, lb, ub, 127, 64, 2002, precision="f32")
    mu64 = kpm.kpm_moments(ctx, D64, lb, ub, 127, 64, 2002, precision="f64")
    _say("oracle reference (degree 512, same probes)")
    Ao = A.rounded_f32()
    c, d = oracle.rescale(lb, ub)
    zeta = oracle.moments_per_vector(Ao, c, d, 512, 64, 2002, nthreads=min(16, os.cpu_count() or 1))
    mu_ref = oracle.normalize(zeta, A.n)
    assert np.max(np.abs(mu64 - mu_ref[:128])) < 1e-12
    assert np.max(np.abs(mu32 - mu_ref[:128])) < 1e-5
    t = oracle.midpoints(200)
    ref = oracle.blurred_kpm(mu_ref, np.ones(513), t, SIGMA, Q=8192)

    rows = _degree_rows(ctx, mu32, mu64, ref)
    M_J, M_L, M_N = _degrees(rows)

    # Stochastic Lanczos method (section 3.2.1), same probes, FP64 recurrence:
    # M Lanczos steps = M sparse products per probe (KPM of degree M uses M/2).
    slq_rows = []
    for Ms in SLQ_STEPS:
        th, t2, _ = kpm.kpm_slq(ctx, D32, lb, ub, Ms, 64, 2002)
        phi = oracle.lanczos_dos((th - c) / d, t2, t, SIGMA)
        assert np.all(phi >= 0.0)
        slq_rows.append(dict(M=Ms, slq_fp64=oracle.l1_error(ref, phi)))
        _say("Lanczos steps=%3d  L1 %.4f" % (Ms, slq_rows[-1]["slq_fp64"]))
    M_S = min(r["M"] for r in slq_rows if r["slq_fp64"] <= 1e-2)
    summary = dict(sigma=SIGMA, rows=rows, M_fp64_jackson=M_J, M_fp32_learned=M_L, M_fp32_none=M_N,
                   slq_rows=slq_rows, M_slq_fp64=M_S)
    _save_study("accuracy_study.json", summary)
    _say(f"degree for L1 <= 1e-2: FP64+Jackson {M_J}, FP32+learned {M_L}, FP32+none {M_N}; Lanczos steps {M_S}")
    assert (M_J, M_L, M_N, M_S) == (bench.M_FP64_JACKSON, bench.M_FP32_LEARNED, bench.M_FP32_NONE, bench.M_SLQ)
    assert M_L < M_J and M_N < M_J
    # the network must not be worse than Jackson at the same degree and precision
    for r in rows:
        assert r["fp32_learned"] <= r["fp32_jackson"] + 1e-3, r


def test_fp32_learned_vs_fp64_jackson_on_large(ctx, trained):
    """The large workload: 3D Anderson 128^3 + 2 random long-range pairs per
    row (n = 2,097,152, nnz ~ 23.07M).  Same criterion, 4 probes (the
    comparison is against the same probes' degree-512 series, so it measures
    truncation and damping, not the probe count); the oracle's reference
    costs about a minute of host time."""
    _say("c5 workload")
    A = synth.config_matrix("c5")
    D32 = kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32), "f32")
    D64 = kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32).astype(np.float64), "f64")
    lb, ub = kpm.kpm_bounds(ctx, D32, 20, 3005, 0.01)
    nvec, seed = 4, 2005
    mu32 = kpm.kpm_moments(ctx, D32, lb, ub, 127, nvec, seed, precision="f32")
    mu64 = kpm.kpm_moments(ctx, D64, lb, ub, 127, nvec, seed, precision="f64")
    _say("oracle reference (degree 512, same 4 probes)")
    c, d = oracle.rescale(lb, ub)
    zeta = oracle.moments_per_vector(A.rounded_f32(), c, d, 512, nvec, seed, nthreads=min(16, os.cpu_count() or 1))
    mu_ref = oracle.normalize(zeta, A.n)
    assert np.max(np.abs(mu64 - mu_ref[:128])) < 1e-12
    assert np.max(np.abs(mu32 - mu_ref[:128])) < 1e-5
    ref = oracle.blurred_kpm(mu_ref, np.ones(513), oracle.midpoints(200), SIGMA, Q=8192)
    rows = _degree_rows(ctx, mu32, mu64, ref)
    M_J, M_L, M_N = _degrees(rows)
    _save_study("accuracy_study_large.json",
                dict(sigma=SIGMA, rows=rows, M_fp64_jackson=M_J, M_fp32_learned=M_L, M_fp32_none=M_N, nvec=nvec))
    _say(f"large workload, degree for L1 <= 1e-2: FP64+Jackson {M_J}, FP32+learned {M_L}, FP32+none {M_N}")
    assert (M_J, M_L, M_N) == (bench.M_LARGE_FP64_JACKSON, bench.M_LARGE_FP32_LEARNED, bench.M_LARGE_FP32_NONE)
    assert M_L < M_J and M_N < M_J
    for r in rows:
        assert r["fp32_learned"] <= r["fp32_jackson"] + 1e-3, r


BATCHED_DEGREES = DEGREES + (160, 200, 256)


def test_equal_accuracy_on_batched_uneven(ctx, trained):
    """The uneven batch (48 matrices: 2D Dirichlet Laplacians 64..512 and 3D
    periodic Laplacians 16..64 with disorder W in {2, 8, 16}), 4 probes per
    matrix, bounds as the benchmark finds them.  Per matrix the reference is
    the FP64 oracle's undamped degree-512 series of the same probes; a form
    reaches the bar at degree M when every matrix has L1 <= 1e-2 there.
    The GPU moments are checked against the same oracle runs (FP64 1e-12,
    FP32 1e-5).  The damping network (trained on random sparse and 2D
    Anderson matrices, degrees <= 127) does not reach the bar on this batch:
    its nearly clean 3D Laplacians have peaky spectra that it over-damps."""
    mats = synth.batched_uneven_set(48)
    D32 = [kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32), "f32") for A in mats]
    D64 = [kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32).astype(np.float64), "f64")
           for A in mats]
    lb, ub, _ = bench.batched_uneven_bounds(kpm, ctx, D32)
    nvec, seed, Mmax = 4, 2003, BATCHED_DEGREES[-1]
    mu32 = kpm.kpm_moments_batched(ctx, D32, lb, ub, Mmax, nvec, seed, precision="f32")
    mu64 = kpm.kpm_moments_batched(ctx, D64, lb, ub, Mmax, nvec, seed, precision="f64")
    _say("oracle references (degree 512, 4 probes per matrix)")
    t = oracle.midpoints(200)
    refs = []
    for m, A in enumerate(mats):
        c, d = oracle.rescale(lb[m], ub[m])
        z = oracle.moments_per_vector(A.rounded_f32(), c, d, 512, nvec, seed + m, nthreads=min(16, os.cpu_count() or 1))
        mu_ref = oracle.normalize(z, A.n)
        assert np.max(np.abs(mu64[m] - mu_ref[:Mmax + 1])) < 1e-12, m
        assert np.max(np.abs(mu32[m] - mu_ref[:Mmax + 1])) < 1e-5, m
        refs.append(oracle.blurred_kpm(mu_ref, np.ones(513), t, SIGMA, Q=8192))

    def worst(mu, gfun, M):
        return max(_blur_l1(mu[m, :M + 1], gfun(m), refs[m]) for m in range(len(mats)))

    rows = []
    for M in BATCHED_DEGREES:
        r = dict(M=M, fp64_jackson=worst(mu64, lambda m: oracle.jackson(M), M),
                 fp32_none=worst(mu32, lambda m: np.ones(M + 1), M),
                 fp32_jackson=worst(mu32, lambda m: oracle.jackson(M), M))
        if M <= 127:
            x = np.zeros((len(mats), 128))
            x[:, :M + 1] = mu32[:, :M + 1]
            G = kpm.kpm_mlp_forward(ctx, x).astype(np.float64)[:, :M + 1]
            r["fp32_learned"] = worst(mu32, lambda m: G[m], M)
        rows.append(r)
        _say("M=%3d  worst L1: fp64+jackson %.4f  fp32+none %.4f  fp32+jackson %.4f  fp32+learned %s"
             % (M, r["fp64_jackson"], r["fp32_none"], r["fp32_jackson"],
                "%.4f" % r["fp32_learned"] if "fp32_learned" in r else "-"))

    def first(key):
        ok = [r["M"] for r in rows if key in r and r[key] <= 1e-2]
        return min(ok) if ok else None

    M_J, M_N, M_L = first("fp64_jackson"), first("fp32_none"), first("fp32_learned")
    _save_study("accuracy_study_batched.json", dict(sigma=SIGMA, nvec=nvec, rows=rows, M_fp64_jackson=M_J,
                                                    M_fp32_none=M_N, M_fp32_learned=M_L))
    _say(f"uneven batch, degree for L1 <= 1e-2 on every matrix: FP64+Jackson {M_J}, FP32+none {M_N}, "
         f"FP32+learned {M_L}")
    assert (M_J, M_N, M_L) == (bench.M_BATCHED_FP64_JACKSON, bench.M_BATCHED_FP32_NONE, bench.M_BATCHED_FP32_LEARNED)
    assert M_N < M_J
