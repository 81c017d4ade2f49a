"""The whole path for many matrices in one call (kpm_dos_pipeline_batched)
and the batched density (kpm_dos_batched).

Bars: kpm_dos_batched row by row bitwise equal to kpm_dos and within 1e-11
of the maximum of the oracle's density; the pipeline bitwise equal to the
separate calls it stands for (per-matrix bounds, one batched moment call,
per-matrix damping factors and densities), its escape recovery equal to
kpm_moments_robust's per matrix (intervals and attempts; the moments
bitwise on the single-matrix path, at the FP32 bar from a sub-batch), and its moments against
the oracle at the bounds it chose (FP32 path 1e-5).
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1308_5467_amd as kpm
import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = kpm.Context(0)
    yield c
    c.close()


def dev(A, dtype):
    vals = A.val if dtype == "f64" else A.val.astype(np.float32)
    return kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, vals, dtype)


@pytest.mark.parametrize("M,npts,per_matrix", [(0, 1, False), (96, 130, False), (127, 200, True),
                                               (4100, 67, True)])
def test_dos_batched_rows_equal_single_calls_and_oracle(ctx, M, npts, per_matrix):
    """Degree 0, a ragged last point tile, per-matrix factors, and a series
    too long for the LDS staging (4,101 > 4,096 coefficients); points
    outside each interval (density 0) included."""
    rng = np.random.default_rng(M + npts)
    nmat = 5
    mu = rng.uniform(-1, 1, (nmat, M + 1)) / (1.0 + np.arange(M + 1))
    mu[:, 0] = 1.0
    lb = rng.uniform(-5, -1, nmat)
    ub = lb + rng.uniform(2, 9, nmat)
    g = rng.uniform(0, 1, (nmat, M + 1)) if per_matrix else oracle.jackson(M)
    x = np.stack([np.linspace(lb[m] - 0.5, ub[m] + 0.5, npts) for m in range(nmat)])
    phi = kpm.kpm_dos_batched(ctx, mu, g, lb, ub, x)
    for m in range(nmat):
        gm = g[m] if per_matrix else g
        assert np.array_equal(phi[m], kpm.kpm_dos(ctx, mu[m], gm, lb[m], ub[m], x[m])), m
        ref = oracle.dos(mu[m], gm, lb[m], ub[m], x[m])
        assert np.max(np.abs(phi[m] - ref)) <= 1e-11 * max(np.max(np.abs(ref)), 1e-300), m


def _mixed():
    return [synth.laplacian2d_dirichlet(32),
            synth.add_diagonal_disorder(synth.laplacian3d_periodic(12), 16.0, 5),
            synth.random_sparse_symmetric(2000, 4.5, 8),
            synth.add_diagonal_disorder(synth.laplacian2d_dirichlet(70), 8.0, 9),
            synth.random_sparse_symmetric(7, 2.0, 3),
            synth.add_diagonal_disorder(synth.laplacian3d_periodic(20), 2.0, 10)]


@pytest.mark.parametrize("damping,M", [(kpm.KPM_DAMP_JACKSON, 150), (kpm.KPM_DAMP_NONE, 64),
                                       (kpm.KPM_DAMP_LEARNED, 127), (kpm.KPM_DAMP_LEARNED, 40)])
def test_pipeline_batched_equals_separate_calls(ctx, damping, M):
    if damping == kpm.KPM_DAMP_LEARNED:
        kpm.kpm_mlp_init(ctx, 5)
    mats = _mixed()
    D = [dev(A, "f32") for A in mats]
    nvec, seed = 24, 41
    lb0, ub0 = kpm.kpm_bounds_batched(ctx, D, 20, 3003, 0.01)
    x = np.stack([np.linspace(lb0[m], ub0[m], 90) for m in range(len(D))])
    _say(f"pipeline batched: damping {damping}, M {M}")
    phi, mu, lb, ub, att = kpm.kpm_dos_pipeline_batched(ctx, D, M, nvec, seed, x, damping=damping)
    assert np.all(att == 1)
    for m, d in enumerate(D):
        assert (lb[m], ub[m]) == kpm.kpm_bounds(ctx, d, 20, 3003, 0.01), m
    rmu = kpm.kpm_moments_batched(ctx, D, lb, ub, M, nvec, seed)
    assert np.array_equal(mu, rmu)
    for m in range(len(D)):
        g = kpm.kpm_damping_factors(ctx, damping, M, mu[m])
        assert np.array_equal(phi[m], kpm.kpm_dos(ctx, mu[m], g, lb[m], ub[m], x[m])), m
    for m in (0, 2, 4):
        ref = oracle.moments(mats[m].rounded_f32(), lb[m], ub[m], M, nvec, seed + m)
        assert np.max(np.abs(mu[m] - ref)) < 1e-5, m


def test_pipeline_batched_escape_recovery_matches_robust(ctx):
    """One Lanczos step gives bounds far too narrow for these spectra: the
    moments escape, the margin x4 does not help and the Gershgorin interval
    is taken (third attempt), as kpm_moments_robust does per matrix."""
    mats = [synth.laplacian2d_dirichlet(32),
            synth.add_diagonal_disorder(synth.laplacian3d_periodic(12), 4.0, 5),
            synth.random_sparse_symmetric(2000, 4.5, 8)]
    D = [dev(A, "f32") for A in mats]
    M, nvec, seed = 60, 8, 5
    x = np.stack([np.linspace(-10.0, 15.0, 50) for _ in D])
    _say("pipeline batched: escape recovery")
    phi, mu, lb, ub, att = kpm.kpm_dos_pipeline_batched(ctx, D, M, nvec, seed, x, lanczos_steps=1,
                                                        lanczos_seed=7)
    for m, d in enumerate(D):
        rmu, rlb, rub, ratt = kpm.kpm_moments_robust(ctx, d, M, nvec, seed + m, steps=1, lanczos_seed=7,
                                                     validate=False)
        assert (lb[m], ub[m], att[m]) == (rlb, rub, ratt), m
        # fewer than 16 escaping matrices: recovered one by one on the
        # single-matrix path, as kpm_moments_robust does
        assert np.array_equal(mu[m], rmu), m
        lam = np.linalg.eigvalsh(mats[m].rounded_f32().dense())
        assert lb[m] < lam[0] and ub[m] > lam[-1]
    assert np.all(att >= 2)
    assert np.all(np.abs(mu) <= 1 + 1e-6)
    ref = oracle.moments(mats[0].rounded_f32(), lb[0], ub[0], M, nvec, seed)
    assert np.max(np.abs(mu[0] - ref)) < 1e-5
    g = kpm.kpm_damping_factors(ctx, kpm.KPM_DAMP_JACKSON, M)
    for m in range(len(D)):
        assert np.array_equal(phi[m], kpm.kpm_dos(ctx, mu[m], g, lb[m], ub[m], x[m]))


# 20 random sparse matrices (n = 300) whose 4-step Lanczos bounds with a 1 %
# margin miss an extreme eigenvalue by 0.6 % of the half-width or more and
# with a 4 % margin enclose the spectrum (found with the oracle's bounds and
# dense eigh)
_SUBBATCH_SEEDS = (105, 109, 118, 119, 125, 130, 131, 133, 136, 140, 146, 147, 154, 156, 159, 165, 168, 174,
                   181, 184)


def test_pipeline_batched_recovers_many_escapes_as_one_sub_batch(ctx):
    """Sixteen or more escaping matrices are recovered in one sub-batch, each
    with its own probes: intervals and attempts as kpm_moments_robust, the
    moments bitwise those of a one-matrix batch call with seed + m (the
    on-chip path runs every (matrix, probe block) pair in its own
    workgroup), and at the oracle's bar."""
    mats = [synth.random_sparse_symmetric(300, 4.5, sd) for sd in _SUBBATCH_SEEDS]
    D = [dev(A, "f32") for A in mats]
    M, nvec, seed = 120, 16, 9
    x = np.stack([np.linspace(-8.0, 8.0, 40) for _ in D])
    _say("pipeline batched: 20 escapes in one sub-batch")
    phi, mu, lb, ub, att = kpm.kpm_dos_pipeline_batched(ctx, D, M, nvec, seed, x, lanczos_steps=4,
                                                        lanczos_seed=7, damping=kpm.KPM_DAMP_NONE)
    assert np.all(att == 2)
    for m in range(len(D)):
        rmu, rlb, rub, ratt = kpm.kpm_moments_robust(ctx, D[m], M, nvec, seed + m, steps=4, lanczos_seed=7,
                                                     validate=False)
        assert (lb[m], ub[m], att[m]) == (rlb, rub, ratt), m
        assert np.max(np.abs(mu[m] - rmu)) < 1e-5, m
        lam = np.linalg.eigvalsh(mats[m].rounded_f32().dense())
        assert lb[m] < lam[0] and ub[m] > lam[-1], m
    for m in (0, 7, 19):
        one = kpm.kpm_moments_batched(ctx, [D[m]], lb[m:m + 1], ub[m:m + 1], M, nvec, seed + m)
        assert np.array_equal(mu[m], one[0]), m
        ref = oracle.moments(mats[m].rounded_f32(), lb[m], ub[m], M, nvec, seed + m)
        assert np.max(np.abs(mu[m] - ref)) < 1e-5, m
    g = np.ones(M + 1)
    for m in (0, 19):
        assert np.array_equal(phi[m], kpm.kpm_dos(ctx, mu[m], g, lb[m], ub[m], x[m]))


def test_pipeline_batched_uneven_batch(ctx):
    """The 48 uneven matrices: matrix 41 (3D Anderson 45^3, W = 16) escapes
    its 20-step bounds (a localised edge state) and is recovered; every other
    matrix keeps its first bounds."""
    mats = synth.batched_uneven_set(48)
    D = [dev(A, "f32") for A in mats]
    lb0, ub0 = kpm.kpm_bounds_batched(ctx, D, 20, 3003, 0.01)
    x = np.stack([np.linspace(lb0[m], ub0[m], 202)[1:-1] for m in range(48)])
    _say("pipeline batched: uneven batch")
    phi, mu, lb, ub, att = kpm.kpm_dos_pipeline_batched(ctx, kpm.MatrixBatch(D), 80, 32, 2003, x,
                                                        damping=kpm.KPM_DAMP_NONE)
    assert att[41] >= 2 and np.sum(att > 1) == 1
    keep = np.arange(48) != 41
    assert np.array_equal(lb[keep], lb0[keep]) and np.array_equal(ub[keep], ub0[keep])
    assert ub[41] > ub0[41]
    assert np.all(np.abs(mu) <= 1 + 1e-4)
    # the other rows from the batched call, the recovered one from its own run
    rmu = kpm.kpm_moments_batched(ctx, D, lb, ub, 80, 32, 2003)
    assert np.array_equal(mu[keep], rmu[keep])
    # matrix 41 recovered alone on the single-matrix path, with its own probes
    assert np.array_equal(mu[41], kpm.kpm_moments(ctx, D[41], lb[41], ub[41], 80, 32, 2003 + 41, validate=False))
    assert np.max(np.abs(mu[41] - rmu[41])) < 1e-5
    g = np.ones(81)
    for m in (0, 41, 47):
        assert np.array_equal(phi[m], kpm.kpm_dos(ctx, mu[m], g, lb[m], ub[m], x[m]))


def test_pipeline_batched_bad_arguments(ctx):
    A = synth.laplacian2d_dirichlet(8)
    D = [dev(A, "f32")]
    x = np.zeros((1, 3))
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_dos_pipeline_batched(ctx, D, 10, 4, 1, x, damping=7)
    assert e.value.status == -1
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_dos_pipeline_batched(ctx, D, 200, 4, 1, x, damping=kpm.KPM_DAMP_LEARNED)
    assert e.value.status == -1
    with pytest.raises(ValueError):
        kpm.kpm_dos_pipeline_batched(ctx, D, 10, 4, 1, np.zeros((2, 3)))
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_dos_batched(ctx, np.ones((2, 3)), np.ones(3), [0.0, 1.0], [1.0, 1.0], np.zeros((2, 4)))
    assert e.value.status == -1 and "matrix 1" in e.value.message
