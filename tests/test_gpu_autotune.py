"""GPU tests of the measured geometry choice (kpm_autotune,
kpm_autotune_batched) and of the gather-width flag: whatever geometry is
chosen, the moments stay within the parity bar against the CPU oracle (FP32
path 1e-5, FP64 path 1e-12) and are bitwise reproducible for that geometry.
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


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("f64", 1e-12)])
def test_gather_widths_match_oracle(ctx, dtype, tol):
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(13), 16.0, 5)
    A = synth.add_long_range(A, 1.0, 0.1, 6)  # rows of 7 to ~11 entries: two batches of 8 or three of 4
    Ao = A if dtype == "f64" else A.rounded_f32()
    b = oracle.lanczos_bounds(Ao, 20, 3)
    D = dev(A, dtype)
    ref = oracle.moments(Ao, b["lb"], b["ub"], 50, 12, 41)
    for gather in (4, 7, 8):
        mu = kpm.kpm_moments(ctx, D, b["lb"], b["ub"], 50, 12, 41, precision=dtype, block=8, gather=gather)
        assert np.max(np.abs(mu - ref)) < tol, gather
    with pytest.raises(ValueError):
        kpm.kpm_moments(ctx, D, b["lb"], b["ub"], 10, 2, 1, precision=dtype, gather=5)


def test_autotune_single_matrix(ctx):
    _say("autotune single matrix")
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(24), 16.0, 7)
    D = dev(A, "f32")
    lb, ub = kpm.kpm_bounds(ctx, D, 20, 3, 0.01)
    t = kpm.kpm_autotune(ctx, D, lb, ub, 64, seed=5)
    _say(f"chosen {t}")
    assert t["block"] in (32, 64) and t["gather"] in (4, 7, 8) and t["rows_per_block"] > 0 and t["us_per_step"] > 0
    mu1 = kpm.kpm_moments(ctx, D, lb, ub, 64, 64, 5, block=t["block"], rows_per_block=t["rows_per_block"],
                          gather=t["gather"])
    mu2 = kpm.kpm_moments(ctx, D, lb, ub, 64, 64, 5, block=t["block"], rows_per_block=t["rows_per_block"],
                          gather=t["gather"])
    assert np.array_equal(mu1, mu2)
    ref = oracle.moments(A.rounded_f32(), lb, ub, 64, 64, 5)
    assert np.max(np.abs(mu1 - ref)) < 1e-5
    # a fixed block width is kept; FP64 candidates
    t64 = kpm.kpm_autotune(ctx, dev(A, "f64"), lb, ub, 40, precision="f64", block=16)
    assert t64["block"] == 16
    # on the renumbered matrix (KPM_FLAG_LOCALITY): the chosen geometry with
    # the flag gives the oracle's moments
    tl = kpm.kpm_autotune(ctx, D, lb, ub, 64, seed=5, locality=True)
    _say(f"chosen with the locality renumbering {tl}")
    assert tl["block"] in (32, 64) and tl["gather"] in (4, 7, 8) and tl["us_per_step"] > 0
    mul = kpm.kpm_moments(ctx, D, lb, ub, 64, 64, 5, block=tl["block"], rows_per_block=tl["rows_per_block"],
                          gather=tl["gather"], locality=True)
    assert np.max(np.abs(mul - ref)) < 1e-5


def test_autotune_batched(ctx):
    _say("autotune batched")
    mats = [synth.add_diagonal_disorder(synth.laplacian2d_dirichlet(L), W, 10 + L)
            for L, W in ((24, 2.0), (40, 8.0))]
    mats += [synth.add_diagonal_disorder(synth.laplacian3d_periodic(L), W, 20 + L) for L, W in ((10, 16.0), (14, 2.0))]
    D = [dev(A, "f32") for A in mats]
    bl = [oracle.lanczos_bounds(A.rounded_f32(), 20, 7) for A in mats]
    lb = np.array([b["lb"] for b in bl])
    ub = np.array([b["ub"] for b in bl])
    t = kpm.kpm_autotune_batched(ctx, D, lb, ub, 32, seed=9)
    _say(f"chosen {t}")
    assert t["block"] in (16, 32) and t["rows_per_block"] > 0 and t["us_per_step"] > 0
    mu = kpm.kpm_moments_batched(ctx, D, lb, ub, 40, 32, 9, block=t["block"], rows_per_block=t["rows_per_block"])
    for m in (0, 3):
        ref = oracle.moments(mats[m].rounded_f32(), lb[m], ub[m], 40, 32, 9 + m)
        assert np.max(np.abs(mu[m] - ref)) < 1e-5, m
