"""The runtime entry points around the path: the context's stream
(kpm_create with a caller stream, kpm_set_stream), the device timing of the
library's kernels (kpm_profile_*) and the copy probe (kpm_hbm_copy_probe)."""
import sys

import numpy as np
import pytest

import oracle
import paper_1308_5467_amd as kpm
import synth

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _matrix():
    return synth.add_diagonal_disorder(synth.laplacian3d_periodic(16), 8.0, 31)


def _ref(A, lb, ub, M, nvec, seed):
    c, d = oracle.rescale(lb, ub)
    return oracle.moments_per_vector(A.rounded_f32(), c, d, M, nvec, seed) / A.n


def test_work_is_ordered_on_the_callers_stream():
    """A context made on a caller stream, and one moved there with
    kpm_set_stream, enqueue on that stream: the matrix values are halved on
    the stream behind a ~20 ms device spin, and the moments that follow are
    those of the halved matrix (work on any other stream would read the old
    values).  The no-allocation call's device outputs are read on the same
    stream without a host wait."""
    import torch
    _say("caller stream ordering")
    A = _matrix()
    half = synth.CSR(A.n, A.row_ptr, A.col_idx, A.val * 0.5)
    lb, ub = -4.5, 16.5  # encloses both spectra: [0, 12] + [-4, 4] and half of it
    s = torch.cuda.Stream()  # default priority
    for how in ("create", "set"):
        D = kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32), "f32")
        torch.cuda.synchronize()
        if how == "create":
            ctx = kpm.Context(0, stream=s.cuda_stream)
        else:
            ctx = kpm.Context(0)
            kpm.kpm_set_stream(ctx, s.cuda_stream)
        with torch.cuda.stream(s):
            torch.cuda._sleep(50_000_000)
            D.val.mul_(0.5)
        _, pv = kpm.kpm_moments(ctx, D, lb, ub, 30, 6, 4, validate=False, per_vector=True)
        assert np.max(np.abs(pv - _ref(half, lb, ub, 30, 6, 4))) < TOL32, how
        # no host wait: the outputs are read on the same stream
        mu = torch.empty(31, dtype=torch.float64, device="cuda")
        with torch.cuda.stream(s):
            torch.cuda._sleep(50_000_000)
            D.val.mul_(2.0)
        kpm.kpm_moments_noalloc(ctx, D, lb, ub, 30, 6, 4, mu)
        with torch.cuda.stream(s):
            got = mu.clone()
        s.synchronize()
        assert np.max(np.abs(got.cpu().numpy() - _ref(A, lb, ub, 30, 6, 4).mean(axis=0))) < TOL32, how
        ctx.close()
    torch.cuda.synchronize()


def test_profile_counts_the_library_launches():
    """kpm_profile_*: with timing on, a moment call of degree M over b
    blocks records b first steps and b (ceil(M/2) - 1) fused steps, a bounds
    call one Lanczos run; times are positive; reset clears them; with timing
    off nothing is recorded; an unknown name reads 0."""
    _say("profile counters")
    A = _matrix()
    D = kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32), "f32")
    ctx = kpm.Context(0)
    lb, ub = kpm.kpm_bounds(ctx, D, 20, 3, 0.01)
    kpm.kpm_profile_reset(ctx)
    kpm.kpm_profile_enable(ctx, True)
    kpm.kpm_bounds(ctx, D, 20, 3, 0.01)
    kpm.kpm_moments(ctx, D, lb, ub, 41, 70, 5, block=64)  # 2 blocks (64 + 6), 21 steps each
    n_first, t_first = kpm.kpm_profile_query(ctx, "cheb_first")
    n_step, t_step = kpm.kpm_profile_query(ctx, "cheb_step")
    n_lz, t_lz = kpm.kpm_profile_query(ctx, "lanczos")
    assert (n_first, n_step, n_lz) == (2, 2 * 20, 1)
    assert t_first > 0 and t_step > 0 and t_lz > 0
    assert kpm.kpm_profile_query(ctx, "no_such_kernel") == (0, 0.0)
    kpm.kpm_profile_reset(ctx)
    assert kpm.kpm_profile_query(ctx, "cheb_step") == (0, 0.0)
    kpm.kpm_profile_enable(ctx, False)
    kpm.kpm_moments(ctx, D, lb, ub, 41, 8, 5)
    assert kpm.kpm_profile_query(ctx, "cheb_step") == (0, 0.0)
    ctx.close()


def test_copy_probe():
    """The copy probe reports a positive rate below twice the 8 TB/s peak
    (reads + writes of a 64 MiB copy) and refuses sizes out of range."""
    ctx = kpm.Context(0)
    g = kpm.kpm_hbm_copy_probe(ctx, 64 << 20, 3)
    assert 100.0 < g < 16000.0, g
    for nbytes, iters in ((1024, 3), (64 << 20, 0)):
        with pytest.raises(kpm.KpmError) as e:
            kpm.kpm_hbm_copy_probe(ctx, nbytes, iters)
        assert e.value.status == -1
    ctx.close()
