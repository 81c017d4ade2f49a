"""kpm_moments_noalloc through the C ABI against kpm_moments.

The no-allocation entry point runs the same launches with the same
geometry as kpm_moments, its work memory in the library's per-device
scratch array instead of context workspace, and writes device outputs
without waiting.  Its moments are checked against kpm_moments' at the
moments' bar (FP32 path 1e-5, FP64 path 1e-12 absolute, per probe) and
must in fact be bitwise equal.  Two calls in a row, the second with a
smaller matrix, fewer probes and a lower degree, so that stale contents
of the shared array from the first call would show.
"""
import sys

import numpy as np
import pytest

import paper_1308_5467_amd as kpm
import synth

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}


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


def _dev(A, prec):
    vals = A.val if prec == "f64" else A.val.astype(np.float32)
    return kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, vals, prec)


def _compare(ctx, A, prec, M, nvec, seed, block, per_vector=True):
    import torch
    D = _dev(A, prec)
    lb, ub = kpm.kpm_bounds(ctx, D, 20, seed + 1, 0.01)
    mu_ref, pv_ref = kpm.kpm_moments(ctx, D, lb, ub, M, nvec, seed, precision=prec, block=block,
                                     validate=True, per_vector=True)
    mu_t = torch.full((M + 1,), float("nan"), dtype=torch.float64, device="cuda")
    pv_t = (torch.full((nvec * (M + 1),), float("nan"), dtype=torch.float64, device="cuda")
            if per_vector else None)
    _say(f"noalloc: n={A.n} prec={prec} M={M} nvec={nvec} block={block} per_vector={per_vector}")
    kpm.kpm_moments_noalloc(ctx, D, lb, ub, M, nvec, seed, mu_t, pv_t, precision=prec, block=block)
    torch.cuda.synchronize()
    mu = mu_t.cpu().numpy()
    assert np.max(np.abs(mu - mu_ref)) <= TOL[prec]
    assert np.array_equal(mu, mu_ref)
    if per_vector:
        pv = pv_t.cpu().numpy().reshape(nvec, M + 1)
        assert np.max(np.abs(pv - pv_ref)) <= TOL[prec]
        assert np.array_equal(pv, pv_ref)


def test_noalloc_matches_moments_two_calls(ctx):
    """First a 40^3 Anderson matrix (FP32, degree 101, 70 probes as a block
    of 64 and a ragged block of 6), then a 12^3 one (degree 40, 20 probes):
    per-probe and mean moments equal kpm_moments' each time."""
    big = synth.add_diagonal_disorder(synth.laplacian3d_periodic(40), 16.0, 71)
    small = synth.add_diagonal_disorder(synth.laplacian3d_periodic(12), 16.0, 72)
    _compare(ctx, big, "f32", 101, 70, 501, 64)
    _compare(ctx, small, "f32", 40, 20, 502, 0)


def test_noalloc_fp64_then_smaller_without_per_probe_output(ctx):
    """FP64 path with FP64 values (blocks of 32 and a ragged 3), then a
    smaller matrix whose per-probe moments stay in the scratch array."""
    A = synth.add_long_range(synth.add_diagonal_disorder(synth.laplacian3d_periodic(20), 8.0, 73), 2.0, 0.1, 74)
    B = synth.random_sparse_symmetric(300, 4.5, 75)
    _compare(ctx, A, "f64", 64, 35, 503, 32)
    _compare(ctx, B, "f64", 17, 9, 504, 0, per_vector=False)
    _compare(ctx, B, "f32", 0, 3, 505, 0)


def test_noalloc_rejects_oversized_problems_and_bad_arguments(ctx):
    """A problem whose probe blocks exceed the scratch array is refused
    before anything is enqueued; host matrices, FP64 values on the FP32
    path and validation are refused too.  The entry point still works
    afterwards."""
    import torch
    n = 600_000  # two blocks of n x 64 FP32 values: 307 MB > 256 MiB
    A = synth.diagonal_matrix(np.linspace(-1.0, 1.0, n))
    D = _dev(A, "f32")
    mu = torch.zeros(11, dtype=torch.float64, device="cuda")
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_moments_noalloc(ctx, D, -1.5, 1.5, 10, 64, 1, mu)
    assert e.value.status == -1 and "scratch" in str(e.value)
    D64 = _dev(A, "f64")
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_moments_noalloc(ctx, D64, -1.5, 1.5, 10, 4, 1, mu, precision="f32")
    assert e.value.status == -1
    lib = kpm.load_library()
    H = kpm.HostCSR(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32))
    o = kpm._opts(10, 4, 1, "f32", 0, False, 0)
    c = H.as_c()
    import ctypes
    assert lib.kpm_moments_noalloc(ctx.handle, ctypes.byref(c), -1.5, 1.5, ctypes.byref(o),
                                   ctypes.c_void_p(mu.data_ptr()), None) == -1
    o = kpm._opts(10, 4, 1, "f32", 0, True, 0)
    c = D.as_c()
    assert lib.kpm_moments_noalloc(ctx.handle, ctypes.byref(c), -1.5, 1.5, ctypes.byref(o),
                                   ctypes.c_void_p(mu.data_ptr()), None) == -6
    o = kpm._opts(10, 4, 1, "f32", 0, False, 0, kpm.KPM_FLAG_LOCALITY)
    assert lib.kpm_moments_noalloc(ctx.handle, ctypes.byref(c), -1.5, 1.5, ctypes.byref(o),
                                   ctypes.c_void_p(mu.data_ptr()), None) == -6
    # a diagonal matrix: the Rademacher estimator is exact
    s = (np.linspace(-1.0, 1.0, 1000) - 0.0) / 1.5
    Asmall = synth.diagonal_matrix(np.linspace(-1.0, 1.0, 1000))
    Ds = _dev(Asmall, "f32")
    kpm.kpm_moments_noalloc(ctx, Ds, -1.5, 1.5, 10, 4, 1, mu)
    torch.cuda.synchronize()
    exact = np.array([np.mean(np.cos(k * np.arccos(s.astype(np.float32).astype(np.float64)))) for k in range(11)])
    assert np.max(np.abs(mu.cpu().numpy() - exact)) < 1e-5
