"""GPU parity of the batched path (many matrices of uneven size, one launch
per recurrence step, HIP-graph replay) against the CPU oracle.

Tolerances: FP32 path 1e-5, FP64 path 1e-12 absolute on every normalised
moment; graph replays must equal the directly launched sequence bitwise.
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


def small_set():
    mats = [synth.add_diagonal_disorder(synth.laplacian2d_dirichlet(L), W, 10 + L)
            for L, W in ((8, 2.0), (13, 8.0), (20, 16.0))]
    mats += [synth.add_diagonal_disorder(synth.laplacian3d_periodic(L), W, 20 + L)
             for L, W in ((5, 2.0), (7, 8.0), (9, 16.0))]
    mats.append(synth.random_sparse_symmetric(777, 4.5, 3))
    return mats


def bounds_of(mats, dtype):
    out = [oracle.lanczos_bounds(A if dtype == "f64" else A.rounded_f32(), 20, 7) for A in mats]
    return np.array([b["lb"] for b in out]), np.array([b["ub"] for b in out])


def dev(A, dtype):
    vals = A.val if dtype == "f64" else A.val.astype(np.float32)
    return kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, vals, dtype)


def oracle_mu(A, lb, ub, M, nvec, seed, dtype):
    Ao = A if dtype == "f64" else A.rounded_f32()
    return oracle.moments(Ao, lb, ub, M, nvec, seed)


@pytest.mark.parametrize("dtype,tol,M,nvec,block,path", [
    ("f32", 1e-5, 40, 10, 4, "auto"), ("f64", 1e-12, 33, 6, 0, "auto"), ("f32", 1e-5, 1, 3, 0, "auto"),
    ("f32", 1e-5, 0, 2, 0, "auto"), ("f32", 1e-5, 3, 5, 0, "auto"), ("f64", 1e-12, 4, 3, 2, "auto"),
    ("f32", 1e-5, 40, 10, 0, "stream"), ("f64", 1e-12, 33, 6, 0, "stream"),
    ("f32", 1e-5, 41, 10, 4, "resident"), ("f32", 1e-5, 40, 37, 8, "resident"), ("f32", 1e-5, 12, 70, 16, "resident"),
    ("f64", 1e-12, 33, 7, 2, "resident"), ("f64", 1e-12, 32, 9, 4, "resident"), ("f64", 1e-12, 2, 3, 8, "resident"),
    ("f64", 1e-12, 0, 3, 0, "resident")])
def test_batched_parity_small(ctx, dtype, tol, M, nvec, block, path):
    """Both device paths, block widths of the on-chip path (N, 2N, 4N values:
    4/8/16 FP32, 2/4/8 FP64) with ragged last blocks, odd and even degrees
    and the degenerate M = 0, 1."""
    _say(f"batched small {dtype} M={M} nvec={nvec} block={block} path={path}")
    mats = small_set()
    lb, ub = bounds_of(mats, dtype)
    D = [dev(A, dtype) for A in mats]
    mu = kpm.kpm_moments_batched(ctx, D, lb, ub, M, nvec, 500, precision=dtype, block=block, validate=True,
                                 path=path)
    for m, A in enumerate(mats):
        ref = oracle_mu(A, lb[m], ub[m], M, nvec, 500 + m, dtype)
        assert np.max(np.abs(mu[m] - ref)) < tol, m
        assert mu[m, 0] == 1.0


@pytest.mark.parametrize("path", ["resident", "stream"])
def test_graph_replay_matches_direct_launch(ctx, path):
    """Replays of the captured graph, with eager work and syncs between them,
    equal the directly launched sequence bitwise; changing the bounds between
    calls updates the replay's scalars."""
    import torch
    mats = small_set()
    lb, ub = bounds_of(mats, "f32")
    D = [dev(A, "f32") for A in mats]
    kw = dict(path=path)
    direct = kpm.kpm_moments_batched(ctx, D, lb, ub, 50, 8, 9, graph=False, **kw)
    for rep in range(3):
        x = torch.randn(1 << 20, device="cuda")
        (x * 2.0).sum().item()  # eager work on the caller's stream
        got = kpm.kpm_moments_batched(ctx, D, lb, ub, 50, 8, 9, graph=True, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(got, direct), rep
    lb2, ub2 = lb - 0.5, ub + 0.25
    got2 = kpm.kpm_moments_batched(ctx, D, lb2, ub2, 50, 8, 9, graph=True, **kw)
    direct2 = kpm.kpm_moments_batched(ctx, D, lb2, ub2, 50, 8, 9, graph=False, **kw)
    assert np.array_equal(got2, direct2)
    assert not np.array_equal(got2, direct)
    got3 = kpm.kpm_moments_batched(ctx, D, lb, ub, 50, 8, 10, graph=True, **kw)  # new seed, same graph
    direct3 = kpm.kpm_moments_batched(ctx, D, lb, ub, 50, 8, 10, graph=False, **kw)
    assert np.array_equal(got3, direct3)


def test_paths_agree_and_flags(ctx):
    """The on-chip and streaming paths at the same probe block width compute
    bitwise the same vectors and sum the dots in different orders: the
    moments agree to rounding (1e-13 FP32 path, 1e-14 FP64).  The on-chip
    path refuses matrices too large for it; the two path flags exclude each
    other."""
    mats = small_set()
    for dtype, tol in (("f32", 1e-13), ("f64", 1e-14)):
        lb, ub = bounds_of(mats, dtype)
        D = [dev(A, dtype) for A in mats]
        for block in ((4, 8, 16) if dtype == "f32" else (2, 4, 8)):
            a = kpm.kpm_moments_batched(ctx, D, lb, ub, 61, 20, 31, precision=dtype, block=block, path="resident")
            b = kpm.kpm_moments_batched(ctx, D, lb, ub, 61, 20, 31, precision=dtype, block=block, path="stream")
            assert np.max(np.abs(a - b)) < tol, (dtype, block)
    big = synth.laplacian2d_dirichlet(100)  # n = 10,000: 2 x 10,000 x 4 FP32 values exceed 160 KB
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_moments_batched(ctx, [dev(big, "f32")], [-0.1], [8.1], 10, 4, 1, path="resident")
    assert e.value.status == -6
    import ctypes
    o = kpm._opts(10, 4, 1, "f32", 0, False, 0, kpm.KPM_FLAG_BATCH_STREAM | kpm.KPM_FLAG_BATCH_RESIDENT)
    arr = (kpm.kpm_csr * 1)(dev(big, "f32").as_c())
    lbv, ubv, mu = np.array([-0.1]), np.array([8.1]), np.zeros(11)
    assert ctx.lib.kpm_moments_batched(ctx.handle, 1, arr, kpm._p(lbv), kpm._p(ubv), ctypes.byref(o), kpm._p(mu),
                                       None) == -1


def test_batched_matches_single_matrix_path(ctx):
    mats = small_set()[:4]
    lb, ub = bounds_of(mats, "f32")
    D = [dev(A, "f32") for A in mats]
    mu = kpm.kpm_moments_batched(ctx, D, lb, ub, 64, 16, 77)
    for m in range(len(mats)):
        single = kpm.kpm_moments(ctx, D[m], lb[m], ub[m], 64, 16, 77 + m)
        assert np.max(np.abs(mu[m] - single)) < 1e-6


def test_batched_spectrum_escape(ctx):
    mats = small_set()[:3]
    lb, ub = bounds_of(mats, "f64")
    ub = ub.copy()
    ub[1] = lb[1] + 0.3 * (ub[1] - lb[1])
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_moments_batched(ctx, [dev(A, "f64") for A in mats], lb, ub, 100, 2, 1, precision="f64")
    assert e.value.status == -4 and "matrix 1" in e.value.message


def test_batched_rejects_host_matrices(ctx):
    A = synth.laplacian2d_dirichlet(8)
    H = kpm.HostCSR(A.n, A.row_ptr, A.col_idx, A.val)
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_moments_batched(ctx, [H], [-0.1], [8.1], 10, 2, 1, precision="f64")
    assert e.value.status == -1


def test_c3_full_size_sampled(ctx):
    """c3: 48 uneven matrices (n from 4,096 to 262,144), M = 200, 32 probes
    per matrix, FP32, one launch per step, graph replay.

    The 20-step Lanczos bound misses a localised edge state of matrix 41
    (3D Anderson 45^3, W = 16: true lambda_max 17.0045 above the bound):
    the batch reports that matrix's escape (max |mu| > 1), its bounds are
    widened (margin x4, then the Gershgorin hull) and the batch re-run.
    The oracle then checks the smallest, a middle, the largest and the
    recovered matrix over all 32 probes."""
    _say("c3 generating 48 matrices")
    mats = synth.batched_uneven_set(48)
    assert len(mats) == 48 and min(A.n for A in mats) == 4096 and max(A.n for A in mats) == 262144
    D = [dev(A, "f32") for A in mats]
    _say("c3 bounds")
    bl = [kpm.kpm_bounds(ctx, d, 20, 3003, 0.01) for d in D]
    lb = np.array([b[0] for b in bl])
    ub = np.array([b[1] for b in bl])
    recovered = set()
    for attempt in range(3):
        _say(f"c3 batched moments, attempt {attempt}")
        mu, mx = kpm.kpm_moments_batched(ctx, D, lb, ub, 200, 32, 2003, return_max_abs=True)
        bad = [m for m in range(48) if not mx[m] <= 1 + 1e-4]
        if not bad:
            break
        recovered.update(bad)
        for m in bad:
            if attempt == 0:
                lb[m], ub[m] = kpm.kpm_bounds(ctx, D[m], 20, 3003, 0.04)
            else:
                lo, hi = kpm.kpm_gershgorin(ctx, D[m])
                lb[m], ub[m] = lo - 0.01 * (hi - lo), hi + 0.01 * (hi - lo)
    assert not bad
    mu2 = kpm.kpm_moments_batched(ctx, D, lb, ub, 200, 32, 2003)
    assert np.array_equal(mu, mu2)
    assert np.all(mu[:, 0] == 1.0) and np.all(np.abs(mu) <= 1 + 1e-6)
    for m in sorted({0, 23, 47} | recovered):
        _say(f"c3 oracle matrix {m} (n={mats[m].n})")
        ref = oracle_mu(mats[m], lb[m], ub[m], 200, 32, 2003 + m, "f32")
        assert np.max(np.abs(mu[m] - ref)) < 1e-5, m


@pytest.mark.parametrize("dtype,tol,block", [("f32", 1e-5, 64), ("f64", 1e-12, 64), ("f32", 1e-5, 0),
                                             ("f64", 1e-12, 0)])
def test_many_small_matrices_every_matrix(ctx, dtype, tol, block):
    """More (matrix, probe block) pairs than resident workgroups (3,000
    random sparse matrices, n = 150..349, 64 probes each).  Block 64: the
    streaming path's work table then splits every pair over up to 16
    workgroups, and each step launch reduces the previous step's partials.
    Block 0: the on-chip path (16 FP32 / 8 FP64 probes per workgroup, 12,000
    / 24,000 pairs).  Every matrix against the oracle."""
    _say(f"many small matrices {dtype} block {block}")
    mats = [synth.random_sparse_symmetric(150 + (i * 37) % 200, 4.5, 50_000 + i) for i in range(3000)]
    D = [dev(A, dtype) for A in mats]
    lo_hi = [kpm.kpm_gershgorin(ctx, d) for d in D]
    lb = np.array([lo - 0.01 * (hi - lo) for lo, hi in lo_hi])
    ub = np.array([hi + 0.01 * (hi - lo) for lo, hi in lo_hi])
    M, nvec = 9, 64
    mu = kpm.kpm_moments_batched(ctx, D, lb, ub, M, nvec, 7000, precision=dtype, block=block)
    mu_direct = kpm.kpm_moments_batched(ctx, D, lb, ub, M, nvec, 7000, precision=dtype, block=block, graph=False)
    assert np.array_equal(mu, mu_direct)
    worst = 0.0
    for m, A in enumerate(mats):
        ref = oracle_mu(A, lb[m], ub[m], M, nvec, 7000 + m, dtype)
        worst = max(worst, float(np.max(np.abs(mu[m] - ref))))
    _say(f"many small matrices {dtype}: worst |mu - oracle| = {worst:.3e}")
    assert worst < tol


def test_training_set_full_size_sampled(ctx):
    """The damping network's training family at full size in one batched
    call: 8,192 random sparse symmetric matrices (n = 2,048) and 1,024 2D
    Anderson 32 x 64 matrices, degree 127, 256 probes each, FP32: on the
    on-chip path (blocks of 8 probes, 294,912 (matrix, probe block) pairs,
    one workgroup each) and on the streaming path (4 blocks of 64, 36,864
    pairs).  Bounds: 20-step Lanczos (one batched call, bitwise the
    per-matrix calls on sampled matrices) with the same escape recovery as the
    uneven batch (random sparse matrices often have an outlying extreme
    eigenvalue the start vector barely sees).  The oracle checks matrices at
    both ends of each family and a few recovered ones over all 256 probes;
    the two paths agree to rounding on every matrix."""
    _say("training set: generating 9,216 matrices")
    mats = synth.damping_training_set()
    assert len(mats) == 9216 and all(A.n == 2048 for A in mats)
    D = [dev(A, "f32") for A in mats]
    _say("training set: bounds (one batched Lanczos call)")
    lb, ub = kpm.kpm_bounds_batched(ctx, D, 20, 3004, 0.01)
    for m in list(range(0, 9216, 577)) + [8191, 8192, 9215]:
        assert (lb[m], ub[m]) == kpm.kpm_bounds(ctx, D[m], 20, 3004, 0.01), m
    recovered = []
    for attempt in range(3):
        _say(f"training set: batched moments, attempt {attempt}")
        mu, mx = kpm.kpm_moments_batched(ctx, D, lb, ub, 127, 256, 2004, return_max_abs=True)
        bad = [m for m in range(len(D)) if not mx[m] <= 1 + 1e-4]
        if not bad:
            break
        recovered += bad
        if attempt == 0:
            lb[bad], ub[bad] = kpm.kpm_bounds_batched(ctx, [D[m] for m in bad], 20, 3004, 0.04)
            assert (lb[bad[0]], ub[bad[0]]) == kpm.kpm_bounds(ctx, D[bad[0]], 20, 3004, 0.04)
            continue
        for m in bad:
            lo, hi = kpm.kpm_gershgorin(ctx, D[m])
            lb[m], ub[m] = lo - 0.01 * (hi - lo), hi + 0.01 * (hi - lo)
    assert not bad
    mu2 = kpm.kpm_moments_batched(ctx, D, lb, ub, 127, 256, 2004)
    assert np.array_equal(mu, mu2)
    _say("training set: streaming path")
    mu_s = kpm.kpm_moments_batched(ctx, D, lb, ub, 127, 256, 2004, block=64)
    _say(f"training set: paths differ by {np.max(np.abs(mu - mu_s)):.2e}")
    assert np.max(np.abs(mu - mu_s)) < 1e-12
    assert mu.shape == (9216, 128)
    assert np.all(mu[:, 0] == 1.0) and np.all(np.abs(mu) <= 1 + 1e-6)
    for m in sorted({0, 1, 4095, 8191, 8192, 9215} | set(recovered[:4])):
        _say(f"training set: oracle matrix {m}")
        ref = oracle_mu(mats[m], lb[m], ub[m], 127, 256, 2004 + m, "f32")
        assert np.max(np.abs(mu[m] - ref)) < 1e-5, m


def test_robust_single_matrix_recovers_escape(ctx):
    """The same edge-state miss on matrix 41 of the uneven set, through the
    single-matrix robust entry point."""
    A = synth.batched_uneven_set(48)[41]
    D = dev(A, "f32")
    mu, lb, ub, attempts, pv = kpm.kpm_moments_robust(ctx, D, 200, 8, 2041, steps=20, lanczos_seed=3003,
                                                      margin=0.01, per_vector=True)
    assert attempts >= 2 and np.all(np.abs(pv) <= 1 + 1e-5)
    ref = oracle_mu(A, lb, ub, 200, 8, 2041, "f32")
    assert np.max(np.abs(mu - ref)) < 1e-5
    with pytest.raises(kpm.KpmError) as e:
        l0, u0 = kpm.kpm_bounds(ctx, D, 20, 3003, 0.01)
        kpm.kpm_moments(ctx, D, l0, u0, 200, 8, 2041)
    assert e.value.status == -4


def test_gershgorin_matches_oracle(ctx):
    for A in small_set():
        lo, hi = kpm.kpm_gershgorin(ctx, dev(A, "f64"))
        rlo, rhi = oracle.gershgorin(A)
        assert abs(lo - rlo) < 1e-12 * max(1, abs(rlo)) and abs(hi - rhi) < 1e-12 * max(1, abs(rhi))


def test_on_chip_plan_detects_changed_structure(ctx):
    """The on-chip path lays each matrix out in slices whose widths are fixed
    when the plan is built; values are re-read at every call.  A caller that
    rewrites a matrix's structure in place (same addresses and sizes) gets
    KPM_ERR_ARG once, and the next call rebuilds the plan and matches the
    oracle."""
    import torch
    n = 96
    A = synth.add_diagonal_disorder(synth.laplacian2d_dirichlet(8), 2.0, 5)  # n = 64
    B = synth.random_sparse_symmetric(n, 1.0, 6)
    # the same sizes: pad B's entry count to A2's with zeros on the diagonal block
    A2 = synth.random_sparse_symmetric(n, 3.0, 7)
    assert B.nnz < A2.nnz
    Sb = B.to_scipy().tolil()
    pairs = ((i, j) for i in range(n) for j in range(i + 1, n))
    while Sb.nnz < A2.nnz:  # long first rows, kept symmetric (2 entries per new pair)
        i, j = next(pairs)
        if Sb[i, j] == 0:
            Sb[i, j] = Sb[j, i] = 1e-3
    Sb = Sb.tocsr()
    Sb.sort_indices()
    assert Sb.nnz == A2.nnz, (Sb.nnz, A2.nnz)
    Bm = synth.CSR(n, Sb.indptr.astype(np.int32), Sb.indices.astype(np.int32), Sb.data.copy())
    D = [dev(A, "f32"), dev(A2, "f32")]
    lb0, ub0 = bounds_of([A, A2], "f32")
    mu = kpm.kpm_moments_batched(ctx, D, lb0, ub0, 20, 8, 3, path="resident")
    # rewrite matrix 1 in place: same n and nnz, a row 0 longer than any of A2's rows
    D[1].row_ptr.copy_(torch.as_tensor(Bm.row_ptr, device="cuda"))
    D[1].col_idx.copy_(torch.as_tensor(Bm.col_idx, device="cuda"))
    D[1].val.copy_(torch.as_tensor(Bm.val.astype(np.float32), device="cuda"))
    lb, ub = bounds_of([A, Bm], "f32")
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_moments_batched(ctx, D, lb, ub, 20, 8, 3, path="resident")
    assert e.value.status == -1 and "structure" in e.value.message
    mu = kpm.kpm_moments_batched(ctx, D, lb, ub, 20, 8, 3, path="resident")
    for m, X in enumerate([A, Bm]):
        ref = oracle_mu(X, lb[m], ub[m], 20, 8, 3 + m, "f32")
        assert np.max(np.abs(mu[m] - ref)) < 1e-5, m


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_on_chip_high_degree(ctx, dtype, tol):
    """The on-chip path at a high degree (301: 151 steps in one launch) on
    matrices of several families and sizes (3D Anderson 6^3..10^3, 2D
    Anderson, random sparse), ragged probe blocks: every matrix against the
    oracle."""
    mats = [synth.add_diagonal_disorder(synth.laplacian3d_periodic(L), 8.0, 60 + L) for L in (6, 8, 10)]
    mats.append(synth.add_diagonal_disorder(synth.laplacian2d_periodic(20, 30), 4.0, 61))
    mats.append(synth.random_sparse_symmetric(900, 4.5, 62))
    lb, ub = bounds_of(mats, dtype)
    D = [dev(A, dtype) for A in mats]
    M, nvec = 301, 11
    mu = kpm.kpm_moments_batched(ctx, D, lb, ub, M, nvec, 900, precision=dtype, path="resident")
    mu_s = kpm.kpm_moments_batched(ctx, D, lb, ub, M, nvec, 900, precision=dtype, path="stream")
    for m, A in enumerate(mats):
        ref = oracle_mu(A, lb[m], ub[m], M, nvec, 900 + m, dtype)
        assert np.max(np.abs(mu[m] - ref)) < tol, m
        assert np.max(np.abs(mu[m] - mu_s[m])) < tol, m


def _arrow(n, seed):
    """Random sparse symmetric (about 10 entries per row) plus a dense row and
    column 0: one row of n entries beside short ones."""
    import scipy.sparse as sp
    R = synth.random_sparse_symmetric(n, 4.5, seed).to_scipy().tolil()
    v = np.random.default_rng(seed).normal(0.0, 0.3, n - 1)
    R[0, 1:] = v
    R[1:, 0] = v[:, None]
    return synth._from_scipy(sp.csr_matrix(R))


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("f64", 1e-12)])
@pytest.mark.parametrize("path,block", [("stream", 0), ("resident", 4)])
def test_long_rows(ctx, dtype, tol, path, block):
    """Long rows on both device paths: an arrow matrix (one row of 2,000
    entries beside short rows: streaming panels staged in LDS beside one
    read directly; on chip a first slice 2,000 slots wide) and a random
    symmetric matrix with about 200 entries in every row, against the
    oracle."""
    mats = [_arrow(2000, 61), synth.random_sparse_symmetric(2000, 100.0, 62, off_scale=0.1),
            synth.laplacian2d_dirichlet(20)]
    lb, ub = [], []
    for A in mats:
        lam = np.linalg.eigvalsh(A.dense())
        w = lam[-1] - lam[0]
        lb.append(lam[0] - 0.02 * w)
        ub.append(lam[-1] + 0.02 * w)
    D = [dev(A, dtype) for A in mats]
    mu = kpm.kpm_moments_batched(ctx, D, lb, ub, 45, 6, 70, precision=dtype, block=block, validate=True, path=path)
    for m, A in enumerate(mats):
        assert np.max(np.abs(mu[m] - oracle_mu(A, lb[m], ub[m], 45, 6, 70 + m, dtype))) < tol, m


def test_matrix_batch_descriptors_built_once(ctx):
    """A MatrixBatch (descriptors built once) gives bitwise the moments of the
    plain list, on both paths; values changed in place are seen by the next
    call through the same MatrixBatch."""
    import torch
    mats = small_set()
    lb, ub = bounds_of(mats, "f32")
    D = [dev(A, "f32") for A in mats]
    batch = kpm.MatrixBatch(D)
    assert len(batch) == len(D)
    for path in ("stream", "resident"):
        a = kpm.kpm_moments_batched(ctx, D, lb, ub, 30, 8, 3, path=path)
        b = kpm.kpm_moments_batched(ctx, batch, lb, ub, 30, 8, 3, path=path)
        assert np.array_equal(a, b), path
    D[0].val.mul_(0.5)
    A0 = synth.CSR(mats[0].n, mats[0].row_ptr, mats[0].col_idx, mats[0].val * 0.5)
    mu = kpm.kpm_moments_batched(ctx, batch, lb, ub, 30, 8, 3)
    torch.cuda.synchronize()
    assert np.max(np.abs(mu[0] - oracle_mu(A0, lb[0], ub[0], 30, 8, 3, "f32"))) < 1e-5


def test_two_cached_plans_alternate_and_a_third_evicts(ctx):
    """The context keeps the plans of the two most recently used shapes:
    alternating between two batches (on both paths) reuses both captured
    graphs, a third shape evicts the older plan, and every call gives
    bitwise the moments of the first call of its shape; the results stay at
    the oracle's bar."""
    mats = small_set()
    lb, ub = bounds_of(mats, "f32")
    D = [dev(A, "f32") for A in mats]
    shapes = [dict(mats=D, lb=lb, ub=ub, M=30, path="stream"),
              dict(mats=D[:3], lb=lb[:3], ub=ub[:3], M=24, path="resident"),
              dict(mats=D[2:], lb=lb[2:], ub=ub[2:], M=17, path="stream")]

    def run(k):
        x = shapes[k]
        return kpm.kpm_moments_batched(ctx, x["mats"], x["lb"], x["ub"], x["M"], 8, 5, path=x["path"])

    first = [run(k) for k in range(3)]
    for k in (0, 1, 0, 1, 2, 0, 2, 1, 1, 0):
        assert np.array_equal(run(k), first[k]), k
    mu = first[2]
    for i in (0, len(mats) - 3):
        ref = oracle_mu(mats[2 + i], lb[2 + i], ub[2 + i], 17, 8, 5 + i, "f32")
        assert np.max(np.abs(mu[i] - ref)) < 1e-5
