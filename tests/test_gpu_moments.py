"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (stated per test): FP64 path 1e-12 absolute on every normalised
moment; FP32 path (FP32 vectors and sparse products, FP64 dots) 1e-5
absolute.  Both sides get identical lb/ub and probe seeds.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_1308_5467_amd as kpm
import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


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


def oracle_per_vec(A, lb, ub, M, nvec, seed, vec0=0, dtype="f64"):
    Ao = A if dtype == "f64" else A.rounded_f32()
    c, d = oracle.rescale(lb, ub)
    z = oracle.moments_per_vector(Ao, c, d, M, nvec, seed, vec0=vec0)
    return z / A.n


# ---------------------------------------------------------------- probe vectors
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n,nvec,ld", [(1000, 7, 9), (1001, 64, 64), (333, 5, 300)])
def test_rademacher_bit_exact(ctx, prec, n, nvec, ld):
    """Leading dimensions below, at and above the 256 columns one fill
    workgroup covers per row pass."""
    import torch
    out = torch.full((n, ld), 5.0, dtype=torch.float32 if prec == "f32" else torch.float64, device="cuda")
    kpm.kpm_rademacher(ctx, 12345, 3, nvec, n, ld, prec, out)
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.rademacher_block(12345, 3, nvec, n)
    assert np.array_equal(got[:, :nvec], ref)
    assert np.all(got[:, nvec:] == 5.0)


# ---------------------------------------------------------------- moments, small cases
def test_c1_fp64_parity(ctx):
    """c1: 2D Dirichlet Laplacian 32x32, FP64, M = 100, 20 probes."""
    _say("c1 fp64")
    A = synth.laplacian2d_dirichlet(32)
    lb, ub = oracle.lanczos_bounds(A, 20, 3001)["lb"], oracle.lanczos_bounds(A, 20, 3001)["ub"]
    D = dev(A, "f64")
    mu, pv = kpm.kpm_moments(ctx, D, lb, ub, 100, 20, 2001, precision="f64", per_vector=True)
    ref = oracle_per_vec(A, lb, ub, 100, 20, 2001)
    assert np.max(np.abs(pv - ref)) < TOL64
    assert np.max(np.abs(mu - ref.mean(axis=0))) < TOL64
    assert mu[0] == 1.0


@pytest.mark.parametrize("L,nvec,block,M", [(16, 64, 64, 256), (13, 40, 16, 31), (11, 5, 0, 2),
                                            (9, 3, 3, 1), (10, 17, 8, 0), (10, 300, 256, 20), (12, 130, 128, 9)])
def test_anderson3d_fp32_parity_ragged(ctx, L, nvec, block, M):
    """3D Anderson model, FP32 path: several workgroups, ragged row tail,
    ragged last probe block, odd/even/tiny M, the widest blocks (256 probes:
    one row per wavefront; 128)."""
    _say(f"anderson3d fp32 L={L} nvec={nvec} block={block} M={M}")
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(L), 16.0, 7 + L)
    b = oracle.lanczos_bounds(A.rounded_f32(), 20, 3)
    D = dev(A, "f32")
    mu, pv = kpm.kpm_moments(ctx, D, b["lb"], b["ub"], M, nvec, 99, precision="f32", block=block,
                             per_vector=True, rows_per_block=32)
    ref = oracle_per_vec(A, b["lb"], b["ub"], M, nvec, 99, dtype="f32")
    assert np.max(np.abs(pv - ref)) < TOL32
    assert np.max(np.abs(mu - ref.mean(axis=0))) < TOL32
    assert mu[0] == 1.0


@pytest.mark.parametrize("block", [0, 4, 6, 128])
def test_random_sparse_fp64_parity(ctx, block):
    _say(f"random sparse fp64 block={block}")
    A = synth.random_sparse_symmetric(3001, 4.5, 17)
    b = oracle.lanczos_bounds(A, 20, 4)
    D = dev(A, "f64")
    mu, pv = kpm.kpm_moments(ctx, D, b["lb"], b["ub"], 67, 10, 5, precision="f64", block=block, per_vector=True)
    ref = oracle_per_vec(A, b["lb"], b["ub"], 67, 10, 5)
    assert np.max(np.abs(pv - ref)) < TOL64


def test_widest_fp64_block_ragged(ctx):
    """FP64 path with the widest probe block (128 probes: 64 rows of 2-wide
    packs per wavefront pass) and a ragged second block of 22, per probe."""
    _say("random sparse fp64 block=128 nvec=150")
    A = synth.random_sparse_symmetric(1001, 4.5, 23)
    b = oracle.lanczos_bounds(A, 20, 4)
    mu, pv = kpm.kpm_moments(ctx, dev(A, "f64"), b["lb"], b["ub"], 21, 150, 6, precision="f64", block=128,
                             per_vector=True)
    ref = oracle_per_vec(A, b["lb"], b["ub"], 21, 150, 6)
    assert np.max(np.abs(pv - ref)) < TOL64
    assert np.max(np.abs(mu - ref.mean(axis=0))) < TOL64


def test_high_degree_fp64(ctx):
    """Degree 2,048 (1,024 steps with the product identity) against the
    oracle's plain three-term recurrence, per probe: the doubling's rounding
    stays at the FP64 bar far out."""
    _say("fp64 M=2048")
    A = synth.add_diagonal_disorder(synth.laplacian2d_dirichlet(24), 4.0, 31)
    lam = np.linalg.eigvalsh(A.dense())  # exact extremes: a 20-step bound can miss an edge state here
    w = lam[-1] - lam[0]
    lb, ub = lam[0] - 0.01 * w, lam[-1] + 0.01 * w
    mu, pv = kpm.kpm_moments(ctx, dev(A, "f64"), lb, ub, 2048, 3, 8, precision="f64", per_vector=True)
    ref = oracle_per_vec(A, lb, ub, 2048, 3, 8)
    assert np.max(np.abs(pv - ref)) < TOL64


def test_fp64_values_fp32_path_rounds_values(ctx):
    """FP64 values on the FP32 path are rounded to FP32 first."""
    A = synth.random_sparse_symmetric(1500, 3.0, 3)
    b = oracle.lanczos_bounds(A, 20, 4)
    D = dev(A, "f64")
    mu = kpm.kpm_moments(ctx, D, b["lb"], b["ub"], 40, 8, 5, precision="f32")
    ref = oracle_per_vec(A, b["lb"], b["ub"], 40, 8, 5, dtype="f32").mean(axis=0)
    assert np.max(np.abs(mu - ref)) < TOL32


def test_host_csr_input(ctx):
    A = synth.laplacian2d_dirichlet(20)
    H = kpm.HostCSR(A.n, A.row_ptr, A.col_idx, A.val)
    mu = kpm.kpm_moments(ctx, H, -0.1, 8.1, 30, 4, 9, precision="f64")
    ref = oracle_per_vec(A, -0.1, 8.1, 30, 4, 9).mean(axis=0)
    assert np.max(np.abs(mu - ref)) < TOL64


def test_diagonal_and_one_by_one(ctx):
    d = np.random.default_rng(1).uniform(-2, 3, 333)
    A = synth.diagonal_matrix(d)
    mu = kpm.kpm_moments(ctx, dev(A, "f64"), -2.5, 3.5, 50, 3, 8, precision="f64")
    c, dd = oracle.rescale(-2.5, 3.5)
    exact = np.array([np.mean(np.cos(k * np.arccos((d - c) / dd))) for k in range(51)])
    assert np.max(np.abs(mu - exact)) < TOL64
    one = synth.diagonal_matrix(np.array([0.0]))
    mu1 = kpm.kpm_moments(ctx, dev(one, "f64"), -1.0, 1.0, 40, 1, 0, precision="f64")
    assert np.max(np.abs(mu1 - np.array([[1.0, 0.0, -1.0, 0.0][k % 4] for k in range(41)]))) < 1e-15


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", TOL64)])
def test_empty_rows_and_zero_matrix(ctx, prec, tol):
    """Rows without stored entries.  The zero matrix (nnz = 0) on [-1, 1]:
    B = 0, so mu_k = T_k(0) = cos(k pi / 2) exactly; its bounds fall back on
    the Gershgorin hull (Lanczos breaks down at once) and enclose 0.  A
    diagonal matrix with every other row empty against the oracle, and both
    in one batch."""
    n = 500
    Z = synth.CSR(n, np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32), np.zeros(0))
    exact = np.array([[1.0, 0.0, -1.0, 0.0][k % 4] for k in range(21)])
    mu = kpm.kpm_moments(ctx, dev(Z, prec), -1.0, 1.0, 20, 8, 5, precision=prec)
    assert np.array_equal(mu, exact)
    lb, ub = kpm.kpm_bounds(ctx, dev(Z, prec), 20, 1, 0.01)
    assert np.isfinite(lb) and np.isfinite(ub) and lb < 0.0 < ub
    d = np.random.default_rng(4).uniform(-2.0, 3.0, n)
    keep = np.arange(n) % 2 == 0
    rp = np.concatenate([[0], np.cumsum(keep)]).astype(np.int32)
    H = synth.CSR(n, rp, np.nonzero(keep)[0].astype(np.int32), d[keep])
    Ho = H if prec == "f64" else H.rounded_f32()
    ref = oracle.moments(Ho, -2.5, 3.5, 30, 6, 11)
    mu_h = kpm.kpm_moments(ctx, dev(H, prec), -2.5, 3.5, 30, 6, 11, precision=prec)
    assert np.max(np.abs(mu_h - ref)) < tol
    mub = kpm.kpm_moments_batched(ctx, [dev(Z, prec), dev(H, prec)], [-1.0, -2.5], [1.0, 3.5], 30, 6, 11,
                                  precision=prec)
    assert np.max(np.abs(mub[0] - np.array([[1.0, 0.0, -1.0, 0.0][k % 4] for k in range(31)]))) < 1e-15
    assert np.max(np.abs(mub[1] - oracle.moments(Ho, -2.5, 3.5, 30, 6, 12))) < tol


def test_deterministic_bitwise(ctx):
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(20), 8.0, 2)
    D = dev(A, "f32")
    lb, ub = kpm.kpm_bounds(ctx, D, 20, 1, 0.01)
    r1 = kpm.kpm_moments(ctx, D, lb, ub, 64, 64, 3)
    r2 = kpm.kpm_moments(ctx, D, lb, ub, 64, 64, 3)
    assert np.array_equal(r1, r2)


# ---------------------------------------------------------------- errors
def test_narrow_bounds_report_spectrum_escape(ctx):
    A = synth.laplacian2d_dirichlet(16)
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_moments(ctx, dev(A, "f64"), 1.0, 5.0, 120, 4, 1, precision="f64")
    assert e.value.status == -4


def test_malformed_csr_is_rejected(ctx):
    A = synth.laplacian2d_dirichlet(8)
    ci = A.col_idx.copy()
    ci[5] = A.n + 3          # out of range
    H = kpm.HostCSR(A.n, A.row_ptr, ci, A.val)
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_moments(ctx, H, -0.1, 8.1, 10, 2, 1, precision="f64", validate=True)
    assert e.value.status == -1
    ci = A.col_idx.copy()
    ci[0], ci[1] = ci[1], ci[0]  # unsorted
    with pytest.raises(kpm.KpmError):
        kpm.kpm_moments(ctx, kpm.HostCSR(A.n, A.row_ptr, ci, A.val), -0.1, 8.1, 10, 2, 1,
                        precision="f64", validate=True)
    v = A.val.copy()
    v[3] = np.nan
    with pytest.raises(kpm.KpmError):
        kpm.kpm_moments(ctx, kpm.HostCSR(A.n, A.row_ptr, A.col_idx, v), -0.1, 8.1, 10, 2, 1,
                        precision="f64", validate=True)


def test_bad_arguments(ctx):
    A = synth.laplacian2d_dirichlet(8)
    D = dev(A, "f64")
    for kw in (dict(M=-1), dict(nvec=0), dict(block=300)):
        args = dict(M=10, nvec=2, block=0)
        args.update(kw)
        with pytest.raises(kpm.KpmError) as e:
            kpm.kpm_moments(ctx, D, -0.1, 8.1, args["M"], args["nvec"], 1, precision="f64", block=args["block"])
        assert e.value.status == -1
    with pytest.raises(kpm.KpmError):
        kpm.kpm_moments(ctx, D, 2.0, 1.0, 10, 2, 1)


# ---------------------------------------------------------------- bounds
@pytest.mark.parametrize("which", ["lap2d", "anderson3d", "random", "diag_breakdown", "tiny"])
def test_bounds_parity_and_enclosure(ctx, which):
    _say(f"bounds {which}")
    if which == "lap2d":
        A = synth.laplacian2d_dirichlet(32)
    elif which == "anderson3d":
        A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(12), 16.0, 5)
    elif which == "random":
        A = synth.random_sparse_symmetric(2000, 4.5, 8)
    elif which == "diag_breakdown":
        A = synth.diagonal_matrix(np.array([1.0, 1.0, 1.0, 2.0, 2.0]))
    else:
        A = synth.random_sparse_symmetric(7, 2.0, 3)
    for prec in ("f64", "f32"):
        Ao = A if prec == "f64" else A.rounded_f32()
        ref = oracle.lanczos_bounds(Ao, 20, 3001)
        lb, ub = kpm.kpm_bounds(ctx, dev(A, prec), 20, 3001, 0.01)
        scale = max(abs(ref["lb"]), abs(ref["ub"]), 1.0)
        assert abs(lb - ref["lb"]) < 1e-9 * scale and abs(ub - ref["ub"]) < 1e-9 * scale
        if A.n <= 4096:
            lam = np.linalg.eigvalsh(Ao.dense())
            assert lb < lam[0] and ub > lam[-1]


# ---------------------------------------------------------------- damping and density
def test_jackson_and_dos_parity(ctx):
    for M in (1, 2, 3, 40, 100, 1000):
        g = kpm.kpm_damping_factors(ctx, kpm.KPM_DAMP_JACKSON, M)
        assert np.max(np.abs(g - oracle.jackson(M))) < 1e-14
    g1 = kpm.kpm_damping_factors(ctx, kpm.KPM_DAMP_NONE, 5)
    assert np.all(g1 == 1.0)
    rng = np.random.default_rng(2)
    M = 100
    mu = np.concatenate([[1.0], rng.normal(0, 0.3, M) / np.arange(1, M + 1)])
    g = oracle.jackson(M)
    x = np.linspace(-3.5, 9.5, 401)
    phi = kpm.kpm_dos(ctx, mu, g, -2.0, 8.0, x)
    ref = oracle.dos(mu, g, -2.0, 8.0, x)
    assert np.max(np.abs(phi - ref)) < 1e-11
    edges = np.linspace(-3, 9, 61)
    mass = kpm.kpm_dos_bins(ctx, mu, g, -2.0, 8.0, edges)
    assert np.max(np.abs(mass - oracle.dos_bins(mu, g, -2.0, 8.0, edges))) < 1e-12
    assert abs(mass.sum() - 1.0) < 1e-12


def test_delta_function_example(ctx):
    """The paper's degree-40 delta-function expansion: 41/pi at 0 undamped."""
    M = 40
    mu = kpm.kpm_moments(ctx, dev(synth.diagonal_matrix(np.array([0.0])), "f64"), -1.0, 1.0, M, 1, 0,
                         precision="f64")
    phi = kpm.kpm_dos(ctx, mu, np.ones(M + 1), -1.0, 1.0, np.array([0.0]))
    assert abs(phi[0] - 41 / math.pi) < 1e-12
    t = np.linspace(-0.999, 0.999, 4001)
    assert kpm.kpm_dos(ctx, mu, np.ones(M + 1), -1.0, 1.0, t).min() < -1.0
    gj = kpm.kpm_damping_factors(ctx, kpm.KPM_DAMP_JACKSON, M)
    assert kpm.kpm_dos(ctx, mu, gj, -1.0, 1.0, t).min() > -1e-12


# ---------------------------------------------------------------- full-size workloads, sampled
@pytest.mark.parametrize("locality", [False, True])
def test_c2_full_size_sampled(ctx, locality):
    """c2 at full size (64^3 Anderson, M = 256, 64 probes, FP32), in the
    launch configuration the benchmark times (with and without the locality
    renumbering, which the benchmark uses); the oracle recomputes probes 0,
    31 and 63 one by one on the original matrix."""
    _say(f"c2 full size, locality={locality}")
    A = synth.config_matrix("c2")
    D = dev(A, "f32")
    lb, ub = kpm.kpm_bounds(ctx, D, 20, 3002, 0.01)
    # 7-point periodic Laplacian spectrum [0, 12] shifted by disorder in [-8, 8]
    assert -8.0 - 1.0 < lb < 0.0 and 12.0 < ub < 20.0 + 1.0
    mu, pv = kpm.kpm_moments(ctx, D, lb, ub, 256, 64, 2002, precision="f32", validate=False, per_vector=True,
                             locality=locality)
    Ao = A.rounded_f32()
    c, d = oracle.rescale(lb, ub)
    for l in (0, 31, 63):
        z = oracle.moments_per_vector(Ao, c, d, 256, 1, 2002, vec0=l)[0] / A.n
        assert np.max(np.abs(pv[l] - z)) < TOL32, l
    assert mu[0] == 1.0 and np.all(np.abs(pv) <= 1 + 1e-5)


GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _c5_golden():
    """Bounds and the oracle's moments of probes 254, 255 at degree 1000,
    written by tests/golden/make_c5_probe_moments.py (oracle only)."""
    rows = [ln.split() for ln in open(f"{GOLDEN}/c5_probe_moments.txt") if ln.strip() and not ln.startswith("#")]
    assert rows[0][0] == "lb" and rows[1][0] == "ub"
    z = np.array([[float(r[1]), float(r[2])] for r in rows[2:]]).T
    assert z.shape == (2, 1001)
    return float(rows[0][1]), float(rows[1][1]), z


def test_c5_full_size_sampled(ctx):
    """c5 at full size: 3D Anderson 128^3 plus random long-range hoppings
    (n = 2,097,152, nnz ~ 23M), degree 1000, 256 probes, FP32: in blocks of
    64 in the caller's numbering, and in the configuration the benchmark
    times, blocks of 32 with the locality renumbering.  Probes 254 and 255
    (the last block) against the oracle at every degree up to 1000, 1e-5; the
    oracle's bounds are used on both sides and the library's own bounds must
    agree with them (1e-9 relative); invariants on every probe; the first
    201 moments equal a degree-200 run bitwise (the same launches)."""
    lb, ub, z = _c5_golden()
    _say("c5 full size: generating matrix")
    A = synth.config_matrix("c5")
    assert A.n == 128**3 and 20_000_000 < A.nnz < 26_000_000
    D = dev(A, "f32")
    _say("c5 bounds")
    glb, gub = kpm.kpm_bounds(ctx, D, 20, 3005, 0.01)
    assert abs(glb - lb) <= 1e-9 * (ub - lb) and abs(gub - ub) <= 1e-9 * (ub - lb), (glb, gub, lb, ub)
    _say("c5 moments M=1000")
    mu, pv = kpm.kpm_moments(ctx, D, lb, ub, 1000, 256, 2005, precision="f32", block=64,
                             validate=True, per_vector=True)
    assert mu[0] == 1.0 and np.all(np.abs(pv) <= 1 + 1e-5)
    err = np.abs(pv[254:256] - z)
    _say(f"c5 probes 254, 255: max |dmu| {err.max():.2e} (degrees 0-200 {err[:, :201].max():.2e}, "
         f"201-1000 {err[:, 201:].max():.2e})")
    assert err.max() < TOL32
    _say("c5 moments M=200")
    mu2, pv2 = kpm.kpm_moments(ctx, D, lb, ub, 200, 256, 2005, precision="f32", block=64,
                               validate=False, per_vector=True)
    assert np.array_equal(pv[:, :201], pv2)
    # the configuration the benchmark times: blocks of 32, the library's
    # locality renumbering
    _say("c5 moments M=1000, blocks of 32, with the locality renumbering")
    mu3, pv3 = kpm.kpm_moments(ctx, D, lb, ub, 1000, 256, 2005, precision="f32", block=32,
                               validate=False, per_vector=True, locality=True)
    assert mu3[0] == 1.0 and np.all(np.abs(pv3) <= 1 + 1e-5)
    err3 = np.abs(pv3[254:256] - z)
    _say(f"c5 locality, probes 254, 255: max |dmu| {err3.max():.2e}; mean moments vs plain "
         f"{np.abs(mu3 - mu).max():.2e}")
    assert err3.max() < TOL32
    assert np.abs(mu3 - mu).max() < TOL32


def test_anderson32_longrange_fp32_degree1000_all_probes(ctx):
    """The large workload's family at 32^3 (3D Anderson + 2 long-range pairs
    per row, n = 32,768), degree 1000, 70 probes (one block of 64 and a
    ragged block of 6), FP32: every probe, every degree against the oracle
    at 1e-5."""
    A = synth.config_matrix("c5", scale=32)
    D = dev(A, "f32")
    lb, ub = kpm.kpm_bounds(ctx, D, 20, 3105, 0.01)
    _say("32^3 + long range, degree 1000, 70 probes")
    mu, pv = kpm.kpm_moments(ctx, D, lb, ub, 1000, 70, 2105, precision="f32", block=64,
                             validate=True, per_vector=True)
    Ao = A.rounded_f32()
    c, d = oracle.rescale(lb, ub)
    z = oracle.moments_per_vector(Ao, c, d, 1000, 70, 2105, nthreads=16) / A.n
    err = np.abs(pv - z)
    _say(f"max |dmu| {err.max():.2e}; mean moments {np.abs(mu - z.mean(axis=0)).max():.2e}")
    assert err.max() < TOL32
    assert np.abs(mu - z.mean(axis=0)).max() < TOL32


def test_context_created_before_torch_is_imported():
    """A script that creates a context before importing torch: the binding
    loads torch's HIP runtime first, so the library binds to the one runtime
    in the process (two runtimes made kpm_create fail).  Run in a child
    process, which imports nothing else first."""
    import subprocess
    code = ("import numpy as np, paper_1308_5467_amd as kpm, synth\n"
            "c = kpm.Context(0)\n"
            "A = synth.diagonal_matrix(np.linspace(-1, 1, 100))\n"
            "D = kpm.DeviceCSR.from_host(A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32), 'f32')\n"
            "mu = kpm.kpm_moments(c, D, -1.5, 1.5, 4, 2, 1)\n"
            "print('ok', mu[0])\n")
    root = __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and "ok 1.0" in r.stdout, (r.stdout, r.stderr)


# ---------------------------------------------------------------- locality renumbering
@pytest.mark.parametrize("prec,tol", [("f32", TOL32), ("f64", TOL64)])
def test_locality_renumbering_parity(ctx, prec, tol):
    """KPM_FLAG_LOCALITY: the matrix renumbered inside the library along its
    grid's Morton curve, probes at the original indices -- per-probe moments
    against the oracle on the original matrix (3D Anderson 24^3 + long-range
    pairs, 2D periodic 40 x 24), and against the plain path.  A second call
    reuses the cached structure with new values."""
    import torch
    mats = [synth.config_matrix("c5", scale=24), synth.add_diagonal_disorder(synth.laplacian2d_periodic(40, 24), 4.0, 9)]
    for A in mats:
        D = dev(A, prec)
        lb, ub = kpm.kpm_bounds(ctx, D, 20, 31, 0.01)
        mu, pv = kpm.kpm_moments(ctx, D, lb, ub, 61, 21, 77, precision=prec, per_vector=True, locality=True)
        ref = oracle_per_vec(A, lb, ub, 61, 21, 77, dtype=prec)
        assert np.max(np.abs(pv - ref)) < tol
        mu0 = kpm.kpm_moments(ctx, D, lb, ub, 61, 21, 77, precision=prec)
        assert np.max(np.abs(mu - mu0)) < tol
    # new values at the same address: the renumbered copy re-reads them
    A = mats[1]
    D = dev(A, prec)
    lb, ub = kpm.kpm_bounds(ctx, D, 20, 31, 0.01)
    kpm.kpm_moments(ctx, D, lb, ub, 10, 4, 5, precision=prec, locality=True)
    B = synth.CSR(A.n, A.row_ptr, A.col_idx, A.val * 0.5)
    D.val.copy_(torch.as_tensor(B.val.astype(np.float32 if prec == "f32" else np.float64), device="cuda"))
    _, pv = kpm.kpm_moments(ctx, D, lb, ub, 30, 4, 5, precision=prec, per_vector=True, locality=True)
    assert np.max(np.abs(pv - oracle_per_vec(B, lb, ub, 30, 4, 5, dtype=prec))) < tol


def test_locality_without_grid_and_other_entry_points(ctx):
    """No grid: the flag changes nothing (bitwise).  Host matrices of equal
    sizes but different structure in a row: each renumbered from its own
    structure.  Legendre moments by conversion take the flag; the Legendre
    recurrence refuses it.  The whole-path pipeline with the flag equals the
    pipeline without it to the moments' bar."""
    R = synth.random_sparse_symmetric(700, 4.5, 4)
    D = dev(R, "f32")
    lb, ub = kpm.kpm_bounds(ctx, D, 20, 3, 0.01)
    a = kpm.kpm_moments(ctx, D, lb, ub, 40, 9, 2, locality=True)
    b = kpm.kpm_moments(ctx, D, lb, ub, 40, 9, 2)
    assert np.array_equal(a, b)
    for L in ((30, 20), (20, 30)):  # same n and nnz, different grids
        A = synth.add_diagonal_disorder(synth.laplacian2d_periodic(*L), 2.0, 6)
        H = kpm.HostCSR(A.n, A.row_ptr, A.col_idx, A.val)
        lb, ub = kpm.kpm_bounds(ctx, H, 20, 3, 0.01)
        _, pv = kpm.kpm_moments(ctx, H, lb, ub, 25, 6, 8, precision="f64", per_vector=True, locality=True)
        assert np.max(np.abs(pv - oracle_per_vec(A, lb, ub, 25, 6, 8))) < TOL64, L
    A = synth.config_matrix("c5", scale=16)
    D = dev(A, "f32")
    lb, ub = kpm.kpm_bounds(ctx, D, 20, 3, 0.01)
    l1 = kpm.kpm_legendre_moments(ctx, D, lb, ub, 33, 8, 4, locality=True)
    l0 = kpm.kpm_legendre_moments(ctx, D, lb, ub, 33, 8, 4)
    assert np.max(np.abs(l1 - l0)) < TOL32
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_legendre_moments(ctx, D, lb, ub, 33, 8, 4, recurrence=True, locality=True)
    assert e.value.status == -6
    x = np.linspace(lb, ub, 50)
    p1, m1, _, _ = kpm.kpm_dos_pipeline(ctx, D, 64, 16, 5, x, locality=True, lanczos_seed=3)
    p0, m0, _, _ = kpm.kpm_dos_pipeline(ctx, D, 64, 16, 5, x, lanczos_seed=3)
    assert np.max(np.abs(m1 - m0)) < TOL32
    assert np.max(np.abs(p1 - p0)) < 1e-3 * np.max(np.abs(p0))


def test_locality_detects_changed_structure(ctx):
    """The renumbered copy is cached per matrix address.  A device matrix
    rewritten in place with another structure of the same sizes (a 30 x 20
    periodic grid replaced by a 20 x 30 one) is detected when the results are
    collected (KPM_ERR_ARG); the next call rebuilds the copy and matches the
    oracle on the new matrix."""
    import torch
    A = synth.add_diagonal_disorder(synth.laplacian2d_periodic(30, 20), 2.0, 6)
    B = synth.add_diagonal_disorder(synth.laplacian2d_periodic(20, 30), 2.0, 7)
    assert A.n == B.n and A.nnz == B.nnz and not np.array_equal(A.col_idx, B.col_idx)
    D = dev(A, "f64")
    lb, ub = -1.5, 10.5
    kpm.kpm_moments(ctx, D, lb, ub, 20, 4, 3, precision="f64", locality=True)
    D.row_ptr.copy_(torch.as_tensor(B.row_ptr, device="cuda"))
    D.col_idx.copy_(torch.as_tensor(B.col_idx, device="cuda"))
    D.val.copy_(torch.as_tensor(B.val, device="cuda"))
    with pytest.raises(kpm.KpmError) as e:
        kpm.kpm_moments(ctx, D, lb, ub, 20, 4, 3, precision="f64", locality=True)
    assert e.value.status == -1 and "structure" in e.value.message
    _, pv = kpm.kpm_moments(ctx, D, lb, ub, 20, 4, 3, precision="f64", per_vector=True, locality=True)
    assert np.max(np.abs(pv - oracle_per_vec(B, lb, ub, 20, 4, 3))) < TOL64


def test_locality_value_types_sharing_one_structure(ctx):
    """Two device matrices sharing the same row-offset and column arrays,
    one with FP32 and one with FP64 values: the renumbered copy is keyed on
    the values' type too (its value buffer is sized for it), so each call
    matches the oracle -- FP32 path on FP32 values, FP64 path and FP32 path
    on FP64 values, then FP32 again."""
    import torch
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(12), 8.0, 21)
    D32 = dev(A, "f32")
    D64 = kpm.DeviceCSR(D32.n, D32.row_ptr, D32.col_idx, D32.val.to(torch.float64))
    lb, ub = kpm.kpm_bounds(ctx, D32, 20, 5, 0.01)
    ref = oracle_per_vec(A, lb, ub, 40, 6, 9, dtype="f32")  # values rounded to FP32 on both
    for D, prec, tol in ((D32, "f32", TOL32), (D64, "f64", TOL64), (D64, "f32", TOL32), (D32, "f32", TOL32)):
        _, pv = kpm.kpm_moments(ctx, D, lb, ub, 40, 6, 9, precision=prec, per_vector=True, locality=True)
        assert np.max(np.abs(pv - ref)) < tol, prec


def test_locality_refuses_malformed_structure_on_the_host(ctx):
    """With the renumbering the whole structure is read on the host: a column
    index past n or decreasing row offsets are refused there (KPM_ERR_ARG)
    even without validation, before any kernel reads the matrix; a valid
    matrix afterwards runs normally."""
    A = synth.add_diagonal_disorder(synth.laplacian2d_periodic(16, 12), 2.0, 3)
    bad_ci = A.col_idx.copy()
    bad_ci[37] = A.n
    bad_rp = A.row_ptr.copy()
    bad_rp[50] = bad_rp[52]
    for rp, ci in ((A.row_ptr, bad_ci), (bad_rp, A.col_idx)):
        D = kpm.DeviceCSR.from_host(A.n, rp, ci, A.val.astype(np.float32), "f32")
        with pytest.raises(kpm.KpmError) as e:
            kpm.kpm_moments(ctx, D, -1.0, 9.0, 10, 4, 1, validate=False, locality=True)
        assert e.value.status == -1 and "malformed" in e.value.message
    D = dev(A, "f32")
    _, pv = kpm.kpm_moments(ctx, D, -1.5, 9.5, 10, 4, 1, per_vector=True, locality=True)
    assert np.max(np.abs(pv - oracle_per_vec(A, -1.5, 9.5, 10, 4, 1, dtype="f32"))) < TOL32


def test_probe_blocks_beyond_4_gib(ctx):
    """Probe blocks of 4 GiB and more take the step kernel's 64-bit offsets:
    3D Anderson 168^3 (n = 4,741,632, nnz = 33.2M) with one block of 256
    FP32 probes (4.86 GB) and one of 128 FP64 probes (4.86 GB), degree 12;
    probes 0, 1, 254 / 126, 127 against the oracle per probe at every degree
    (1e-5 / 1e-12), every probe within |mu| <= 1, and the same probes in
    blocks of 64 (32-bit offsets) agreeing with the wide block.  The batched
    path refuses blocks of 4 GiB (its offsets are 32-bit)."""
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(168), 16.0, 1168)
    assert A.n * 256 * 4 >= 1 << 32
    lb, ub = -8.2, 20.2  # encloses [0 - 8, 12 + 8] (Gershgorin)
    Ao = A.rounded_f32()
    c, d = oracle.rescale(lb, ub)
    for prec, nvec, tol, probes in (("f32", 256, TOL32, (0, 1, 254)), ("f64", 128, TOL64, (126, 127))):
        D = dev(A, prec)
        _say(f"168^3, one block of {nvec} {prec} probes")
        mu, pv = kpm.kpm_moments(ctx, D, lb, ub, 12, nvec, 77, precision=prec, block=nvec, validate=False,
                                 per_vector=True)
        assert np.all(np.abs(pv) <= 1 + 1e-5) and mu[0] == 1.0
        for l in probes:
            z = oracle.moments_per_vector(Ao if prec == "f32" else A, c, d, 12, 1, 77, vec0=l, nthreads=2)[0] / A.n
            assert np.max(np.abs(pv[l] - z)) < tol, (prec, l)
        _, pv64 = kpm.kpm_moments(ctx, D, lb, ub, 12, nvec, 77, precision=prec, block=64 if prec == "f32" else 32,
                                  validate=False, per_vector=True)
        assert np.max(np.abs(pv64 - pv)) < tol
        if prec == "f32":
            with pytest.raises(kpm.KpmError) as e:
                kpm.kpm_moments_batched(ctx, [D], [lb], [ub], 12, 256, 77, block=256)
            assert e.value.status == -6
        del D


def _arrow(n, seed):
    """Random sparse symmetric (about 10 entries per row) plus a dense row
    and column 0 (an arrow): one row of n entries, every other row one more."""
    import scipy.sparse as sp
    R = synth.random_sparse_symmetric(n, 4.5, seed).to_scipy().tolil()
    rng = np.random.default_rng(seed)
    v = rng.normal(0.0, 0.3, n - 1)
    R[0, 1:] = v
    R[1:, 0] = v[:, None]
    return synth._from_scipy(sp.csr_matrix(R))


@pytest.mark.parametrize("prec,tol", [("f32", TOL32), ("f64", TOL64)])
def test_long_rows_take_the_unstaged_path(ctx, prec, tol):
    """Row panels whose CSR slice does not fit the step's LDS staging read
    the CSR directly: an arrow matrix (n = 3,000, one row of 3,000 entries,
    the others about 11: staged panels beside one unstaged panel) and a
    random symmetric matrix with about 200 entries in every row (every
    panel unstaged); per-probe moments against the oracle, degree 60."""
    mats = [_arrow(3000, 41), synth.random_sparse_symmetric(3000, 100.0, 42, off_scale=0.1)]
    assert mats[0].row_ptr[1] - mats[0].row_ptr[0] == 3000
    assert np.min(np.diff(mats[1].row_ptr)) > 120
    for A in mats:
        D = dev(A, prec)
        lb, ub = kpm.kpm_bounds(ctx, D, 20, 3, 0.01)
        lam = np.linalg.eigvalsh(A.dense())
        if not (lb <= lam[0] and lam[-1] <= ub):  # a 20-step run can miss an outlying edge
            lb, ub = lam[0] - 0.05 * (lam[-1] - lam[0]), lam[-1] + 0.05 * (lam[-1] - lam[0])
        _, pv = kpm.kpm_moments(ctx, D, lb, ub, 60, 10, 9, precision=prec, per_vector=True)
        assert np.max(np.abs(pv - oracle_per_vec(A, lb, ub, 60, 10, 9, dtype=prec))) < tol
