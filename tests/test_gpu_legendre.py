"""GPU parity of the Legendre expansions through the C ABI against the CPU
oracle (``oracle/dgl.py``), same probes and the same (lb, ub):

* Legendre moments (section 3.1.3) by both device routes -- Chebyshev
  moments of the fused step converted with non-negative weights (default),
  and the paper's Legendre recurrence in the fused step
  (KPM_FLAG_LEGENDRE_RECURRENCE) -- against the oracle's recurrence: FP64
  path 1e-12, FP32 path 1e-5 per normalised moment (the moments' bar);
* the DGL density (eq. (dglexpansion)) from given moments: 1e-12 relative
  plus the recurrence's own amplification of last-ulp differences (measured
  on the oracle), stopping degrees identical; divergence reported;
* KPM with Legendre polynomials (Appendix A) from given moments: 1e-12
  relative;
* end to end with a tolerance derived from the moments' bar and the
  expansion's coefficients.
"""
import math
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


TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("recurrence", [False, True])
@pytest.mark.parametrize("M,nvec,block", [(0, 3, 0), (1, 5, 0), (2, 4, 3), (7, 10, 4), (50, 12, 8)])
def test_moments_anderson3d(ctx, dtype, recurrence, M, nvec, block):
    """Several workgroups, a ragged row tail, ragged probe blocks."""
    _say(f"legendre moments {dtype} rec={recurrence} M={M} nvec={nvec} block={block}")
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(13), 16.0, 91)
    Ao = A if dtype == "f64" else A.rounded_f32()
    b = oracle.lanczos_bounds(Ao, 20, 3)
    c, d = oracle.rescale(b["lb"], b["ub"])
    mu, pv = kpm.kpm_legendre_moments(ctx, dev(A, dtype), b["lb"], b["ub"], M, nvec, 41, precision=dtype,
                                      block=block, per_vector=True, recurrence=recurrence)
    ref = oracle.legendre_moments_per_vector(Ao, c, d, M, nvec, 41) / A.n
    assert np.max(np.abs(pv - ref)) < TOL[dtype]
    assert np.max(np.abs(mu - ref.mean(axis=0))) < TOL[dtype]
    assert mu[0] == 1.0


def test_routes_agree_and_diagonal_exact(ctx):
    A = synth.random_sparse_symmetric(3001, 4.5, 23)
    b = oracle.lanczos_bounds(A, 20, 4)
    D = dev(A, "f64")
    m1 = kpm.kpm_legendre_moments(ctx, D, b["lb"], b["ub"], 81, 16, 7, precision="f64")
    m2 = kpm.kpm_legendre_moments(ctx, D, b["lb"], b["ub"], 81, 16, 7, precision="f64", recurrence=True)
    assert np.max(np.abs(m1 - m2)) < 1e-12
    assert np.array_equal(m1, kpm.kpm_legendre_moments(ctx, D, b["lb"], b["ub"], 81, 16, 7, precision="f64"))
    s = np.linspace(-0.9, 0.95, 257) ** 3
    Dg = dev(synth.diagonal_matrix(s), "f64")
    from scipy.special import eval_legendre
    ref = np.array([np.mean(eval_legendre(k, s)) for k in range(61)])
    for rec in (False, True):
        mu = kpm.kpm_legendre_moments(ctx, Dg, -1.0, 1.0, 60, 5, 3, precision="f64", recurrence=rec)
        assert np.max(np.abs(mu - ref)) < 1e-13


def test_escape_detected(ctx):
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(10), 8.0, 5)
    D = dev(A, "f64")
    for rec in (False, True):
        with pytest.raises(kpm.KpmError) as e:
            kpm.kpm_legendre_moments(ctx, D, -1.0, 1.0, 60, 4, 3, precision="f64", recurrence=rec)
        assert e.value.status == -4


def _oracle_moments(n=2000, M=400):
    A = synth.random_sparse_symmetric(n, 4.5, 31)
    b = oracle.lanczos_bounds(A, 20, 5)
    mu = oracle.legendre_moments(A, b["lb"], b["ub"], M, 6, 13)
    return A, b["lb"], b["ub"], mu


@pytest.mark.parametrize("tol,sigfrac,npts", [(1e-6, 0.02, 300), (1e-8, 0.05, 257), (1e-6, 0.3, 1)])
def test_dgl_density_on_oracle_moments(ctx, tol, sigfrac, npts):
    _say(f"dgl density tol={tol} sigma={sigfrac} npts={npts}")
    A, lb, ub, mu = _oracle_moments()
    d = 0.5 * (ub - lb)
    sigma = sigfrac * d
    x = np.linspace(lb - 0.5 * d, ub + 0.5 * d, npts)
    phi, deg = kpm.kpm_dgl_dos(ctx, mu, lb, ub, sigma, x, tol=tol)
    rphi, rdeg = oracle.dgl_dos(mu, x, sigma, tol, lb, ub)
    assert np.array_equal(deg, rdeg)
    # The gamma recurrence amplifies last-ulp differences (erf, exp of two
    # math libraries) by the growth section 3.1.3 warns of, more the longer
    # it runs (smaller tol): the bar adds ten times the oracle's own largest
    # change under 1e-15 relative changes of sigma and of the points.
    sens = np.zeros(len(x))
    for xs, ss in ((x, sigma * (1.0 + 1e-15)), (x, sigma * (1.0 - 1e-15)), (x * (1.0 + 1e-15), sigma)):
        sens = np.maximum(sens, np.abs(oracle.dgl_dos(mu, xs, ss, tol, lb, ub)[0] - rphi))
    bar = 1e-12 * np.max(np.abs(rphi)) + 10.0 * sens
    assert np.all(np.abs(phi - rphi) <= bar)


def test_dgl_caps_divergence_and_errors(ctx):
    A, lb, ub, mu = _oracle_moments(M=60)
    d = 0.5 * (ub - lb)
    x = np.linspace(lb, ub, 50)
    # sigma = 0.3 d needs ~20 terms at tol 1e-6: more than 10 moments caps the degree
    phi, deg = kpm.kpm_dgl_dos(ctx, mu[:11], lb, ub, 0.1 * d, x, tol=1e-6)
    rphi, rdeg = oracle.dgl_dos(mu[:11], x, 0.1 * d, 1e-6, lb, ub)
    assert np.max(deg) == 10 and np.array_equal(deg, rdeg)
    assert np.max(np.abs(phi - rphi)) < 1e-12 * np.max(np.abs(rphi))
    with pytest.raises(kpm.KpmError) as e:  # tol below what the recurrence reaches
        kpm.kpm_dgl_dos(ctx, mu, lb, ub, 0.3 * d, x, tol=1e-13)
    assert e.value.status == -5
    for args in ((mu, lb, ub, 0.0, x), (mu, ub, lb, 0.1, x)):
        with pytest.raises(kpm.KpmError) as e:
            kpm.kpm_dgl_dos(ctx, *args)
        assert e.value.status == -1
    with pytest.raises(kpm.KpmError):
        kpm.kpm_dgl_dos(ctx, mu, lb, ub, 0.1, x, tol=-1.0)
    assert kpm.kpm_dgl_dos(ctx, mu, lb, ub, 0.1, np.zeros(0))[0].size == 0


def test_kpml_density_on_oracle_moments(ctx):
    A, lb, ub, mu = _oracle_moments(M=120)
    x = np.linspace(lb - 0.3, ub + 0.3, 301)
    for g in (None, oracle.jackson(120)):
        phi = kpm.kpm_legendre_dos(ctx, mu, lb, ub, x, g)
        ref = oracle.legendre_dos(mu, g, x, lb, ub)
        assert np.max(np.abs(phi - ref)) < 1e-12 * np.max(np.abs(ref))
    c, d = oracle.rescale(lb, ub)
    assert kpm.kpm_legendre_dos(ctx, mu, lb, ub, np.array([c + 1.01 * d]))[0] == 0.0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dgl_end_to_end(ctx, dtype):
    """Device moments and density against oracle moments and density; the
    tolerance is the moments' bar times sum_k (k + 1/2) |gamma_k| / sqrt(2 pi s^2) / d."""
    _say(f"dgl end to end {dtype}")
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(12), 8.0, 17)
    Ao = A if dtype == "f64" else A.rounded_f32()
    lam = np.linalg.eigvalsh(Ao.dense())  # n = 1728: exact extremes, 1 % margin
    lb, ub = lam[0] - 0.01 * (lam[-1] - lam[0]), lam[-1] + 0.01 * (lam[-1] - lam[0])
    c, d = oracle.rescale(lb, ub)
    M, sigma, tol = 200, 0.03 * d, 1e-7
    mu = kpm.kpm_legendre_moments(ctx, dev(A, dtype), lb, ub, M, 16, 77, precision=dtype)
    ref_mu = oracle.legendre_moments(Ao, lb, ub, M, 16, 77)
    x = np.linspace(lb, ub, 120)
    phi, deg = kpm.kpm_dgl_dos(ctx, mu, lb, ub, sigma, x, tol=tol)
    rphi, rdeg = oracle.dgl_dos(ref_mu, x, sigma, tol, lb, ub)
    sb = sigma / d
    for i in range(len(x)):
        g, m = oracle.dgl_gamma((x[i] - c) / d, sb, tol, M)
        bound = TOL[dtype] * np.sum((np.arange(m + 1) + 0.5) * np.abs(g)) / math.sqrt(2 * math.pi) / sb / d
        assert abs(phi[i] - rphi[i]) <= bound + 1e-13, i
    assert np.max(np.abs(deg - rdeg)) == 0


def test_c2_full_size_sampled(ctx):
    """64^3 Anderson (n = 262,144), degree 256, 64 probes, FP32: both
    routes per probe against the oracle's recurrence on probes 0, 31, 63."""
    _say("legendre c2 full size")
    A = synth.config_matrix("c2")
    D = dev(A, "f32")
    lb, ub = kpm.kpm_bounds(ctx, D, 20, 3002, 0.01)
    c, d = oracle.rescale(lb, ub)
    Ao = A.rounded_f32()
    _, pv = kpm.kpm_legendre_moments(ctx, D, lb, ub, 256, 64, 2002, per_vector=True, validate=False)
    _, pr = kpm.kpm_legendre_moments(ctx, D, lb, ub, 256, 64, 2002, per_vector=True, validate=False,
                                     recurrence=True)
    for l in (0, 31, 63):
        ref = oracle.legendre_moments_per_vector(Ao, c, d, 256, 1, 2002, vec0=l)[0] / A.n
        assert np.max(np.abs(pv[l] - ref)) < 1e-5, l
        assert np.max(np.abs(pr[l] - ref)) < 1e-5, l
