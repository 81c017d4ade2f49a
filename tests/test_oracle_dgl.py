"""Pins of the oracle's Legendre expansions (KPM with Legendre polynomials,
Appendix A; the Delta-Gauss-Legendre method, section 3.1.3 and Appendix B)
against facts the mathematics fixes, independently of its recurrences:

* diagonal matrices: the +/-1 estimator is exact, mu_k = mean_i L_k(s_i)
  (scipy's Legendre evaluation);
* per-probe moments v^T L_k(B) v against dense eigendecomposition;
* the 1 x 1 zero matrix: mu_k = L_k(0) in closed form;
* gamma_k(t) of eq. (DGLcoeff) against adaptive quadrature of its integral;
* the truncated expansion of eq. (dglexpansion) reproduces the Gaussian on
  [-1, 1], better for a smaller stopping tolerance, and needs more terms
  for narrower Gaussians; a tolerance the unstable recurrence cannot reach
  is reported (|gamma_k| <= gamma_0 holds exactly);
* DGL of exact moments equals the Gaussian-regularised density
  (1/n) sum_j g_sigma(x - lambda_j) of eq. (blurphi) (with the 1/n);
* KPM-Legendre of the 1 x 1 zero matrix equals the Christoffel-Darboux
  closed form, and every KPM-Legendre density has unit mass on [-1, 1].
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import eval_legendre

import oracle
import synth


def test_diagonal_estimator_is_exact():
    s = np.linspace(-0.95, 0.9, 37) ** 3
    A = synth.diagonal_matrix(s)
    mu = oracle.legendre_moments(A, -1.0, 1.0, 40, 3, 7)
    ref = np.array([np.mean(eval_legendre(k, s)) for k in range(41)])
    assert np.max(np.abs(mu - ref)) < 1e-13


def test_per_probe_moments_against_eigh():
    A = synth.random_sparse_symmetric(300, 4.5, 5)
    lam, U = np.linalg.eigh(A.dense())
    lb, ub = lam[0] - 0.1, lam[-1] + 0.2
    c, d = oracle.rescale(lb, ub)
    z = oracle.legendre_moments_per_vector(A, c, d, 30, 3, 11)
    V = oracle.rademacher_block(11, 0, 3, A.n)
    W = (U.T @ V) ** 2
    s = (lam - c) / d
    ref = np.stack([[np.sum(W[:, l] * eval_legendre(k, s)) for k in range(31)] for l in range(3)])
    assert np.max(np.abs(z - ref)) < 1e-12 * A.n


def test_one_by_one_zero_matrix():
    A = synth.diagonal_matrix(np.array([0.0]))
    mu = oracle.legendre_moments(A, -1.0, 1.0, 12, 2, 0)
    # L_k(0) = 0 for odd k, (-1)^(k/2) (k-1)!!/k!! for even k
    ref = np.zeros(13)
    for k in range(0, 13, 2):
        ref[k] = (-1) ** (k // 2) * math.prod(range(k - 1, 0, -2)) / math.prod(range(k, 0, -2))
    assert np.max(np.abs(mu - ref)) < 1e-15


def _gamma_ref(k, t, sigma):
    return quad(lambda s: eval_legendre(k, s) * math.exp(-0.5 * ((s - t) / sigma) ** 2), -1.0, 1.0,
                points=[t] if abs(t) < 1 else None, limit=400, epsabs=1e-15, epsrel=1e-12)[0]


@pytest.mark.parametrize("sigma,t", [(0.02, 0.3), (0.1, -0.7), (0.3, 0.0), (0.05, 0.97), (0.02, 1.2)])
def test_gamma_against_quadrature(sigma, t):
    """Every coefficient up to the degree the paper's rule stops at (tol 1e-6)."""
    g, m = oracle.dgl_gamma(t, sigma, 1e-6, 5000)
    assert 0 < m < 5000 and g.size == m + 1
    for k in range(m + 1):
        assert abs(g[k] - _gamma_ref(k, t, sigma)) < 1e-10, k


def test_stopping_rule_truncation():
    """The stopped expansion (k + 1/2) gamma_k L_k reproduces the Gaussian on
    [-1, 1]; a smaller tol buys accuracy; narrower Gaussians need more terms."""
    s = np.linspace(-1.0, 1.0, 801)
    deg = {}
    for sigma in (0.3, 0.1, 0.05, 0.02):
        for t in (-0.6, 0.0, 0.45, 0.97):
            exact = np.exp(-0.5 * ((s - t) / sigma) ** 2)
            err = {}
            for tol in (1e-6, 1e-8):
                g, m = oracle.dgl_gamma(t, sigma, tol, 5000)
                assert m < 5000
                err[tol] = np.max(np.abs(np.polynomial.legendre.legval(s, (np.arange(m + 1) + 0.5) * g) - exact))
                deg[(sigma, t, tol)] = m
            assert err[1e-8] < 2e-4 and err[1e-8] < 0.2 * err[1e-6], (sigma, t, err)
    for t in (-0.6, 0.0, 0.45, 0.97):
        ms = [deg[(sigma, t, 1e-8)] for sigma in (0.3, 0.1, 0.05, 0.02)]
        assert ms == sorted(ms) and ms[0] < ms[-1]


def test_divergence_is_reported():
    """A tol below what the unstable recurrence can reach (section 3.1.3's
    warning) ends in an error, not in amplified noise."""
    with pytest.raises(FloatingPointError):
        oracle.dgl_gamma(0.45, 0.3, 1e-12, 5000)


def test_dgl_of_exact_moments_is_the_blurred_density():
    lam = np.sort(np.random.default_rng(4).uniform(-3.0, 5.0, 60))
    A = synth.diagonal_matrix(lam)
    lb, ub = -3.5, 5.5
    mu = oracle.legendre_moments(A, lb, ub, 1500, 1, 3)
    x = np.linspace(-4.0, 6.0, 57)
    sigma = 0.15
    phi, deg = oracle.dgl_dos(mu, x, sigma, 1e-8, lb, ub)
    ref = np.array([np.mean(oracle.gauss(xi - lam, sigma)) for xi in x])
    assert np.all(deg < 1500)
    assert np.max(np.abs(phi - ref)) < 5e-4 * np.max(ref)


def test_kpml_christoffel_darboux_and_mass():
    M = 30
    mu = np.array([eval_legendre(k, 0.0) for k in range(M + 1)])
    t = np.array([-0.9, -0.31, 0.2, 0.77])
    phi = oracle.legendre_dos(mu, None, t, -1.0, 1.0)
    ref = (M + 1) / 2 * (eval_legendre(M + 1, 0.0) * eval_legendre(M, t)
                         - eval_legendre(M, 0.0) * eval_legendre(M + 1, t)) / (0.0 - t)
    assert np.max(np.abs(phi - ref)) < 1e-12
    # unit mass (Gauss-Legendre quadrature is exact for the degree-M polynomial), in A's units
    A = synth.random_sparse_symmetric(200, 4.5, 2)
    b = oracle.lanczos_bounds(A, 20, 1)
    muA = oracle.legendre_moments(A, b["lb"], b["ub"], 40, 4, 9)
    c, d = oracle.rescale(b["lb"], b["ub"])
    nodes, w = np.polynomial.legendre.leggauss(64)
    for g in (None, oracle.jackson(40)):
        assert abs(np.sum(w * oracle.legendre_dos(muA, g, c + d * nodes, b["lb"], b["ub"])) * d - 1.0) < 1e-13
    assert np.all(oracle.legendre_dos(muA, None, np.array([b["lb"] - 0.1, b["ub"] + 0.1]), b["lb"], b["ub"]) == 0)
