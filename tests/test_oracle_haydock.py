"""Pins of the oracle's Haydock density (section 3.2.2) against facts the
mathematics fixes, independently of its dense complex solves:

* the resolvent entry e_1^T (z - T)^{-1} e_1 equals sum_k tau_k^2 / (z - theta_k)
  over the eigenpairs of T (LAPACK's tridiagonal eigensolver), so the
  density equals the Lorentzian-blurred Lanczos quadrature;
* a full run on a diagonal matrix (Krylov space = whole space) gives the
  exact Lorentzian-regularised density (1/n) sum_j L_eta(x - lambda_j) of the
  paper's first form of phi_eta, for +/-1 probes;
* repeated values end the run early and keep the exact density;
* a 1 x 1 matrix gives one Lorentzian; the density is non-negative (the
  -Im reading) with unit mass.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _lorentz_sum(theta, tau2, x, eta):
    return np.array([np.sum(tau2 * oracle.lorentz(xi - theta, eta)) for xi in x]) / theta.shape[0]


@pytest.mark.parametrize("M,eta", [(8, 0.3), (30, 0.05)])
def test_equals_lorentzian_over_ritz_nodes(M, eta):
    A = synth.random_sparse_symmetric(400, 4.5, 3)
    b = oracle.lanczos_bounds(A, 20, 4)
    c, d = oracle.rescale(b["lb"], b["ub"])
    al, be = oracle.lanczos_tridiag(A, c, d, M, 4, 11)
    th, t2, m = oracle.lanczos_nodes(al, be)
    x = np.linspace(b["lb"] - 1.0, b["ub"] + 1.0, 97)
    phi = oracle.haydock_dos(al, be, m, x, eta, c, d)
    ref = _lorentz_sum(c + d * th, t2, x, eta)
    assert np.max(np.abs(phi - ref)) < 1e-11 * np.max(ref)


def test_full_run_on_diagonal_is_exact_density():
    lam = np.linspace(-2.0, 3.0, 10) ** 3 / 9.0
    A = synth.diagonal_matrix(np.random.default_rng(0).permutation(lam))
    c, d = 0.2, 4.0
    al, be = oracle.lanczos_tridiag(A, c, d, 10, 3, 5)
    m = oracle.lanczos_steps_used(al, be)
    assert np.all(m == 10)
    x = np.linspace(-4.0, 4.0, 161)
    eta = 0.07
    ref = np.array([np.mean(oracle.lorentz(xi - lam, eta)) for xi in x])
    phi = oracle.haydock_dos(al, be, m, x, eta, c, d)
    assert np.max(np.abs(phi - ref)) < 1e-10 * np.max(ref)


def test_repeated_values_break_down_exactly():
    vals = np.array([-0.5] * 50 + [0.1] * 30 + [0.7] * 40)
    A = synth.diagonal_matrix(np.random.default_rng(2).permutation(vals))
    al, be = oracle.lanczos_tridiag(A, 0.0, 1.0, 8, 2, 4)
    m = oracle.lanczos_steps_used(al, be)
    assert np.all(m == 3)
    x = np.linspace(-1.0, 1.0, 41)
    eta = 0.02
    ref = (50 * oracle.lorentz(x + 0.5, eta) + 30 * oracle.lorentz(x - 0.1, eta)
           + 40 * oracle.lorentz(x - 0.7, eta)) / 120.0
    phi = oracle.haydock_dos(al, be, m, x, eta, 0.0, 1.0)
    assert np.max(np.abs(phi - ref)) < 1e-11 * np.max(ref)


def test_one_by_one():
    A = synth.diagonal_matrix(np.array([2.5]))
    al, be = oracle.lanczos_tridiag(A, 2.0, 0.5, 3, 1, 0)
    m = oracle.lanczos_steps_used(al, be)
    assert m[0] == 1
    x = np.array([1.0, 2.5, 2.6, 7.0])
    phi = oracle.haydock_dos(al, be, m, x, 0.1, 2.0, 0.5)
    assert np.max(np.abs(phi - 0.1 / math.pi / ((x - 2.5) ** 2 + 0.01))) < 1e-13


def test_nonnegative_unit_mass():
    A = synth.add_diagonal_disorder(synth.laplacian2d_dirichlet(12), 4.0, 8)
    b = oracle.lanczos_bounds(A, 20, 6)
    c, d = oracle.rescale(b["lb"], b["ub"])
    al, be = oracle.lanczos_tridiag(A, c, d, 25, 3, 8)
    m = oracle.lanczos_steps_used(al, be)
    eta, R = 0.1, 40.0
    x = np.arange(c - R, c + R + 1e-9, eta / 10.0)
    phi = oracle.haydock_dos(al, be, m, x, eta, c, d)
    assert np.all(phi > 0.0)
    mass = np.trapezoid(phi, x)
    # every node lies within d of c: a Lorentzian's mass beyond distance r of
    # its centre is ~ (2/pi) eta / r, with r between R - d and R + d here
    lo = 1.0 - 2.0 / math.pi * eta / (R - d)
    hi = 1.0 - 2.0 / math.pi * eta / (R + d)
    assert lo - 1e-5 < mass < hi + 1e-5
