"""Pins of the stochastic Lanczos oracle (section 3.2.1) against facts the
mathematics fixes, independently of the oracle's own recurrence:

* Gauss quadrature (eq. (tauexpand)): the nodes and weights of an M-step run
  reproduce q_0^T B^q q_0 for every degree q <= 2M - 1 -- computed here by
  repeated products with the dense matrix -- and not for q = 2M;
* diagonal matrices: nodes are the distinct diagonal values and each weight
  is the fraction of the probe's mass on that value (1/n per entry for +/-1
  probes); repeated values end the run early (breakdown) with exact nodes;
* a 1 x 1 matrix;
* unit mass per probe and a non-negative density;
* the blurred density of a long run equals the probe-weighted blurred
  spectrum from dense eigendecomposition (quadrature of a smooth function).
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _bounds(A, pad=0.05):
    lam = np.linalg.eigvalsh(A.dense())
    return lam[0] - pad, lam[-1] + pad


@pytest.mark.parametrize("M", [1, 5, 12])
def test_quadrature_reproduces_probe_moments(M):
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(7), 8.0, 3)
    c, d = oracle.rescale(*_bounds(A))
    nvec, seed = 3, 5
    al, be = oracle.lanczos_tridiag(A, c, d, M, nvec, seed)
    th, t2, m = oracle.lanczos_nodes(al, be)
    assert np.all(m == M)
    qm = oracle.quadrature_moments(th, t2, 2 * M)
    B = (A.dense() - c * np.eye(A.n)) / d
    V = oracle.rademacher_block(seed, 0, nvec, A.n) / math.sqrt(A.n)
    ref = np.zeros_like(qm)
    X = V.copy()
    for q in range(2 * M + 1):
        ref[:, q] = np.sum(V * X, axis=0)
        X = B @ X
    assert np.max(np.abs(qm[:, :2 * M] - ref[:, :2 * M])) < 1e-13
    assert np.max(np.abs(qm[:, 2 * M] - ref[:, 2 * M])) > 1e-10  # degree 2M is beyond the rule


def test_diagonal_matrix_nodes_and_weights():
    d = np.linspace(-0.8, 0.9, 10) ** 3
    A = synth.diagonal_matrix(d)
    al, be = oracle.lanczos_tridiag(A, 0.0, 1.0, 10, 2, 9)
    th, t2, m = oracle.lanczos_nodes(al, be)
    assert np.all(m == 10)
    assert np.max(np.abs(th - np.sort(d))) < 1e-12
    assert np.max(np.abs(t2 - 0.1)) < 1e-12


def test_repeated_values_break_down_with_exact_nodes():
    vals = np.array([-0.5] * 5 + [0.1] * 3 + [0.7] * 4)
    A = synth.diagonal_matrix(np.random.default_rng(2).permutation(vals))
    al, be = oracle.lanczos_tridiag(A, 0.0, 1.0, 8, 3, 4)
    th, t2, m = oracle.lanczos_nodes(al, be)
    assert np.all(m == 3)
    assert np.max(np.abs(th[:, :3] - np.array([-0.5, 0.1, 0.7]))) < 1e-13
    assert np.max(np.abs(t2[:, :3] - np.array([5, 3, 4]) / 12.0)) < 1e-13
    assert np.all(t2[:, 3:] == 0.0)


def test_one_by_one():
    A = synth.diagonal_matrix(np.array([2.5]))
    al, be = oracle.lanczos_tridiag(A, 2.5, 0.5, 5, 1, 0)
    th, t2, m = oracle.lanczos_nodes(al, be)
    assert m[0] == 1 and th[0, 0] == 0.0 and t2[0, 0] == 1.0 and be[0, 0] == 0.0


def test_unit_mass_and_nonnegative_density():
    A = synth.random_sparse_symmetric(400, 4.5, 6)
    c, d = oracle.rescale(*_bounds(A))
    al, be = oracle.lanczos_tridiag(A, c, d, 30, 5, 2)
    th, t2, m = oracle.lanczos_nodes(al, be)
    assert np.max(np.abs(t2.sum(axis=1) - 1.0)) < 1e-13
    t = np.linspace(-1.5, 1.5, 6001)
    phi = oracle.lanczos_dos(th, t2, t, 0.03)
    assert np.all(phi >= 0.0)
    assert abs(np.sum(phi) * (t[1] - t[0]) - 1.0) < 1e-9


def test_long_run_equals_probe_weighted_spectrum():
    """sigma = 0.05: 100 steps integrate the Gaussian exactly to rounding."""
    A = synth.laplacian2d_dirichlet(32)
    lam, U = np.linalg.eigh(A.dense())
    c, d = oracle.rescale(lam[0] - 0.05, lam[-1] + 0.05)
    v = oracle.rademacher_block(7, 0, 1, A.n)[:, 0]
    w = (U.T @ v) ** 2 / A.n
    t = oracle.midpoints(200)
    exact = oracle.gauss(np.subtract.outer(t, (lam - c) / d), 0.05) @ w
    al, be = oracle.lanczos_tridiag(A, c, d, 100, 1, 7)
    th, t2, _ = oracle.lanczos_nodes(al, be)
    assert np.max(np.abs(oracle.lanczos_dos(th, t2, t, 0.05) - exact)) < 1e-12
    al, be = oracle.lanczos_tridiag(A, c, d, 20, 1, 7)
    th, t2, _ = oracle.lanczos_nodes(al, be)
    assert np.max(np.abs(oracle.lanczos_dos(th, t2, t, 0.05) - exact)) > 1e-3  # too short a run
