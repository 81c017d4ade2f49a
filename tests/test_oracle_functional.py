"""Pins of the oracle's density functionals (eq. (errormetric_g)) and the
heat-capacity function of section 4.3, against what the mathematics fixes:

* g_T equals the paper's printed form x^2 e^{-x} / (1 - e^{-x})^2, tends to
  1 at high temperature and 0 at low temperature, and C_v(T) rises with T;
* the KPM functional of exact moments is exact for polynomial g of degree
  <= M (no damping): the truncated series integrates T_0..T_M exactly;
* the Lanczos functional is Gauss quadrature: exact for polynomials of
  degree <= 2m - 1 against v^T p(B) v / v^T v from dense products;
* the KPM heat capacity of exact moments converges to the exact one on a
  spectrum where g_T is analytic.
"""
import math

import numpy as np

import oracle
import synth


def test_heat_capacity_function():
    x = np.concatenate([np.linspace(0.01, 2.0, 50), np.linspace(2.0, 40.0, 50)])
    paper = x ** 2 * np.exp(-x) / (1.0 - np.exp(-x)) ** 2
    assert np.max(np.abs(oracle.heat_capacity_g(x ** 2, 1.0) / paper - 1.0)) < 1e-13
    assert oracle.heat_capacity_g(np.array([0.0, -0.3]), 0.5).tolist() == [1.0, 1.0]
    assert abs(oracle.heat_capacity_g(np.array([4.0]), 1e3)[0] - 1.0) < 1e-6
    assert oracle.heat_capacity_g(np.array([4.0]), 1e-2)[0] < 1e-80
    lam = np.linspace(0.1, 8.0, 30)
    cv = [oracle.functional_exact(lam, lambda l, T=T: oracle.heat_capacity_g(l, T)) for T in np.linspace(0.05, 3, 25)]
    assert np.all(np.diff(cv) > 0)


def test_kpm_functional_exact_for_polynomials():
    lam = np.linspace(-2.0, 3.0, 23) ** 3 / 10.0
    A = synth.diagonal_matrix(lam)
    lb, ub = -3.0, 3.0
    mu = oracle.moments(A, lb, ub, 10, 2, 5)   # diagonal A: the +/-1 estimator is exact
    p = np.polynomial.Polynomial([0.3, -1.0, 0.5, 0.2, -0.05, 0.01, 0.002, -0.001])
    got = oracle.functional_kpm(mu, None, p, lb, ub)
    assert abs(got - np.mean(p(lam))) < 1e-12


def test_lanczos_functional_is_gauss_quadrature():
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(6), 4.0, 9)
    lam = np.linalg.eigvalsh(A.dense())
    c, d = 0.5 * (lam[0] + lam[-1]), 0.6 * (lam[-1] - lam[0])
    m, nvec, seed = 4, 3, 7
    al, be = oracle.lanczos_tridiag(A, c, d, m, nvec, seed)
    th, t2, used = oracle.lanczos_nodes(al, be)
    assert np.all(used == m)
    p = np.polynomial.Polynomial([1.0, 0.2, -0.3, 0.05, 0.01, -0.002, 0.0004, 1e-5])  # degree 7 = 2m - 1
    got = oracle.functional_lanczos(c + d * th, t2, p)
    V = oracle.rademacher_block(seed, 0, nvec, A.n)
    Ad = A.dense()
    ref = 0.0
    for l in range(nvec):
        v = V[:, l]
        pv = sum(coef * np.linalg.matrix_power(Ad, j) @ v for j, coef in enumerate(p.coef))
        ref += v @ pv / (v @ v)
    assert abs(got - ref / nvec) < 1e-10 * abs(ref / nvec)


def test_kpm_heat_capacity_converges():
    A = synth.laplacian2d_dirichlet(16)
    N = 16
    i = np.arange(1, N + 1)
    lam = np.add.outer(4 - 2 * np.cos(i * np.pi / (N + 1)), -2 * np.cos(i * np.pi / (N + 1))).ravel() + 0.5
    Ad = A.dense() + 0.5 * np.eye(A.n)  # shifted Dirichlet Laplacian: spectrum in [0.5, 8.5]
    assert np.max(np.abs(np.sort(lam) - np.linalg.eigvalsh(Ad))) < 1e-12
    S = synth.diagonal_matrix(lam)
    lb, ub = 0.4, 8.6
    mu = oracle.moments(S, lb, ub, 120, 1, 3)   # exact moments (diagonal, +/-1 probe)
    for T in (0.2, 0.7, 2.0):
        f = lambda l, T=T: oracle.heat_capacity_g(l, T)
        assert abs(oracle.functional_kpm(mu, None, f, lb, ub) - oracle.functional_exact(lam, f)) < 1e-9
