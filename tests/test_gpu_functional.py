"""GPU parity of the density functionals (eq. (errormetric_g)) and the heat
capacity of section 4.3 through the C ABI against the CPU oracle
(``oracle/functional.py``: adaptive quadrature of the definition, and the
Lanczos sum).

The device integrates by Gauss-Chebyshev quadrature on Q nodes; on
functions analytic on [lb, ub] (a spectrum bounded away from the kink of
g_T at lambda = 0) this converges geometrically, so the bar is 1e-12 of the
value on oracle-made moments.  End to end the moments' bar (FP64 1e-12)
enters through sum_k |f_k| <= 2 max|f|, hence 1e-10.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1308_5467_amd as kpm
import synth

pytestmark = pytest.mark.gpu


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


def _shifted_laplacian():
    """2D Dirichlet Laplacian 24 x 24 + 0.5 I: spectrum inside [0.5, 8.5]."""
    A = synth.laplacian2d_dirichlet(24)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    A.val[rows == A.col_idx] += 0.5
    return A, 0.45, 8.55


def test_functional_on_oracle_moments(ctx):
    A = synth.random_sparse_symmetric(1500, 4.5, 3)
    b = oracle.lanczos_bounds(A, 20, 4)
    lb, ub = b["lb"], b["ub"]
    mu = oracle.moments(A, lb, ub, 80, 8, 5)
    f = lambda l: np.exp(-0.2 * l * l) * np.cos(l)
    for g in (None, oracle.jackson(80)):
        got = kpm.kpm_functional(ctx, mu, lb, ub, f, Q=1024, g=g)
        ref = oracle.functional_kpm(mu, g, f, lb, ub)
        assert abs(got - ref) < 1e-12 * max(1.0, abs(ref))


def test_polynomial_exactness(ctx):
    lam = np.linspace(-2.0, 3.0, 23) ** 3 / 10.0
    A = synth.diagonal_matrix(lam)
    mu = kpm.kpm_moments(ctx, dev(A, "f64"), -3.0, 3.0, 10, 2, 5, precision="f64")
    p = np.polynomial.Polynomial([0.3, -1.0, 0.5, 0.2, -0.05, 0.01, 0.002, -0.001])
    assert abs(kpm.kpm_functional(ctx, mu, -3.0, 3.0, p, Q=16) - np.mean(p(lam))) < 1e-12


def test_heat_capacity_kpm(ctx):
    A, lb, ub = _shifted_laplacian()
    D = dev(A, "f64")
    T = np.array([0.1, 0.3, 1.0, 3.0])
    mu = kpm.kpm_moments(ctx, D, lb, ub, 120, 16, 9, precision="f64")
    ref_mu = oracle.moments(A, lb, ub, 120, 16, 9)
    for g in (None, oracle.jackson(120)):
        cv = kpm.kpm_heat_capacity(ctx, ref_mu, lb, ub, T, g=g)
        ref = np.array([oracle.functional_kpm(ref_mu, g, lambda l, t=t: oracle.heat_capacity_g(l, t), lb, ub)
                        for t in T])
        assert np.max(np.abs(cv - ref) / np.abs(ref)) < 1e-12
        cv2 = kpm.kpm_heat_capacity(ctx, mu, lb, ub, T, g=g)  # device moments end to end
        assert np.max(np.abs(cv2 - ref)) < 1e-10
    lam = np.linalg.eigvalsh(A.dense())
    exact = np.array([oracle.functional_exact(lam, lambda l, t=t: oracle.heat_capacity_g(l, t)) for t in T])
    assert np.all(np.diff(cv2) > 0) and np.max(np.abs(cv2 - exact)) < 0.05  # 16 probes: stochastic error


def test_heat_capacity_lanczos(ctx):
    A, lb, ub = _shifted_laplacian()
    T = np.array([0.05, 0.2, 1.0, 4.0])
    th, t2, used = kpm.kpm_slq(ctx, dev(A, "f64"), lb, ub, 40, 6, 11)
    cv = kpm.kpm_slq_heat_capacity(ctx, th, t2, T)
    ref = np.array([oracle.functional_lanczos(th, t2, lambda l, t=t: oracle.heat_capacity_g(l, t)) for t in T])
    assert np.max(np.abs(cv - ref) / np.abs(ref)) < 1e-13
    c, d = oracle.rescale(lb, ub)
    al, be = oracle.lanczos_tridiag(A, c, d, 40, 6, 11)
    rth, rt2, _ = oracle.lanczos_nodes(al, be)
    ref2 = np.array([oracle.functional_lanczos(c + d * rth, rt2, lambda l, t=t: oracle.heat_capacity_g(l, t))
                     for t in T])
    assert np.max(np.abs(cv - ref2)) < 1e-10


def test_errors(ctx):
    mu = np.array([1.0, 0.1, 0.0])
    for T in (np.array([0.0]), np.array([-1.0]), np.array([np.nan])):
        with pytest.raises(kpm.KpmError) as e:
            kpm.kpm_heat_capacity(ctx, mu, 0.0, 1.0, T)
        assert e.value.status == -1
    with pytest.raises(kpm.KpmError):
        kpm.kpm_heat_capacity(ctx, mu, 1.0, 1.0, np.array([1.0]))
    with pytest.raises(kpm.KpmError):
        kpm.kpm_functional(ctx, mu, 0.0, 1.0, np.zeros(0), Q=0)
    assert kpm.kpm_heat_capacity(ctx, mu, 0.0, 1.0, np.zeros(0)).size == 0
