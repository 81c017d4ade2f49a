"""Host logic of the stochastic Lanczos path: the library's tridiagonal
eigensolver (nodes and weights of eq. (landist)) against LAPACK through
scipy, on the CPU (no device work)."""
import numpy as np
import pytest
import scipy.linalg as sla

import paper_1308_5467_amd as kpm


def _ref(a, b):
    if len(a) == 1:
        return np.array(a, dtype=float), np.ones(1)
    w, Z = sla.eigh_tridiagonal(a, b)
    return w, Z[0] ** 2


@pytest.mark.parametrize("m,seed", [(1, 0), (2, 1), (3, 2), (17, 3), (100, 4), (300, 5)])
def test_random_tridiagonal(m, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, m)
    b = rng.uniform(0.05, 0.7, max(m - 1, 0))
    th, w = kpm.kpm_tridiag_eig(a, b)
    rth, rw = _ref(a, b)
    assert np.max(np.abs(th - rth)) < 1e-13
    assert np.max(np.abs(w - rw)) < 1e-11
    assert abs(w.sum() - 1.0) < 1e-13 and np.all(np.diff(th) >= 0)


def test_lanczos_like_matrix_with_close_nodes():
    """Coefficients of a long run on a 2D Laplacian: clustered Ritz values."""
    n = 40
    lam = np.sort(np.add.outer(2 - 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)),
                               2 - 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))).ravel())
    s = (lam - 4.0) / 4.1
    v = np.random.default_rng(0).choice([-1.0, 1.0], s.size) / np.sqrt(s.size)
    # Lanczos on diag(s) (plain recurrence, 120 steps)
    q, qp, bp = v.copy(), np.zeros_like(v), 0.0
    a, b = [], []
    for _ in range(120):
        w = s * q - bp * qp
        al = q @ w
        w -= al * q
        be = np.linalg.norm(w)
        a.append(al)
        b.append(be)
        qp, q, bp = q, w / be, be
    th, w = kpm.kpm_tridiag_eig(np.array(a), np.array(b[:-1]))
    rth, rw = _ref(np.array(a), np.array(b[:-1]))
    assert np.max(np.abs(th - rth)) < 1e-12
    assert np.max(np.abs(w - rw)) < 1e-10


def test_decoupled_blocks_and_zero_diagonal():
    a = np.array([0.0, 0.0, 0.3, 0.3, -0.2])
    b = np.array([0.5, 0.0, 1e-20, 0.4])
    th, w = kpm.kpm_tridiag_eig(a, b)
    rth, rw = _ref(a, b)
    assert np.max(np.abs(th - rth)) < 1e-14
    assert np.max(np.abs(w - rw)) < 1e-14
    # weight only on the block that contains the first unit vector
    assert abs(w[np.argmin(np.abs(th + 0.5))] - 0.5) < 1e-14


def test_rejects_bad_input():
    with pytest.raises(kpm.KpmError):
        kpm.kpm_tridiag_eig(np.array([1.0, np.nan]), np.array([0.1]))
    with pytest.raises(kpm.KpmError):
        kpm.kpm_tridiag_eig(np.array([1.0, 2.0]), np.array([np.inf]))


# Randomised cases (hypothesis): sizes 1..80, coefficients spanning several
# orders of magnitude, including exact zeros in the off-diagonal (decoupled
# blocks) -- the library's QR iteration against LAPACK.
from hypothesis import given, settings, strategies as st  # noqa: E402


@settings(max_examples=60, deadline=None)
@given(m=st.integers(1, 80), seed=st.integers(0, 2**31 - 1), scale=st.sampled_from([1e-6, 1e-2, 1.0, 1e3]),
       zeros=st.integers(0, 3))
def test_random_tridiagonals_property(m, seed, scale, zeros):
    rng = np.random.default_rng(seed)
    a = rng.normal(0.0, scale, m)
    b = np.abs(rng.normal(0.0, scale, max(m - 1, 0)))
    for _ in range(min(zeros, max(m - 1, 0))):
        b[rng.integers(0, m - 1)] = 0.0
    th, w = kpm.kpm_tridiag_eig(a, b)
    rth, rw = _ref(a, b)
    tol = 1e-12 * max(scale, np.max(np.abs(rth)))
    assert np.max(np.abs(th - rth)) <= tol
    assert abs(w.sum() - 1.0) < 1e-12 and np.all(w >= 0.0) and np.all(np.diff(th) >= 0)
    # weights: compare where eigenvalues are well separated (otherwise only
    # their sum over a cluster is determined)
    gaps = np.diff(rth)
    iso = np.ones(m, dtype=bool)
    if m > 1:
        small = gaps < 1e-6 * max(scale, 1e-300)
        iso[:-1] &= ~small
        iso[1:] &= ~small
    assert np.max(np.abs(w[iso] - rw[iso]), initial=0.0) < 1e-9


@pytest.mark.parametrize("m,seed", [(1, 10), (2, 11), (5, 12), (20, 13), (32, 14)])
def test_flipped_matrix_gives_last_components(m, seed):
    """The spectral bounds widen the extreme Ritz values by beta_m |s_m| with
    s_m the last component of the Ritz vector (section 3.1.1): the library
    takes it from the first-component weights of the reversed tridiagonal
    J T J (J the reversal), whose eigenvectors are T's read backwards."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-2, 2, m)
    b = rng.uniform(0.1, 1.0, max(m - 1, 0))
    th, w = kpm.kpm_tridiag_eig(a[::-1].copy(), b[::-1].copy())
    if m == 1:
        rth, last = a.copy(), np.ones(1)
    else:
        rth, Z = sla.eigh_tridiagonal(a, b)
        last = Z[-1] ** 2
    assert np.max(np.abs(th - rth)) < 1e-13
    assert np.max(np.abs(w - last)) < 1e-11
