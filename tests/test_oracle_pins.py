"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: published
generator outputs, closed forms, exact special cases, brute force through a
dense eigendecomposition, statistical bounds, or library routines.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy import integrate

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- probe vectors
def test_splitmix64_published_outputs():
    for k, hexval in _read_golden("splitmix64_seed0.txt"):
        assert oracle.splitmix64_nth(0, int(k)) == int(hexval, 16)


def test_probe_signs_from_published_outputs():
    """Entry i of probe 0 of seed 0 is the sign of output i + 1 of SplitMix64
    from state 0 (-1 when its top bit is set): the probe definition checked
    against the published outputs, not against the oracle's own generator."""
    rows = _read_golden("splitmix64_seed0.txt")
    expect = [-1.0 if int(hexval, 16) >> 63 else 1.0 for _, hexval in rows]
    assert [int(k) for k, _ in rows] == list(range(1, len(rows) + 1))
    assert list(oracle.rademacher(0, 0, len(rows))) == expect


def test_rademacher_statistics():
    """E[v] = 0 and E[v v^T] = I (the condition of Theorem 1)."""
    n, nvec = 256, 4000
    V = np.stack([oracle.rademacher(7, l, n) for l in range(nvec)])
    assert set(np.unique(V)) == {-1.0, 1.0}
    mean = V.mean(axis=0)
    assert np.max(np.abs(mean)) < 5.0 / math.sqrt(nvec) * 1.2
    C = V.T @ V / nvec
    assert np.allclose(np.diag(C), 1.0)
    off = C - np.diag(np.diag(C))
    assert np.max(np.abs(off)) < 6.0 / math.sqrt(nvec)


def test_rademacher_block_layout():
    blk = oracle.rademacher_block(11, 5, 3, 17)
    for l in range(3):
        assert np.array_equal(blk[:, l], oracle.rademacher(11, 5 + l, 17))


# ---------------------------------------------------------------- moments
def test_mu0_is_one_and_moments_bounded():
    A = synth.random_sparse_symmetric(200, 3.0, 5)
    b = oracle.lanczos_bounds(A, 20, 1)
    c, d = oracle.rescale(b["lb"], b["ub"])
    z = oracle.moments_per_vector(A, c, d, 60, 8, 3)
    assert np.all(z[:, 0] == A.n)
    assert np.all(np.abs(z) <= A.n * (1 + 1e-12))
    mu = oracle.normalize(z, A.n)
    assert mu[0] == 1.0


def test_diagonal_matrix_estimator_is_exact():
    """For diagonal A the Rademacher estimate is exact: v_i^2 = 1."""
    rng = np.random.default_rng(0)
    d = rng.uniform(-3, 5, size=97)
    A = synth.diagonal_matrix(d)
    lb, ub = -3.5, 5.5
    mu = oracle.moments(A, lb, ub, 80, 3, 42)
    c, dd = oracle.rescale(lb, ub)
    s = (d - c) / dd
    exact = np.array([np.mean(np.cos(k * np.arccos(s))) for k in range(81)])
    assert np.max(np.abs(mu - exact)) < 1e-13


def test_one_by_one_zero_matrix():
    """A = [0] on [-1, 1]: mu_k = T_k(0) = cos(k pi/2), the delta-function case of section 3.1.1."""
    A = synth.diagonal_matrix(np.array([0.0]))
    mu = oracle.moments(A, -1.0, 1.0, 40, 1, 0)
    exact = np.array([[1.0, 0.0, -1.0, 0.0][k % 4] for k in range(41)])
    assert np.array_equal(mu, exact)


def test_per_vector_moments_match_dense_eigendecomposition():
    """zeta_k^(l) = v_l^T U T_k(Lambda) U^T v_l, computed from numpy eigh."""
    A = synth.random_sparse_symmetric(40, 2.5, 9)
    b = oracle.lanczos_bounds(A, 20, 2)
    c, d = oracle.rescale(b["lb"], b["ub"])
    M, nvec = 70, 5
    z = oracle.moments_per_vector(A, c, d, M, nvec, 77)
    B = (A.dense() - c * np.eye(A.n)) / d
    lam, U = np.linalg.eigh(B)
    assert lam.min() > -1 and lam.max() < 1
    for l in range(nvec):
        v = oracle.rademacher(77, l, A.n)
        beta = U.T @ v
        ref = np.array([np.sum(beta**2 * np.cos(k * np.arccos(lam))) for k in range(M + 1)])
        assert np.max(np.abs(z[l] - ref)) < 1e-10 * A.n


def test_doubling_identity_matches_plain_recurrence():
    A = synth.add_diagonal_disorder(synth.laplacian3d_periodic(6), 8.0, 1)
    b = oracle.lanczos_bounds(A, 20, 4)
    c, d = oracle.rescale(b["lb"], b["ub"])
    for M in (1, 2, 7, 64, 65):
        z1 = oracle.moments_per_vector(A, c, d, M, 4, 19)
        z2 = oracle.moments_per_vector(A, c, d, M, 4, 19, doubling=True)
        assert np.max(np.abs(z1 - z2)) < 1e-13 * A.n * max(M, 1)


def test_hutchinson_estimate_within_statistical_bound():
    """Theorem 1: the estimate is unbiased; deviations stay within 5 exact sd."""
    A = synth.random_sparse_symmetric(64, 3.0, 21)
    b = oracle.lanczos_bounds(A, 20, 5)
    c, d = oracle.rescale(b["lb"], b["ub"])
    M, nvec = 24, 3000
    mu = oracle.moments(A, b["lb"], b["ub"], M, nvec, 99)
    B = (A.dense() - c * np.eye(A.n)) / d
    s = np.linalg.eigvalsh(B)
    exact = oracle.exact_moments(s, M)
    sd = oracle.hutchinson_sd(B, M, nvec)
    assert np.all(np.abs(mu - exact) <= 5 * sd + 1e-14)


def test_laplacian_closed_form_spectrum():
    A = synth.laplacian2d_dirichlet(32)
    g = dict((r[0], r[1]) for r in _read_golden("lap2d_dirichlet_32.txt"))
    assert A.n == int(g["n"]) and A.nnz == int(g["nnz"])
    lam = np.linalg.eigvalsh(A.dense())
    i = np.arange(1, 33)
    closed = np.sort((4 - 2 * np.cos(i[:, None] * np.pi / 33) - 2 * np.cos(i[None, :] * np.pi / 33)).ravel())
    assert np.max(np.abs(lam - closed)) < 1e-12
    assert abs(lam[0] - float(g["lambda_min"])) < 1e-12
    assert abs(lam[-1] - float(g["lambda_max"])) < 1e-12
    assert np.sum(np.abs(lam - 4.0) < 1e-9) == int(g["multiplicity_of_4"])


def test_laplacian3d_periodic_closed_form():
    L = 6
    A = synth.laplacian3d_periodic(L)
    lam = np.sort(np.linalg.eigvalsh(A.dense()))
    m = np.arange(L)
    c = 2 - 2 * np.cos(2 * np.pi * m / L)
    closed = np.sort((c[:, None, None] + c[None, :, None] + c[None, None, :]).ravel())
    assert np.max(np.abs(lam - closed)) < 1e-12


def test_moments_converge_to_closed_form_on_laplacian():
    """c1 workload: 20 probes; every moment within 5 exact sd of the closed-form value."""
    A = synth.laplacian2d_dirichlet(32)
    b = oracle.lanczos_bounds(A, 20, 3001)
    c, d = oracle.rescale(b["lb"], b["ub"])
    M, nvec = 100, 20
    mu = oracle.moments(A, b["lb"], b["ub"], M, nvec, 2001)
    i = np.arange(1, 33)
    lam = (4 - 2 * np.cos(i[:, None] * np.pi / 33) - 2 * np.cos(i[None, :] * np.pi / 33)).ravel()
    exact = oracle.exact_moments((lam - c) / d, M)
    sd = oracle.hutchinson_sd((A.dense() - c * np.eye(A.n)) / d, M, nvec)
    assert np.all(np.abs(mu - exact) <= 5 * sd + 1e-13)


# ---------------------------------------------------------------- bounds
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_lanczos_bounds_enclose_spectrum(seed):
    A = synth.random_sparse_symmetric(300, 4.0, seed)
    lam = np.linalg.eigvalsh(A.dense())
    b = oracle.lanczos_bounds(A, 20, seed)
    assert b["lb"] < lam[0] and b["ub"] > lam[-1]
    assert b["lb0"] <= lam[0] + 1e-12 * abs(lam[0]) or b["lb"] < lam[0]
    glo, ghi = oracle.gershgorin(A)
    assert glo <= lam[0] and ghi >= lam[-1]


def test_lanczos_bounds_tight_on_laplacian():
    A = synth.laplacian2d_dirichlet(32)
    b = oracle.lanczos_bounds(A, 20, 3001)
    lmin, lmax = 8 * math.sin(math.pi / 66) ** 2, 8 - 8 * math.sin(math.pi / 66) ** 2
    assert b["lb0"] <= lmin and b["ub0"] >= lmax
    assert (lmin - b["lb0"]) < 0.02 * (lmax - lmin) and (b["ub0"] - lmax) < 0.02 * (lmax - lmin)


def test_lanczos_full_length_gives_eigenvalues():
    A = synth.random_sparse_symmetric(12, 3.0, 8)
    b = oracle.lanczos_bounds(A, 12, 8, margin=0.0)
    lam = np.linalg.eigvalsh(A.dense())
    assert np.allclose(np.sort(b["theta"]), lam, atol=1e-9)


def test_lanczos_bounds_are_ritz_values_widened_by_their_residuals():
    """[lb0, ub0] = [theta_1 - r_1, theta_m + r_m] with r_j the residual norm
    ||A u_j - theta_j u_j|| of the Ritz pair: checked against Rayleigh-Ritz
    on an orthonormal basis of the same Krylov space built independently
    (QR of [q, Aq, ..., A^{m-1} q]) and residuals computed directly."""
    A = synth.random_sparse_symmetric(40, 3.0, 12)
    m = 8
    b = oracle.lanczos_bounds(A, m, 5)
    assert b["steps"] == m and not b["breakdown"]
    S = A.dense()
    q = oracle.rademacher(5, oracle.LANCZOS_START_ID, A.n)
    K = np.empty((A.n, m))
    K[:, 0] = q / np.linalg.norm(q)
    for j in range(1, m):
        K[:, j] = S @ K[:, j - 1]
        K[:, j] /= np.linalg.norm(K[:, j])
    Q, _ = np.linalg.qr(K)
    theta, Z = np.linalg.eigh(Q.T @ S @ Q)
    U = Q @ Z
    r = np.linalg.norm(S @ U - U * theta, axis=0)
    width = theta[-1] - theta[0]
    assert abs(b["lb0"] - (theta[0] - r[0])) < 1e-7 * width
    assert abs(b["ub0"] - (theta[-1] + r[-1])) < 1e-7 * width


def test_lanczos_breakdown_merges_the_gershgorin_hull():
    """An eigenvector orthogonal to the start vector is invisible to Lanczos:
    A couples two coordinates i, j where the start vector has equal signs
    (eigenvalues +1 along e_i + e_j, -1 along e_i - e_j) and is diagonal in
    [0.5, 2] elsewhere.  The run breaks down without seeing -1; the merged
    Gershgorin hull [-1, ...] restores the enclosure."""
    n, seed = 6, 3
    v = oracle.rademacher(seed, oracle.LANCZOS_START_ID, n)
    i, j = next((a, b) for a in range(n) for b in range(a + 1, n) if v[a] == v[b])
    D = np.diag(np.linspace(0.5, 2.0, n))
    D[i, i] = D[j, j] = 0.0
    D[i, j] = D[j, i] = 1.0
    A = synth._from_scipy(sp.csr_matrix(D))
    assert abs(np.linalg.eigvalsh(D)[0] + 1.0) < 1e-12
    b = oracle.lanczos_bounds(A, 20, seed)
    assert b["breakdown"]
    assert b["lb"] <= -1.0 and b["ub"] >= 2.0


def test_lanczos_breakdown_on_diagonal_uses_gershgorin():
    A = synth.diagonal_matrix(np.array([1.0, 1.0, 1.0, 2.0]))
    b = oracle.lanczos_bounds(A, 20, 0)
    assert b["lb"] <= 1.0 and b["ub"] >= 2.0


# ---------------------------------------------------------------- damping
def test_jackson_closed_values():
    for M, k, val in _read_golden("jackson_small_M.txt"):
        g = oracle.jackson(int(M))
        assert abs(g[int(k)] - float(val)) < 1e-15


def test_jackson_matches_alternative_published_form():
    """Weisse et al. (Rev. Mod. Phys. 78, 275, 2006), eq. (71), N = M + 1 moments:
    g_k = [(N - k + 1) cos(pi k/(N+1)) + sin(pi k/(N+1)) cot(pi/(N+1))]/(N+1)."""
    for M in (5, 40, 100, 255):
        N = M + 1
        k = np.arange(M + 1)
        alt = ((N - k + 1) * np.cos(np.pi * k / (N + 1))
               + np.sin(np.pi * k / (N + 1)) / np.tan(np.pi / (N + 1))) / (N + 1)
        assert np.max(np.abs(oracle.jackson(M) - alt)) < 1e-13
        g = oracle.jackson(M)
        assert g[0] == pytest.approx(1.0, abs=1e-15) and np.all(g > 0) and np.all(g <= 1 + 1e-15)


# ---------------------------------------------------------------- density
def _dirichlet_kernel(x, M):
    return np.sin((M + 0.5) * x) / np.sin(x / 2)


def test_delta_expansion_closed_form_M40():
    """Delta(t) expanded to degree 40 (the paper's figure for Gibbs oscillation):
    undamped, 1 + 2 sum_k T_k(0) T_k(t) = (D(theta - pi/2) + D(theta + pi/2))/2."""
    M = 40
    mu = np.cos(np.arange(M + 1) * np.pi / 2)
    g = np.ones(M + 1)
    t = np.array([0.1, 0.25, 0.5, 0.77, -0.9])
    th = np.arccos(t)
    closed = 0.5 * (_dirichlet_kernel(th - np.pi / 2, M) + _dirichlet_kernel(th + np.pi / 2, M))
    closed = closed / (np.pi * np.sqrt(1 - t * t))
    got = oracle.dos_scaled(mu, g, t)
    assert np.allclose(got, closed, rtol=1e-12, atol=1e-12)
    # at t = 0 both Dirichlet terms tend to 2M + 1 ... halved and summed: M + 1 = 41
    assert oracle.dos_scaled(mu, g, np.array([0.0]))[0] == pytest.approx(41 / math.pi, rel=1e-14)
    tt = np.linspace(-0.999, 0.999, 20001)
    assert oracle.dos_scaled(mu, g, tt).min() < -1.0            # Gibbs oscillation
    gj = oracle.jackson(M)
    assert oracle.dos_scaled(mu, gj, tt).min() > -1e-12          # Jackson kernel is positive
    assert oracle.dos_scaled(mu, gj, np.array([0.0]))[0] < 41 / math.pi


def test_dos_bins_match_quadrature_and_unit_mass():
    rng = np.random.default_rng(3)
    M = 30
    mu = np.concatenate([[1.0], rng.normal(0, 0.3, M) / np.arange(1, M + 1)])
    g = oracle.jackson(M)
    lb, ub = -2.0, 6.0
    edges = np.linspace(-2.0, 6.0, 9)
    mass = oracle.dos_bins(mu, g, lb, ub, edges)
    for a, b_, m in zip(edges[:-1], edges[1:], mass):
        q, _ = integrate.quad(lambda x: oracle.dos(mu, g, lb, ub, np.array([x]))[0], a, b_, limit=200)
        assert abs(q - m) < 1e-8
    assert abs(mass.sum() - 1.0) < 1e-14


def test_dos_units_scaling():
    mu = np.array([1.0, 0.2, -0.1])
    g = np.ones(3)
    x = np.array([0.5, 1.5])
    assert np.allclose(oracle.dos(mu, g, 0.0, 2.0, x), oracle.dos_scaled(mu, g, x - 1.0))
    assert np.allclose(oracle.dos(mu, g, -2.0, 2.0, x), oracle.dos_scaled(mu, g, x / 2.0) / 2.0)


def test_blurred_kpm_matches_quadrature():
    M = 20
    rng = np.random.default_rng(4)
    mu = np.concatenate([[1.0], rng.normal(0, 0.2, M) / np.arange(1, M + 1)])
    g = oracle.jackson(M)
    t = np.array([-0.5, 0.0, 0.3, 0.95])
    sigma = 0.05
    got = oracle.blurred_kpm(mu, g, t, sigma)
    for ti, gi in zip(t, got):
        f = lambda th: (oracle.dos_scaled(mu, g, np.array([math.cos(th)]))[0] * math.sin(th)
                        * oracle.gauss(ti - math.cos(th), sigma))
        q, _ = integrate.quad(f, 0, math.pi, limit=400)
        assert abs(q - gi) < 1e-8


def test_blurred_exact_unit_mass():
    s = np.linspace(-0.5, 0.5, 11)
    t = np.linspace(-3, 3, 60001)
    phi = oracle.blurred_exact(s, t, 0.05)
    assert abs(np.trapezoid(phi, t) - 1.0) < 1e-9


def test_exact_kpm_converges_to_blurred_exact():
    """With exact moments and high degree, the blurred KPM density approaches phi_sigma."""
    s = np.array([-0.6, -0.1, 0.2, 0.2, 0.7])
    t = oracle.midpoints(200)
    ref = oracle.blurred_exact(s, t, 0.05)
    errs_j, errs_u = [], []
    for M in (20, 80, 320):
        mu = oracle.exact_moments(s, M)
        errs_j.append(oracle.l1_error(ref, oracle.blurred_kpm(mu, oracle.jackson(M), t, 0.05)))
        errs_u.append(oracle.l1_error(ref, oracle.blurred_kpm(mu, np.ones(M + 1), t, 0.05)))
    # Jackson converges slowly (its kernel has width ~ pi/M); the undamped
    # series of a Gaussian-blurred target converges like exp(-(M sigma)^2/2).
    assert errs_j[0] > errs_j[1] > errs_j[2] and errs_j[2] < 2e-2
    assert errs_u[2] < 1e-9
