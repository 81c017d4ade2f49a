"""Stochastic Lanczos DOS -- TEST INFRASTRUCTURE ONLY (see the package header).

Restates the "Lanczos method" of Lin, Saad & Yang, section 3.2.1 (eqs.
(lanfact), (landist), (lanapprox), (landos)) in plain numpy, in the paper's
order:

* ``lanczos_tridiag``  -- for every probe vector v_l, an M-step Lanczos
  factorisation A V_M = V_M T_M + f_M e_M^T (eq. (lanfact)) started from
  v_l / ||v_l||, by the plain three-term recurrence (no re-orthogonalisation:
  the paper's method counts M matrix-vector products per probe);
* ``lanczos_nodes``    -- eigenvalues theta_k of T_M and the squared first
  components tau_k^2 of its normalised eigenvectors (eq. (landist));
* ``lanczos_dos``      -- the Gaussian-blurred average over probes, eq.
  (landos);
* ``haydock_dos``      -- Haydock's method (section 3.2.2): the
  Lorentzian-regularised density -(1/pi) Im e_1^T (z - T_M)^{-1} e_1 of
  each probe's tridiagonal matrix, averaged over probes.  The paper's
  second form of phi_eta writes +Im; the imaginary part of the resolvent is
  negative there, so the density takes -Im (a reading).

Normalisation (the paper's eq. (lanapprox) carries a 1/n whose matching
factor is the squared norm of the start vector): a Rademacher probe has
||v||^2 = n, the Lanczos basis starts from v/||v||, and the weight of node
theta_k is ||v||^2 tau_k^2 / n = tau_k^2, so every probe contributes unit
mass.  The run is on B = (A - cI)/d (eq. (cd)); Ritz values are mapped back
as c + d theta.  Lanczos is shift- and scale-invariant, so this changes only
rounding.

Breakdown: the run of a probe stops at the first step k whose residual norm
beta_k is at most 1e-12 of the largest |alpha_j|, beta_j seen so far; its
tridiagonal matrix is then k + 1 square (an invariant subspace was found and
its nodes and weights are exact).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import rademacher_block, gauss

BREAKDOWN_REL = 1e-12


def lanczos_tridiag(A, c: float, d: float, M: int, nvec: int, seed: int, vec0: int = 0):
    """alpha[l, k], beta[l, k] (k < M) of the M-step Lanczos run of probe
    vec0 + l on B = (A - cI)/d.  beta[l, k] = ||r_k||, the coupling between
    q_k and q_{k+1}; beta[l, M - 1] is the norm of the final residual f_M.

    One step (q_{-1} = 0, beta_{-1} = 0):
        w = B q_k - beta_{k-1} q_{k-1};  alpha_k = q_k . w;
        r_k = w - alpha_k q_k;  beta_k = ||r_k||;  q_{k+1} = r_k / beta_k.
    Columns of the [n x nvec] block are independent probes.
    """
    S = A.to_scipy().tocsr()
    n = A.n
    V = rademacher_block(seed, vec0, nvec, n)
    Q = V / np.sqrt(np.sum(V * V, axis=0))
    Qp = np.zeros_like(Q)
    bp = np.zeros(nvec)
    alpha = np.zeros((nvec, M))
    beta = np.zeros((nvec, M))
    for k in range(M):
        W = (S @ Q - c * Q) / d - bp * Qp
        a = np.sum(Q * W, axis=0)
        R = W - a * Q
        b = np.sqrt(np.sum(R * R, axis=0))
        alpha[:, k] = a
        beta[:, k] = b
        inv = np.where(b > 0.0, 1.0 / np.where(b > 0.0, b, 1.0), 0.0)
        Qp, Q, bp = Q, R * inv, b
    return alpha, beta


def steps_used(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Size of each probe's tridiagonal matrix after the breakdown rule."""
    nvec, M = alpha.shape
    out = np.full(nvec, M, dtype=np.int64)
    for l in range(nvec):
        scale = 0.0
        for k in range(M - 1):
            scale = max(scale, abs(alpha[l, k]), beta[l, k])
            if beta[l, k] <= BREAKDOWN_REL * scale:
                out[l] = k + 1
                break
    return out


def lanczos_nodes(alpha: np.ndarray, beta: np.ndarray):
    """theta[l, k] ascending and tau2[l, k] (zero past the probe's size m_l),
    and m_l, from the tridiagonal matrices T = tridiag(beta, alpha, beta)."""
    nvec, M = alpha.shape
    m = steps_used(alpha, beta)
    theta = np.zeros((nvec, M))
    tau2 = np.zeros((nvec, M))
    for l in range(nvec):
        k = int(m[l])
        if k == 1:
            w, Z = np.array([alpha[l, 0]]), np.ones((1, 1))
        else:
            w, Z = sla.eigh_tridiagonal(alpha[l, :k], beta[l, :k - 1])
        theta[l, :k] = w
        tau2[l, :k] = Z[0, :] ** 2
    return theta, tau2, m


def lanczos_dos(theta: np.ndarray, tau2: np.ndarray, t: np.ndarray, sigma: float) -> np.ndarray:
    """Eq. (landos): (1/nvec) sum_l sum_k tau2[l, k] g_sigma(t - theta[l, k])
    (nodes and t in the same units; unused slots have tau2 = 0)."""
    th = theta.ravel()
    w = tau2.ravel()
    out = np.zeros(len(t))
    for lo in range(0, len(th), 8192):
        out += gauss(np.subtract.outer(t, th[lo:lo + 8192]), sigma) @ w[lo:lo + 8192]
    return out / theta.shape[0]


def quadrature_moments(theta: np.ndarray, tau2: np.ndarray, qmax: int) -> np.ndarray:
    """sum_k tau2[l, k] theta[l, k]^q for q = 0..qmax (per probe)."""
    return np.stack([np.sum(tau2 * theta ** q, axis=1) for q in range(qmax + 1)], axis=1)


def haydock_dos(alpha: np.ndarray, beta: np.ndarray, m: np.ndarray, x: np.ndarray, eta: float,
                c: float, d: float) -> np.ndarray:
    """Haydock's method (section 3.2.2): the Lorentzian-regularised density
    at points x (A's units) from the Lanczos matrices alone, no Ritz values:

        phi_eta(x) = (1/nvec) sum_l -(1/pi) Im e_1^T ((x + i eta) I - T_l)^{-1} e_1,

    T_l = c I + d tridiag(beta, alpha, beta)[:m_l, :m_l] the probe's
    tridiagonal matrix in A's units (alpha, beta are those of B).  Written
    from the definition: one dense complex solve per probe and point (the
    continued fraction of eq. (cfHaydock) is the same quantity).  The minus
    sign makes the density non-negative: Im 1/(x + i eta - lambda) < 0.
    Unit mass per probe, as in ``lanczos_dos``."""
    x = np.asarray(x, dtype=np.float64)
    nvec = alpha.shape[0]
    out = np.zeros(x.size)
    for l in range(nvec):
        k = int(m[l])
        T = np.diag(c + d * alpha[l, :k]).astype(complex)
        if k > 1:
            off = d * beta[l, :k - 1]
            T += np.diag(off, 1) + np.diag(off, -1)
        e1 = np.zeros((x.size, k, 1), dtype=complex)
        e1[:, 0, 0] = 1.0
        Z = (x + 1j * eta)[:, None, None] * np.eye(k) - T  # one matrix per point
        g = np.linalg.solve(Z, e1)[:, 0, 0]
        out += -g.imag / math.pi
    return out / nvec


def lorentz(t, eta: float):
    """Lorentzian of half-width eta, unit mass: (eta/pi) / (t^2 + eta^2)."""
    return (eta / math.pi) / (np.asarray(t) ** 2 + eta * eta)
