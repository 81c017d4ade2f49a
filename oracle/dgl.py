"""Legendre expansions: KPM with Legendre polynomials and the
Delta-Gauss-Legendre (DGL) method -- TEST INFRASTRUCTURE ONLY (see the
package header).

Restates, in plain numpy and in the paper's order (Lin, Saad & Yang):

* ``legendre_moments`` -- the stochastic Legendre moments of Algorithm DGL
  (section 3.1.3): for every probe, the three-term recurrence of the Legendre
  polynomials (the step of Algorithm DGL; eq. (Leg) of Appendix B),
      v_1 = B v_0,   v_{k+1} = (2k+1)/(k+1) B v_k - k/(k+1) v_{k-1},
  zeta_k = v_0^T v_k, averaged over probes and divided by n (so that
  mu_0 = 1 for the library's unnormalised +/-1 probes);
* ``dgl_gamma``       -- the expansion coefficients gamma_k(t) of eq.
  (DGLcoeff) by the recurrence of eq. (Leg3) with gamma_0 of eq. (gam0),
  psi_0 = 0, psi_1 = gamma_0, stopped by the rule of eq. (StopRecur);
* ``dgl_dos``         -- eq. (dglexpansion) with the stochastic moments: the
  Gaussian-regularised density at the points;
* ``legendre_dos``    -- KPM with Legendre polynomials (the variant named in
  Appendix A): phi(t) = sum_k (k + 1/2) g_k mu_k L_k(t), the expansion of the
  delta sum in the basis orthogonal for the unit weight on [-1, 1].

Readings: the stopping rule tests |gamma_{k-1}| + |gamma_k| <= k tol once two
coefficients exist (k >= 1); the degree used at a point is that k, capped by
the number of moments available.  The recurrence amplifies rounding noise
once the coefficients have decayed (the instability the paper describes);
since |L_k| <= 1 on [-1, 1] gives |gamma_k| <= gamma_0 exactly, a computed
|gamma_k| > gamma_0 proves divergence and is reported as an error (a tol
too small for the recurrence to reach) instead of returning noise.  Densities are returned in A's units: with
t = (x - c)/d and sigma_B = sigma/d, phi_A(x) = phi_B(t)/d.
"""
from __future__ import annotations

import math

import numpy as np

from . import rademacher_block, rescale


def legendre_moments_per_vector(A, c: float, d: float, M: int, nvec: int, seed: int,
                                vec0: int = 0) -> np.ndarray:
    """zeta[l, k] = v_l^T L_k(B) v_l, k = 0..M, by the Legendre recurrence.
    Probes are rows of a [nvec x n] array, so each dot is a pairwise sum
    over a contiguous row."""
    S = A.to_scipy().tocsr()
    V0 = np.ascontiguousarray(rademacher_block(seed, vec0, nvec, A.n).T)

    def Bx(X):
        return ((S @ X.T).T - c * X) / d

    zeta = np.zeros((nvec, M + 1))
    zeta[:, 0] = np.sum(V0 * V0, axis=1)
    if M == 0:
        return zeta
    Vp, V = V0, Bx(V0)
    zeta[:, 1] = np.sum(V0 * V, axis=1)
    for k in range(1, M):
        Vn = (2 * k + 1) / (k + 1) * Bx(V) - k / (k + 1) * Vp
        zeta[:, k + 1] = np.sum(V0 * Vn, axis=1)
        Vp, V = V, Vn
    return zeta


def legendre_moments(A, lb: float, ub: float, M: int, nvec: int, seed: int) -> np.ndarray:
    """Normalised stochastic Legendre moments mu_k = tr L_k(B) / n estimates,
    k = 0..M, of B = (A - cI)/d."""
    c, d = rescale(lb, ub)
    return legendre_moments_per_vector(A, c, d, M, nvec, seed).sum(axis=0) / (A.n * nvec)


def dgl_gamma(t: float, sigma: float, tol: float, kmax: int):
    """gamma_0..gamma_m(t) for the Gaussian exp(-((s - t)/sigma)^2 / 2) on
    [-1, 1] and the degree m at which eq. (StopRecur) stops the recurrence
    (m <= kmax).  Returns (gamma[0..m], m)."""
    r2s = math.sqrt(2.0) * sigma
    a, b = (1.0 - t) / r2s, (1.0 + t) / r2s
    # eq. (gam0): erf(a) + erf(b); for a centre outside [-1, 1] one argument
    # is negative and the sum cancels, so it is taken as a difference of erfc
    if a < 0.0:
        s = math.erfc(-a) - math.erfc(b)
    elif b < 0.0:
        s = math.erfc(-b) - math.erfc(a)
    else:
        s = math.erf(a) + math.erf(b)
    g = [sigma * math.sqrt(math.pi / 2.0) * s]
    if kmax == 0:
        return np.array(g), 0
    e_hi = math.exp(-0.5 * ((1.0 - t) / sigma) ** 2)  # Gaussian at s = 1
    e_lo = math.exp(-0.5 * ((1.0 + t) / sigma) ** 2)  # Gaussian at s = -1
    psi = [0.0]  # psi_0
    for k in range(kmax):
        zeta_k = e_hi - (e_lo if k % 2 == 0 else -e_lo)
        g_km1 = g[k - 1] if k > 0 else 0.0
        psi_km1 = psi[k - 1] if k > 0 else 0.0
        g.append((2 * k + 1) / (k + 1) * (sigma * sigma * (psi[k] - zeta_k) + t * g[k]) - k / (k + 1) * g_km1)
        psi.append((2 * k + 1) * g[k] + psi_km1)
        m = k + 1
        if not abs(g[m]) <= g[0]:
            # |L_k| <= 1 on [-1, 1] bounds every |gamma_k| by gamma_0: the
            # recurrence has amplified its rounding noise (tol too small)
            raise FloatingPointError(f"gamma recurrence diverged at k = {m} (t = {t}, sigma = {sigma})")
        if abs(g[m - 1]) + abs(g[m]) <= m * tol:
            return np.array(g), m
    return np.array(g), kmax


def dgl_dos(mu: np.ndarray, x: np.ndarray, sigma: float, tol: float, lb: float, ub: float):
    """Eq. (dglexpansion) at points x (A's units) from Legendre moments mu
    (mu_0..mu_M of B): sum_{k <= m_i} (k + 1/2) gamma_k(t_i) mu_k /
    sqrt(2 pi sigma_B^2) / d.  Returns (phi, degree used per point)."""
    c, d = rescale(lb, ub)
    sb = sigma / d
    M = len(mu) - 1
    phi = np.zeros(len(x))
    deg = np.zeros(len(x), dtype=np.int64)
    for i, xi in enumerate(np.asarray(x, dtype=np.float64)):
        g, m = dgl_gamma((xi - c) / d, sb, tol, M)
        k = np.arange(m + 1)
        phi[i] = np.sum((k + 0.5) * g * mu[:m + 1]) / math.sqrt(2.0 * math.pi * sb * sb) / d
        deg[i] = m
    return phi, deg


def legendre_dos(mu: np.ndarray, g: np.ndarray | None, x: np.ndarray, lb: float, ub: float) -> np.ndarray:
    """KPM with Legendre polynomials: sum_k (k + 1/2) g_k mu_k L_k(t) / d at
    t = (x - c)/d (0 for |t| > 1, where the expansion does not apply);
    g = None means no damping."""
    c, d = rescale(lb, ub)
    M = len(mu) - 1
    w = (np.arange(M + 1) + 0.5) * mu * (np.ones(M + 1) if g is None else g)
    t = (np.asarray(x, dtype=np.float64) - c) / d
    out = np.polynomial.legendre.legval(t, w) / d
    return np.where(np.abs(t) <= 1.0, out, 0.0)
