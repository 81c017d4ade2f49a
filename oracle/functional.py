"""Functionals of the density (section 2, eq. (errormetric_g)) and the heat
capacity of section 4.3 -- TEST INFRASTRUCTURE ONLY (see the package header).

For a smooth g, <phi, g> = int g(lambda) phi(lambda) dlambda = (1/n) sum_j
g(lambda_j), and an approximate density is measured by
E[phi~; g] = |<phi, g> - <phi~, g>|.  Restated here in plain numpy/scipy:

* ``functional_exact``   -- (1/n) sum_j g(lambda_j) from the eigenvalues;
* ``functional_kpm``     -- <phi~, g> for the KPM density of eq. (tdosFinal)
  with damping g_k, as the integral of g times the density, written in
  theta = arccos t and integrated by adaptive quadrature:
      (1/pi) int_0^pi g(c + d cos theta) sum_k (2 - delta_k0) g_k mu_k cos(k theta) dtheta;
* ``functional_lanczos`` -- <phi~, g> for the Lanczos density of eq.
  (lanapprox) with g in place of the Gaussian (as section 4.3 does):
  (1/nvec) sum_l sum_k tau_k^2 g(theta_k);
* ``heat_capacity_g``    -- g of eq. (gfunc) in units where k_B = 1 and
  hbar c / k_B = 1, as a function of lambda = omega^2:
      g_T(lambda) = x^2 e^{-x} / (1 - e^{-x})^2,  x = sqrt(lambda) / T,
  which equals (x / (2 sinh(x/2)))^2 (-> 1 as x -> 0).

Reading: eq. (heatcv) integrates over frequencies omega = sqrt(lambda) >= 0
(a Hessian has no negative eigenvalues); an approximate density may put
mass slightly below 0 (the bounds' margin), where g_T is taken at lambda = 0
(its value 1).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad


def heat_capacity_g(lam, T: float):
    """g_T(lambda) of eq. (gfunc) (k_B = hbar c / k_B = 1), elementwise."""
    x = np.sqrt(np.maximum(np.asarray(lam, dtype=np.float64), 0.0)) / T
    out = np.ones_like(x)
    nz = x > 0.0
    h = 0.5 * x[nz]
    out[nz] = (h / np.sinh(h)) ** 2
    return out


def functional_exact(lam: np.ndarray, f) -> float:
    """(1/n) sum_j f(lambda_j)."""
    return float(np.mean(f(np.asarray(lam, dtype=np.float64))))


def functional_kpm(mu: np.ndarray, g: np.ndarray | None, f, lb: float, ub: float,
                   breakpoints=()) -> float:
    """<phi~, f> of the damped KPM density (mu: normalised Chebyshev moments
    mu_0..mu_M of B), by adaptive quadrature in theta; `breakpoints` are
    points of A's axis where f is not smooth."""
    c, d = 0.5 * (lb + ub), 0.5 * (ub - lb)
    M = len(mu) - 1
    w = (np.ones(M + 1) if g is None else np.asarray(g)) * np.asarray(mu)
    w = w * np.where(np.arange(M + 1) == 0, 1.0, 2.0)
    k = np.arange(M + 1)

    def integrand(th):
        return float(f(np.array([c + d * math.cos(th)]))[0]) * float(np.dot(w, np.cos(k * th)))

    pts = sorted(math.acos(min(1.0, max(-1.0, (p - c) / d))) for p in breakpoints if lb < p < ub)
    edges = [0.0] + pts + [math.pi]
    total = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        total += quad(integrand, a, b, limit=2000, epsabs=1e-14, epsrel=1e-13)[0]
    return total / math.pi


def functional_lanczos(theta: np.ndarray, tau2: np.ndarray, f) -> float:
    """(1/nvec) sum_l sum_k tau2[l, k] f(theta[l, k]) (unused slots have
    tau2 = 0)."""
    return float(np.sum(tau2 * f(theta)) / theta.shape[0])
