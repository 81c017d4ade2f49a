"""CPU FP64 oracle for the KPM path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library (``paper_1308_5467_amd``) never imports
it, links it or calls it, and the two share no code; only the seeded matrix
generators in ``synth`` feed both.

Each function restates a step of Lin, Saad & Yang, "Approximating spectral
densities of large matrices" in plain numpy / C, in the paper's order:

* ``lanczos_bounds``  -- spectral bounds from a k-step Lanczos run, Ritz values
  widened by their residual norms (section 3.1.1, paragraph after eq. (cd));
* ``rescale``         -- c and d of eq. (cd);
* ``moments``         -- Algorithm 1 with the stochastic trace of eqs. (nuk),
  (muEst) and the recurrence (3term), in C (``kpm_oracle.c``);
* ``jackson``         -- eq. (jackson) of Appendix A;
* ``dos``             -- eq. (tdosFinal) with the (2 - delta_k0)/pi factor of
  eq. (expmu) and the damping of Appendix A;
* ``dos_bins``        -- the same density integrated over intervals;
* ``blurred_*``       -- the Gaussian-regularised densities of eq. (blurphi)
  (with the 1/n that keeps unit mass) and the blurred KPM approximation used
  for comparisons in section 4;
* ``mlp_*``           -- FP64 forward/backward of the damping network;
* ``adam_step``, ``train_full_batch`` -- the Adam update (Kingma & Ba 2015,
  Algorithm 1) the network is trained with, and a full-batch trajectory;
* ``lanczos_*``       -- the stochastic Lanczos method of section 3.2.1
  (``slq.py``);
* ``haydock_dos``     -- Haydock's method of section 3.2.2 from the same
  Lanczos matrices (``slq.py``);
* ``legendre_*``, ``dgl_*`` -- Legendre moments, KPM with Legendre
  polynomials and the Delta-Gauss-Legendre method (section 3.1.3,
  Appendix B) (``dgl.py``);
* ``functional_*``, ``heat_capacity_g`` -- functionals <phi~, g> of the
  approximate densities (eq. (errormetric_g)) and the heat capacity of
  section 4.3 (``functional.py``).

Moments are normalised as mu_hat_k = zeta_k / n (so mu_hat_0 = 1); the
paper's (2 - delta_k0)/pi factor is applied when the density is evaluated.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np
import scipy.linalg as sla

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "kpm_oracle.c")
_lib = None
_lock = threading.Lock()

LANCZOS_START_ID = 2**31 - 1  # probe-vector id reserved for the Lanczos start vector


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (OpenMP over probe vectors)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            i64, u64, i32, dbl, ptr = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_void_p)
            lib.oracle_rademacher.argtypes = [u64, i64, i64, ptr]
            lib.oracle_rademacher.restype = None
            lib.oracle_rademacher_block.argtypes = [u64, i64, i32, i64, ptr]
            lib.oracle_rademacher_block.restype = None
            lib.oracle_splitmix64_nth.argtypes = [u64, u64]
            lib.oracle_splitmix64_nth.restype = u64
            for fn in (lib.oracle_moments, lib.oracle_moments_doubling):
                fn.argtypes = [i64, ptr, ptr, ptr, dbl, dbl, i32, i32, u64, i64, ptr, i32]
                fn.restype = i32
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Probe vectors
# --------------------------------------------------------------------------
def splitmix64_nth(seed: int, k: int) -> int:
    """Output number k (k >= 1) of SplitMix64 started from ``seed``."""
    return int(_load().oracle_splitmix64_nth(seed & (2**64 - 1), k))


def rademacher(seed: int, l: int, n: int) -> np.ndarray:
    """Probe vector l (entries +/-1)."""
    out = np.empty(n, dtype=np.float64)
    _load().oracle_rademacher(seed, l, n, _ptr(out))
    return out


def rademacher_block(seed: int, vec0: int, nvec: int, n: int) -> np.ndarray:
    """Row-major [n x nvec] block of probe vectors vec0 .. vec0+nvec-1."""
    out = np.empty((n, nvec), dtype=np.float64)
    _load().oracle_rademacher_block(seed, vec0, nvec, n, _ptr(out))
    return out


# --------------------------------------------------------------------------
# Bounds and rescaling (section 3.1.1, eq. (cd) and the Lanczos paragraph)
# --------------------------------------------------------------------------
def gershgorin(A) -> tuple[float, float]:
    """Gershgorin hull of the spectrum."""
    S = A.to_scipy()
    diag = S.diagonal()
    absrow = np.asarray(abs(S).sum(axis=1)).ravel() - np.abs(diag)
    return float(np.min(diag - absrow)), float(np.max(diag + absrow))


def lanczos_bounds(A, steps: int = 20, seed: int = 0, margin: float = 0.01) -> dict:
    """Bounds of the spectrum of A from a ``steps``-step Lanczos run.

    Follows the paper: ub = theta_k + ||(A - theta_k) u_k||, lb = theta_1 -
    ||(A - theta_1) u_1||, the residual norms taken from the bottom entries
    of the tridiagonal matrix's eigenvectors (residual = beta_k |z_{k,j}|).
    The start vector is the probe vector with the reserved id 2^31 - 1,
    normalised; every new Lanczos vector is re-orthogonalised twice against
    all previous ones.  On breakdown (beta below 1e-12 of the largest
    coefficient) the Gershgorin hull is merged in.  The interval is then
    widened so that [lb0, ub0] maps into [-(1 - margin), 1 - margin].
    """
    S = A.to_scipy()
    n = A.n
    m = min(steps, n)
    q = rademacher(seed, LANCZOS_START_ID, n)
    q = q / np.linalg.norm(q)
    Q = [q]
    alpha, beta = [], []
    scale = 0.0
    breakdown = False
    beta_last = 0.0
    for j in range(m):
        w = S @ Q[j]
        a = float(Q[j] @ w)
        w = w - a * Q[j]
        if j > 0:
            w = w - beta[j - 1] * Q[j - 1]
        Qm = np.stack(Q, axis=1)
        for _ in range(2):
            w = w - Qm @ (Qm.T @ w)
        b = float(np.linalg.norm(w))
        alpha.append(a)
        scale = max(scale, abs(a), b)
        if j == m - 1:
            beta_last = b
            break
        if b <= 1e-12 * scale:
            breakdown = True
            beta_last = b
            break
        beta.append(b)
        Q.append(w / b)
    k = len(alpha)
    if k == 1:
        theta = np.array(alpha)
        Z = np.ones((1, 1))
    else:
        theta, Z = sla.eigh_tridiagonal(np.array(alpha), np.array(beta[: k - 1]))
    r = beta_last * np.abs(Z[-1, :])
    lb0 = float(theta[0] - r[0])
    ub0 = float(theta[-1] + r[-1])
    if breakdown:
        g_lo, g_hi = gershgorin(A)
        lb0, ub0 = min(lb0, g_lo), max(ub0, g_hi)
    c = 0.5 * (lb0 + ub0)
    d = 0.5 * (ub0 - lb0) / (1.0 - margin)
    d = max(d, margin * max(abs(c), 1.0))
    return dict(lb=c - d, ub=c + d, lb0=lb0, ub0=ub0, alpha=np.array(alpha),
                beta=np.array(beta + [beta_last]), theta=theta, steps=k, breakdown=breakdown)


def rescale(lb: float, ub: float) -> tuple[float, float]:
    """c and d of eq. (cd): B = (A - c I)/d maps [lb, ub] onto [-1, 1]."""
    return 0.5 * (lb + ub), 0.5 * (ub - lb)


# --------------------------------------------------------------------------
# Moments (Algorithm 1)
# --------------------------------------------------------------------------
def moments_per_vector(A, c: float, d: float, M: int, nvec: int, seed: int, vec0: int = 0,
                       nthreads: int = 0, doubling: bool = False) -> np.ndarray:
    """zeta[l, k] = v_l^T T_k(B) v_l for probe vectors vec0 .. vec0+nvec-1."""
    lib = _load()
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    zeta = np.zeros((nvec, M + 1), dtype=np.float64)
    fn = lib.oracle_moments_doubling if doubling else lib.oracle_moments
    rc = fn(A.n, _ptr(rp), _ptr(ci), _ptr(va), c, d, M, nvec, seed, vec0, _ptr(zeta), nthreads)
    if rc != 0:
        raise MemoryError("oracle_moments failed")
    return zeta


def normalize(zeta: np.ndarray, n: int) -> np.ndarray:
    """mu_hat_k = (sum over probe vectors of zeta_k) / (n * nvec), summed exactly."""
    nvec = zeta.shape[0]
    return np.array([math.fsum(zeta[:, k]) for k in range(zeta.shape[1])]) / (n * nvec)


def moments(A, lb: float, ub: float, M: int, nvec: int, seed: int, **kw) -> np.ndarray:
    """Normalised stochastic Chebyshev moments mu_hat_0..M of B = (A - cI)/d."""
    c, d = rescale(lb, ub)
    return normalize(moments_per_vector(A, c, d, M, nvec, seed, **kw), A.n)


# --------------------------------------------------------------------------
# Damping (Appendix A)
# --------------------------------------------------------------------------
def jackson(M: int) -> np.ndarray:
    """Jackson damping factors g_k^M, k = 0..M, eq. (jackson)."""
    a = math.pi / (M + 2)
    k = np.arange(M + 1, dtype=np.float64)
    return ((1.0 - k / (M + 2)) * math.sin(a) * np.cos(k * a)
            + (1.0 / (M + 2)) * math.cos(a) * np.sin(k * a)) / math.sin(a)


# --------------------------------------------------------------------------
# Density evaluation (eq. (tdosFinal), (expmu))
# --------------------------------------------------------------------------
def cheb_T(k: np.ndarray, t: np.ndarray) -> np.ndarray:
    """T_k(t) = cos(k arccos t) for |t| <= 1."""
    return np.cos(np.multiply.outer(np.arccos(np.clip(t, -1.0, 1.0)), k))


def dos_scaled(mu: np.ndarray, g: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Density of B at points t in (-1, 1); 0 for |t| >= 1."""
    M = len(mu) - 1
    t = np.asarray(t, dtype=np.float64)
    w = np.where(np.arange(M + 1) == 0, 1.0, 2.0) / math.pi   # (2 - delta_k0)/pi
    coef = w * g * mu
    inside = np.abs(t) < 1.0
    out = np.zeros_like(t)
    ti = t[inside]
    out[inside] = (cheb_T(np.arange(M + 1), ti) @ coef) / np.sqrt(1.0 - ti * ti)
    return out


def dos(mu, g, lb: float, ub: float, x) -> np.ndarray:
    """Density of A at points x: phi_A(x) = phi_B((x - c)/d) / d."""
    c, d = rescale(lb, ub)
    return dos_scaled(np.asarray(mu), np.asarray(g), (np.asarray(x) - c) / d) / d


def dos_bins(mu, g, lb: float, ub: float, edges) -> np.ndarray:
    """Mass of the density over [edges[i], edges[i+1]], by integrating each
    Chebyshev term exactly in theta = arccos t."""
    c, d = rescale(lb, ub)
    mu, g = np.asarray(mu), np.asarray(g)
    t = np.clip((np.asarray(edges, dtype=np.float64) - c) / d, -1.0, 1.0)
    th = np.arccos(t)
    M = len(mu) - 1
    k = np.arange(1, M + 1)
    F = g[0] * mu[0] * (-th) + 2.0 * (np.sin(np.multiply.outer(th, k)) / k) @ (g[1:] * mu[1:]) * (-1.0)
    F = F / math.pi  # antiderivative in t (increasing with t)
    return np.diff(F)


# --------------------------------------------------------------------------
# Regularised densities and error metrics (section 2, section 4)
# --------------------------------------------------------------------------
def gauss(t, sigma: float):
    """g_sigma of eq. (gauss)."""
    return np.exp(-np.square(t) / (2.0 * sigma * sigma)) / math.sqrt(2.0 * math.pi * sigma * sigma)


def midpoints(npts: int = 200) -> np.ndarray:
    """npts midpoints of [-1, 1] (spacing 2/npts)."""
    return -1.0 + (np.arange(npts) + 0.5) * (2.0 / npts)


def blurred_exact(s: np.ndarray, t: np.ndarray, sigma: float) -> np.ndarray:
    """phi_sigma(t) = (1/n) sum_j g_sigma(t - s_j) for eigenvalues s_j (in B's units)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros(len(t))
    for lo in range(0, len(s), 4096):
        out += gauss(np.subtract.outer(t, s[lo:lo + 4096]), sigma).sum(axis=1)
    return out / len(s)


def blurred_kpm(mu, g, t: np.ndarray, sigma: float, Q: int = 8192) -> np.ndarray:
    """<phi_tilde, g_sigma(. - t)>: the KPM density integrated against a
    Gaussian, in theta = arccos t' with the Q-point midpoint rule."""
    mu, g = np.asarray(mu), np.asarray(g)
    M = len(mu) - 1
    th = (np.arange(Q) + 0.5) * math.pi / Q
    cq = np.cos(np.multiply.outer(th, np.arange(M + 1)))   # [Q, M+1]
    coef = np.where(np.arange(M + 1) == 0, 1.0, 2.0) * g * mu
    series = cq @ coef                                      # [Q]
    G = gauss(np.subtract.outer(t, np.cos(th)), sigma)      # [npts, Q]
    return (G @ series) / Q


def l1_error(phi_ref: np.ndarray, phi: np.ndarray, npts_interval: float = 2.0) -> float:
    """L1 distance on a uniform midpoint grid of the interval (eq. (err2), p = 1)."""
    return float(np.sum(np.abs(phi_ref - phi)) * npts_interval / len(phi))


def linf_error(phi_ref: np.ndarray, phi: np.ndarray) -> float:
    """L-infinity distance on the grid (eq. (errormetric) at the grid points)."""
    return float(np.max(np.abs(phi_ref - phi)))


def exact_moments(s: np.ndarray, M: int) -> np.ndarray:
    """mu_k = (1/n) sum_j T_k(s_j): the moments the stochastic estimate targets."""
    return cheb_T(np.arange(M + 1), np.asarray(s)).mean(axis=0)


def hutchinson_sd(Bdense: np.ndarray, M: int, nvec: int) -> np.ndarray:
    """Standard deviation of mu_hat_k under Rademacher probes:
    Var(v^T X v) = 2 (||X||_F^2 - sum_i X_ii^2) for symmetric X."""
    n = Bdense.shape[0]
    lam, U = np.linalg.eigh(Bdense)
    out = np.zeros(M + 1)
    for k in range(M + 1):
        X = (U * cheb_T(np.array([k]), lam)[:, 0]) @ U.T
        out[k] = math.sqrt(max(2.0 * (np.sum(X * X) - np.sum(np.diag(X) ** 2)), 0.0) / (n * n * nvec))
    return out


def scaled_eigenvalues(A, lb: float, ub: float) -> np.ndarray:
    """Eigenvalues of B = (A - cI)/d by dense eigh (small matrices only)."""
    c, d = rescale(lb, ub)
    return (np.linalg.eigvalsh(A.dense()) - c) / d


from .mlp import (mlp_init, mlp_forward, mlp_backward, mlp_loss_and_grads,  # noqa: E402
                  blur_operator, gelu, adam_step, train_full_batch)
from .slq import (lanczos_tridiag, lanczos_nodes, lanczos_dos, quadrature_moments,  # noqa: E402
                  steps_used as lanczos_steps_used, haydock_dos, lorentz)
from .dgl import (legendre_moments, legendre_moments_per_vector, dgl_gamma, dgl_dos,  # noqa: E402
                  legendre_dos)
from .functional import (heat_capacity_g, functional_exact, functional_kpm,  # noqa: E402
                         functional_lanczos)
