"""FP64 reference of the learned damping network -- TEST INFRASTRUCTURE ONLY.

The paper damps the Chebyshev coefficients with Jackson factors (Appendix A,
eq. (jackson)) and notes that Jackson damping over-smooths (sections 3.1.1 and
4).  The learned alternative maps the first 128 normalised moments to
per-degree damping factors g_k in (0, 1):

    h1 = gelu(x W1 + b1)         128 -> 256
    h2 = gelu(h1 W2 + b2)        256 -> 256
    g  = sigmoid(h2 W3 + b3)     256 -> 128,   g_0 := 1

where gelu(u) = u * Phi(u) (Phi the standard normal CDF).  Training minimises
the L1 distance (eq. (err2), p = 1) between the Gaussian-blurred damped KPM
density and the blurred exact density, on npts midpoints of [-1, 1]:

    phi_tilde_sigma = K (g * mu),   K[i, k] = <w_k T_k / (pi sqrt(1-t^2)), g_sigma(t_i - .)>

with w_0 = 1, w_k = 2 (eq. (expmu) and (tdosFinal), blurred as in section 4).
Parity unpinned (against the paper): the paper has no learned part.  The
oracle is pinned instead by central finite differences (backward), plain
torch CPU layers (forward) and hand-worked steps of the published Adam
algorithm (Kingma & Ba 2015) for the update.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

NIN, NH, NOUT = 128, 256, 128


def gelu(u):
    return 0.5 * u * (1.0 + erf(u / math.sqrt(2.0)))


def gelu_grad(u):
    return 0.5 * (1.0 + erf(u / math.sqrt(2.0))) + u * np.exp(-0.5 * u * u) / math.sqrt(2.0 * math.pi)


def mlp_init(seed: int) -> dict:
    """Weights with fan-in scaled normal entries, zero biases (test helper)."""
    rng = np.random.default_rng(seed)
    return dict(
        W1=rng.normal(0, 1 / math.sqrt(NIN), (NIN, NH)), b1=np.zeros(NH),
        W2=rng.normal(0, 1 / math.sqrt(NH), (NH, NH)), b2=np.zeros(NH),
        W3=rng.normal(0, 1 / math.sqrt(NH), (NH, NOUT)), b3=np.zeros(NOUT),
    )


def mlp_forward(p: dict, X: np.ndarray):
    """Damping factors g [N, 128] for moments X [N, 128]; returns (g, cache)."""
    z1 = X @ p["W1"] + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = gelu(z2)
    z3 = h2 @ p["W3"] + p["b3"]
    g = 1.0 / (1.0 + np.exp(-z3))
    g[:, 0] = 1.0
    return g, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, g=g)


def mlp_backward(p: dict, cache: dict, dg: np.ndarray) -> dict:
    """Gradients of a loss with dL/dg = dg through the network."""
    g = cache["g"]
    dz3 = dg * g * (1.0 - g)
    dz3[:, 0] = 0.0
    grads = dict(W3=cache["h2"].T @ dz3, b3=dz3.sum(axis=0))
    dh2 = dz3 @ p["W3"].T
    dz2 = dh2 * gelu_grad(cache["z2"])
    grads.update(W2=cache["h1"].T @ dz2, b2=dz2.sum(axis=0))
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * gelu_grad(cache["z1"])
    grads.update(W1=cache["X"].T @ dz1, b1=dz1.sum(axis=0))
    return grads


def blur_operator(nmom: int = NOUT, npts: int = 200, sigma: float = 0.02, Q: int = 8192) -> np.ndarray:
    """K[i, k]: blurred density at midpoint t_i contributed by unit g_k mu_k.

    (1/pi) int_0^pi w_k cos(k theta) g_sigma(t_i - cos theta) d theta,
    midpoint rule with Q nodes.
    """
    t = -1.0 + (np.arange(npts) + 0.5) * (2.0 / npts)
    th = (np.arange(Q) + 0.5) * math.pi / Q
    G = np.exp(-np.square(np.subtract.outer(t, np.cos(th))) / (2 * sigma * sigma)) / math.sqrt(2 * math.pi * sigma * sigma)
    C = np.cos(np.multiply.outer(th, np.arange(nmom)))
    w = np.where(np.arange(nmom) == 0, 1.0, 2.0)
    return (G @ C) * w / Q


def mlp_loss_and_grads(p: dict, X: np.ndarray, target: np.ndarray, K: np.ndarray):
    """Mean over the batch of the L1 distance dt * sum_i |K (g*mu) - target|."""
    N, npts = target.shape
    dt = 2.0 / npts
    g, cache = mlp_forward(p, X)
    phi = (g * X) @ K.T
    e = phi - target
    loss = float(np.sum(np.abs(e)) * dt / N)
    dphi = np.sign(e) * dt / N
    dg = (dphi @ K) * X
    return loss, mlp_backward(p, cache, dg), g


# ---------------------------------------------------------------- Adam
# The network is trained with Adam (Kingma & Ba, "Adam: a method for
# stochastic optimization", ICLR 2015, Algorithm 1): exponential moving
# averages of the gradient and of its square, each divided by one minus its
# decay rate raised to the step count (the bias correction of their
# section 3), and a step of lr * m_hat / (sqrt(v_hat) + eps).
ADAM_BETA1, ADAM_BETA2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_step(p: dict, grads: dict, m: dict, v: dict, t: int, lr: float,
              beta1: float = ADAM_BETA1, beta2: float = ADAM_BETA2, eps: float = ADAM_EPS):
    """One Adam update at step t >= 1 (FP64).  Returns new (p, m, v) dicts;
    the inputs are not modified."""
    if t < 1:
        raise ValueError("Adam's step count starts at 1")
    p_new, m_new, v_new = {}, {}, {}
    for name, g in grads.items():
        m_t = beta1 * m[name] + (1.0 - beta1) * g
        v_t = beta2 * v[name] + (1.0 - beta2) * g * g
        m_hat = m_t / (1.0 - beta1 ** t)
        v_hat = v_t / (1.0 - beta2 ** t)
        p_new[name] = p[name] - lr * m_hat / (np.sqrt(v_hat) + eps)
        m_new[name] = m_t
        v_new[name] = v_t
    return p_new, m_new, v_new


def train_full_batch(p: dict, X: np.ndarray, target: np.ndarray, K: np.ndarray, steps: int, lr: float):
    """Adam on the whole batch for `steps` updates from p (moments start at
    zero).  Returns the parameters after each update, the loss before each
    update, and the smallest |residual| of the blurred density met on the
    way (the L1 loss's gradient changes sign where a residual does)."""
    m = {k: np.zeros_like(a) for k, a in p.items()}
    v = {k: np.zeros_like(a) for k, a in p.items()}
    traj, losses, min_resid = [], [], np.inf
    for t in range(1, steps + 1):
        loss, grads, g = mlp_loss_and_grads(p, X, target, K)
        min_resid = min(min_resid, float(np.min(np.abs((g * X) @ K.T - target))))
        p, m, v = adam_step(p, grads, m, v, t, lr)
        traj.append(p)
        losses.append(loss)
    return traj, losses, min_resid
