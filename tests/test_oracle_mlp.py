"""Pins of the oracle's learned-damping network (FP64).

Parity of the learned part with the paper is unpinned (the paper has none);
the oracle's forward pass is pinned to plain torch CPU layers, its backward
pass to central finite differences, and its blur operator to the
quadrature-checked blurred KPM density.
"""
import math

import numpy as np
import torch

import oracle
from oracle import mlp as omlp


def _batch(N=6, seed=0):
    rng = np.random.default_rng(seed)
    X = np.concatenate([np.ones((N, 1)), rng.normal(0, 0.3, (N, 127)) / np.sqrt(np.arange(1, 128))], axis=1)
    T = np.abs(rng.normal(0, 1, (N, 200)))
    return X, T


def test_forward_matches_torch_layers():
    p = oracle.mlp_init(3)
    X, _ = _batch()
    g, _ = oracle.mlp_forward(p, X)
    t = {k: torch.tensor(v, dtype=torch.float64) for k, v in p.items()}
    x = torch.tensor(X, dtype=torch.float64)
    h = torch.nn.functional.gelu(x @ t["W1"] + t["b1"], approximate="none")
    h = torch.nn.functional.gelu(h @ t["W2"] + t["b2"], approximate="none")
    ref = torch.sigmoid(h @ t["W3"] + t["b3"]).numpy()
    ref[:, 0] = 1.0
    assert np.max(np.abs(g - ref)) < 1e-14


def test_gelu_grad_matches_autograd():
    u = torch.linspace(-6, 6, 1001, dtype=torch.float64, requires_grad=True)
    torch.nn.functional.gelu(u, approximate="none").sum().backward()
    assert np.max(np.abs(omlp.gelu_grad(u.detach().numpy()) - u.grad.numpy())) < 1e-14


def test_blur_operator_matches_blurred_kpm():
    K = oracle.blur_operator(128, 200, 0.02, 4096)
    rng = np.random.default_rng(1)
    mu = np.concatenate([[1.0], rng.normal(0, 0.3, 127) / np.arange(1, 128)])
    g = oracle.jackson(127)
    t = oracle.midpoints(200)
    assert np.max(np.abs(K @ (g * mu) - oracle.blurred_kpm(mu, g, t, 0.02, Q=4096))) < 1e-11


def test_backward_matches_finite_differences():
    p = oracle.mlp_init(5)
    X, T = _batch(4, 2)
    K = oracle.blur_operator(128, 200, 0.05, 2048)
    _, grads, _ = oracle.mlp_loss_and_grads(p, X, T, K)
    rng = np.random.default_rng(7)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=6, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _, _ = oracle.mlp_loss_and_grads(p, X, T, K)
            flat[idx] = old - h
            lm, _, _ = oracle.mlp_loss_and_grads(p, X, T, K)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = grads[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)


def test_output_zero_is_pinned_to_one():
    p = oracle.mlp_init(1)
    X, _ = _batch()
    g, _ = oracle.mlp_forward(p, X)
    assert np.all(g[:, 0] == 1.0) and np.all((g > 0) & (g <= 1))
