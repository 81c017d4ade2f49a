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


# ---------------------------------------------------------------- Adam
GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _scalar(v):
    return {"w": np.array([float(v)])}


def test_adam_two_steps_hand_worked():
    """Two updates of one scalar against values worked by hand in exact
    rational arithmetic (tests/golden/adam_two_steps.txt)."""
    rows = [ln.split() for ln in open(f"{GOLDEN}/adam_two_steps.txt") if ln.strip() and not ln.startswith("#")]
    p, m, v = _scalar(1.0), _scalar(0.0), _scalar(0.0)
    for (step, m_ref, v_ref, th_ref), g in zip(rows, (0.5, -0.25)):
        p, m, v = oracle.adam_step(p, _scalar(g), m, v, int(step), 0.1)
        assert abs(m["w"][0] - float(m_ref)) < 4e-17
        assert abs(v["w"][0] - float(v_ref)) < 1e-18
        assert abs(p["w"][0] - float(th_ref)) < 1e-15


def test_adam_matches_torch_optimizer():
    """torch.optim.Adam implements the same published algorithm: same
    gradient sequence, same FP64 trajectory."""
    rng = np.random.default_rng(4)
    shapes = {"a": (5, 3), "b": (7,)}
    p = {k: rng.normal(0, 1, s) for k, s in shapes.items()}
    m = {k: np.zeros(s) for k, s in shapes.items()}
    v = {k: np.zeros(s) for k, s in shapes.items()}
    tp = {k: torch.tensor(a.copy(), requires_grad=True) for k, a in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 30):
        g = {k: rng.normal(0, 10.0 ** rng.uniform(-4, 1), s) for k, s in shapes.items()}
        p, m, v = oracle.adam_step(p, g, m, v, t, 3e-3)
        for k in shapes:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
        for k in shapes:
            assert np.max(np.abs(tp[k].detach().numpy() - p[k])) < 1e-14


def test_adam_bias_correction_constant_gradient():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so each update is exactly lr * g / (|g| + eps); a missing or
    mis-powered correction changes the early steps."""
    g = np.array([2.0, -3e-3, 7e-6])
    p, m, v = _scalar(0.0), _scalar(0.0), _scalar(0.0)
    p, m, v = {"w": np.zeros(3)}, {"w": np.zeros(3)}, {"w": np.zeros(3)}
    for t in range(1, 41):
        p, m, v = oracle.adam_step(p, {"w": g}, m, v, t, 1e-2)
        assert np.allclose(p["w"], -t * 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_step_bound():
    """Kingma & Ba, section 2.1: with (1 - beta1) > sqrt(1 - beta2) the
    effective step never exceeds lr (1 - beta1) / sqrt(1 - beta2), and it
    approaches that bound for a gradient spike after a long run of zero
    gradients (the sparse case the paper describes)."""
    lr = 1e-3
    bound = lr * 0.1 / np.sqrt(0.001)
    rng = np.random.default_rng(5)
    spike_at = np.array([1, 2, 10, 100, 1000, 6000])
    p, m, v = {"w": np.zeros(6)}, {"w": np.zeros(6)}, {"w": np.zeros(6)}
    spike_step = np.zeros(6)
    for t in range(1, 6001):
        g = np.where(spike_at == t, rng.normal(0, 1, 6), 0.0)
        if t > 6000 - 50:
            g = g + np.where(spike_at < 6000, rng.normal(0, 1e-3, 6), 0.0)
        p_new, m, v = oracle.adam_step(p, {"w": g}, m, v, t, lr)
        step = np.abs(p_new["w"] - p["w"])
        assert np.all(step <= bound * (1 + 1e-9))
        spike_step = np.where(spike_at == t, step, spike_step)
        p = p_new
    assert abs(spike_step[0] - lr) < 1e-6 * lr      # first step: lr * sign(g), up to eps / |g|
    assert spike_step[-1] > 0.95 * bound            # after 5,999 zero gradients


def test_full_batch_trajectory_descends_and_matches_steps():
    """train_full_batch is adam_step applied to mlp_loss_and_grads in turn."""
    p = oracle.mlp_init(8)
    X, T = _batch(5, 9)
    K = oracle.blur_operator(128, 200, 0.05, 1024)
    traj, losses, min_resid = oracle.train_full_batch(p, X, T, K, 3, 1e-3)
    m = {k: np.zeros_like(a) for k, a in p.items()}
    v = {k: np.zeros_like(a) for k, a in p.items()}
    q = p
    for t in range(1, 4):
        loss, grads, _ = oracle.mlp_loss_and_grads(q, X, T, K)
        assert loss == losses[t - 1]
        q, m, v = oracle.adam_step(q, grads, m, v, t, 1e-3)
        for k in q:
            assert np.array_equal(q[k], traj[t - 1][k])
    assert losses[-1] < losses[0] and min_resid > 0


def test_damping_labels_file_matches_its_recipe():
    """tests/golden/damping_labels.npz holds what make_damping_labels.py
    computes: recompute one training and one held-out matrix of each family
    from the oracle (eigh bounds, blurred exact density), and check the
    counts and that no matrix is both a training and a held-out one."""
    import os
    import sys
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, here)
    try:
        import make_damping_labels as mk
    finally:
        sys.path.remove(here)
    z = np.load(os.path.join(here, "damping_labels.npz"))
    fam, idx, split = z["family"], z["index"], z["split"]
    assert len(fam) == 2848 and int(np.sum(split == 0)) == 2560 and float(z["sigma"]) == 0.02
    keys = {(int(f), int(i)) for f, i in zip(fam, idx)}
    assert len(keys) == len(fam)
    for f in (0, 1, 2, 3):
        for s in (0, 1):
            k = int(np.flatnonzero((fam == f) & (split == s))[0])
            lb, ub, phi = mk.label((int(fam[k]), int(idx[k])))
            assert abs(lb - z["lb"][k]) < 1e-12 * abs(ub - lb) + 1e-12 and abs(ub - z["ub"][k]) < 1e-9
            assert np.max(np.abs(phi - z["label"][k])) < 1e-6 * max(1.0, np.max(phi))
            assert abs(np.sum(phi) * 0.01 - 1.0) < 2e-3  # unit mass up to the tails beyond [-1, 1]
