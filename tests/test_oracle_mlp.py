"""Pins of the learned-preconditioner network oracle: gradients against central
finite differences, the untrained network equal to its base preconditioner,
positive homogeneity of the preconditioned vector, the loss of a zero network,
and Adam's closed-form steps."""
import numpy as np

import synth
from oracle import mlp


def _data(S=5, H=6, nleaf=7, seed=0):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(1, S + 1, nleaf)
    sizes[2] = S                                   # a full leaf
    leaf_ptr = np.concatenate([[0], np.cumsum(sizes)])
    n = leaf_ptr[-1]
    r = synth.complex_normal(n, seed + 1)
    b = synth.complex_normal(n, seed + 2)
    e = synth.complex_normal(n, seed + 3)
    b[leaf_ptr[4]:leaf_ptr[5]] = 0                 # a leaf with zero base output
    return leaf_ptr, r, b, e


def test_gradient_matches_central_differences():
    S, H = 5, 6
    leaf_ptr, r, b, e = _data(S, H)
    u, _ = mlp.features(r, b, leaf_ptr, S)
    t, mask = mlp.targets(e, b, leaf_ptr, S)
    theta = synth.mlp_weights(S, H, seed=5, zero_last=False, bias_std=0.3).astype(np.float64)
    loss, g = mlp.loss_and_grad(theta, u, t, mask, S, H)
    h = 1e-6
    rng = np.random.default_rng(9)
    idx = np.concatenate([rng.choice(len(theta), 60, replace=False),
                          [len(theta) - 1, 4 * S * H]])   # last bias, first c1 entry
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, u, t, mask, S, H)[0] - mlp.loss_and_grad(tm, u, t, mask, S, H)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
    # ReLU kinks aside, a small step along -g lowers the loss by about eps |g|^2
    eps = 1e-4 / np.linalg.norm(g)
    l2 = mlp.loss_and_grad(theta - eps * g, u, t, mask, S, H)[0]
    assert abs((loss - l2) - eps * g @ g) <= 1e-2 * eps * g @ g


def test_untrained_network_is_the_base():
    S, H = 5, 6
    leaf_ptr, r, b, e = _data(S, H)
    theta = synth.mlp_weights(S, H, seed=1)        # zero last layer
    z = mlp.apply(theta, r, lambda v: b, leaf_ptr, S, H)
    assert np.array_equal(z, b)


def test_positive_homogeneity():
    S, H = 5, 6
    leaf_ptr, r, b, e = _data(S, H)
    M = np.random.default_rng(3).standard_normal((len(r), len(r)))   # a linear base
    theta = synth.mlp_weights(S, H, seed=2, zero_last=False, bias_std=0.1).astype(np.float64)
    z1 = mlp.apply(theta, r, lambda v: M @ v, leaf_ptr, S, H)
    z2 = mlp.apply(theta, 7.5 * r, lambda v: M @ v, leaf_ptr, S, H)
    assert np.allclose(z2, 7.5 * z1, rtol=1e-13, atol=0)


def test_features_unit_norm_and_padding():
    S = 5
    leaf_ptr, r, b, e = _data(S)
    u, scale = mlp.features(r, b, leaf_ptr, S)
    for a in range(len(leaf_ptr) - 1):
        Sa = leaf_ptr[a + 1] - leaf_ptr[a]
        assert abs(np.linalg.norm(u[a, :2 * S]) - 1) < 1e-14
        assert np.all(u[a, Sa:S] == 0) and np.all(u[a, 2 * S + Sa:3 * S] == 0)
        if scale[a] > 0:
            assert abs(np.linalg.norm(u[a, 2 * S:]) - 1) < 1e-14
        else:
            assert np.all(u[a, 2 * S:] == 0)


def test_loss_of_zero_network_is_target_energy():
    S, H = 5, 6
    leaf_ptr, r, b, e = _data(S, H)
    u, _ = mlp.features(r, b, leaf_ptr, S)
    t, mask = mlp.targets(e, b, leaf_ptr, S)
    theta = synth.mlp_weights(S, H, seed=1)
    loss, _ = mlp.loss_and_grad(theta, u, t, mask, S, H)
    rows = [a for a in range(len(leaf_ptr) - 1) if np.linalg.norm(b[leaf_ptr[a]:leaf_ptr[a + 1]]) > 0]
    energy = sum(np.linalg.norm((e - b)[leaf_ptr[a]:leaf_ptr[a + 1]]) ** 2
                 / np.linalg.norm(b[leaf_ptr[a]:leaf_ptr[a + 1]]) ** 2 for a in rows)
    assert abs(loss - energy / len(rows)) <= 1e-12 * loss


def test_adam_closed_form_steps():
    # constant gradient: m_hat = g and v_hat = g^2 at every step, so each step
    # moves lr * |g| / (|g| + eps) against the sign of g
    g = np.array([3.0, -0.5, 1e-3])
    opt = mlp.Adam(3, lr=0.01)
    th = np.zeros(3)
    for k in range(5):
        th = opt.step(th, g)
        step = 0.01 * np.abs(g) / (np.abs(g) + 1e-8)
        assert np.allclose(th, -(k + 1) * np.sign(g) * step, rtol=1e-12, atol=0)
    # two different gradients: hand-evaluated second step
    opt = mlp.Adam(1, lr=0.1)
    th = opt.step(np.zeros(1), np.array([1.0]))
    th = opt.step(th, np.array([-2.0]))
    m = 0.9 * 0.1 * 1.0 + 0.1 * -2.0
    v = 0.999 * 0.001 * 1.0 + 0.001 * 4.0
    expect = -0.1 / (1 + 1e-8) - 0.1 * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert abs(th[0] - expect) <= 1e-14
