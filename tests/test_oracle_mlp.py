"""Pins of the cost-model oracle (oracle.mlp) against facts that do not come
from its own formulas: the library's bfloat16 conversion, central finite
differences, closed forms of degenerate networks and of Adam's first step."""
import numpy as np
import pytest
import torch

from oracle import mlp

D, H, O = 7, 5, 2


def params(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(mlp.count(D, H, O)) * scale).astype(np.float32)


def data(seed, B=9):
    rng = np.random.default_rng(seed + 100)
    return rng.standard_normal((B, D)), rng.standard_normal((B, O))


def test_bf16_matches_torch_conversion():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.standard_normal(5000).astype(np.float32) * 10.0 ** rng.integers(-8, 8, 5000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, -2.5], np.float32)])
    # exact ties: float32 values halfway between two bfloat16 values
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    a = np.concatenate([a, ties, -ties])
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(a), want)


def test_gradient_matches_finite_differences():
    theta = mlp.bf16(params(1))
    x, t = data(1)
    g = mlp.grad_at(theta, x, t, D, H, O)
    eps = 1e-6
    for k in range(len(theta)):
        e = np.zeros_like(theta)
        e[k] = eps
        fd = (mlp.loss_at(theta + e, x, t, D, H, O) - mlp.loss_at(theta - e, x, t, D, H, O)) / (2 * eps)
        assert abs(fd - g[k]) < 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_grad_uses_bf16_values():
    theta = params(2)
    x, t = data(2)
    assert np.allclose(mlp.grad(theta, x, t, D, H, O), mlp.grad_at(mlp.bf16(theta), x, t, D, H, O))
    assert mlp.loss(theta, x, t, D, H, O) == pytest.approx(mlp.loss_at(mlp.bf16(theta), x, t, D, H, O))


def test_dead_hidden_layer_closed_form():
    # W1 = 0, b1 = 0: h = 0, y = b2; only b2 has a gradient, mean(b2 - t)
    theta = params(3)
    W1, b1, W2, b2 = mlp.unpack(theta, D, H, O)
    W1[:] = 0
    b1[:] = 0
    x, t = data(3)
    g = mlp.grad(theta, x, t, D, H, O)
    gW1, gb1, gW2, gb2 = mlp.unpack(g, D, H, O)
    assert not gW1.any() and not gb1.any() and not gW2.any()
    assert np.allclose(gb2, (mlp.bf16(b2)[None, :] - t).mean(axis=0))
    y, _ = mlp.forward(theta, x, D, H, O)
    assert np.allclose(y, np.broadcast_to(mlp.bf16(b2), y.shape))


def test_linear_regime_closed_form():
    # every pre-activation positive: the network is the linear map
    # x (W1 W2) + (b1 W2 + b2)
    theta = params(4, 0.1)
    W1, b1, W2, b2 = mlp.unpack(theta, D, H, O)
    b1[:] = 50.0
    x, _ = data(4)
    y, z = mlp.forward(theta, x, D, H, O)
    assert (z > 0).all()
    Wq, bq, W2q, b2q = mlp.unpack(mlp.bf16(theta), D, H, O)
    assert np.allclose(y, x @ (Wq @ W2q) + (bq @ W2q + b2q))


def test_adam_first_step_is_sign_step():
    # bias-corrected m/sqrt(v) equals g/|g| at step 1
    theta = mlp.bf16(params(5)).astype(np.float32)
    x, t = data(5)
    g = mlp.grad(theta, x, t, D, H, O)
    lr = 1e-3
    p1 = mlp.adam(theta, x, t, D, H, O, 1, lr, eps=0.0)
    want = (theta.astype(np.float64) - lr * np.sign(g)).astype(np.float32)
    assert np.array_equal(p1.astype(np.float32), want)


def test_adam_reduces_loss():
    theta = params(6, 0.3)
    x, t = data(6, B=40)
    before = mlp.loss(theta, x, t, D, H, O)
    after = mlp.loss(mlp.adam(theta, x, t, D, H, O, 200, 1e-2), x, t, D, H, O)
    assert after < 0.5 * before
