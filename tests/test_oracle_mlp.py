"""Pins of the FP64 reference for the learned Newton guess (oracle/mlp.py)."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_matches_normal_distribution_table():
    # Phi(1) = 0.8413447460685429, Phi(2) = 0.9772498680518208 (standard normal table)
    x = np.array([-2.0, -1.0, 0.0, 1.0, 2.0])
    phi = np.array([1 - 0.9772498680518208, 1 - 0.8413447460685429, 0.5, 0.8413447460685429,
                    0.9772498680518208])
    assert np.allclose(mlp.gelu(x), x * phi, rtol=1e-15, atol=1e-16)


def test_gelu_derivative_by_finite_differences():
    x = np.linspace(-4, 4, 81)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_prime(x))) < 1e-9
    assert mlp.gelu_prime(np.array([0.0]))[0] == 0.5


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_by_central_finite_differences(seed):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.3, mlp.N_PARAM)
    X = rng.normal(size=(7, mlp.N_IN))
    t = rng.normal(size=7)
    L, g = mlp.loss_and_grad(theta, X, t)
    assert abs(L - mlp.loss(theta, X, t)) == 0.0
    # coordinates from every block: W1, b1, W2, b2, W3, b3
    blocks = [(0, 320), (320, 384), (384, 4480), (4480, 4544), (4544, 4608), (4608, 4609)]
    idx = np.concatenate([rng.choice(np.arange(a, b), min(6, b - a), replace=False) for a, b in blocks])
    h = 1e-5
    for i in idx:
        e = np.zeros(mlp.N_PARAM)
        e[i] = h
        fd = (mlp.loss(theta + e, X, t) - mlp.loss(theta - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_rounding_bit_patterns():
    f32 = lambda u: np.array([u], dtype=np.uint32).view(np.float32)[0]
    cases = [
        (0x3F800000, 0x3F800000),   # 1.0 exact
        (0x3F808000, 0x3F800000),   # 1 + 2^-8: halfway, ties to even (down)
        (0x3F818000, 0x3F820000),   # 1 + 3*2^-8: halfway, ties to even (up)
        (0x3F808001, 0x3F810000),   # just above halfway: up
        (0x3F807FFF, 0x3F800000),   # just below halfway: down
        (0xBF818000, 0xBF820000),   # negative, symmetric
        (0x477FFFFF, 0x47800000),   # carry into the exponent
    ]
    for u, r in cases:
        assert mlp.bf16_round(np.array([f32(u)]))[0] == float(f32(r)), hex(u)
    assert np.isnan(mlp.bf16_round(np.array([np.nan], dtype=np.float32))[0])


def test_adam_first_step_and_quadratic():
    # first step from zero moments moves each coordinate by lr * g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3])
    th, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    assert np.allclose(th, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # minimises 0.5 |theta - c|^2
    c = np.array([1.0, -2.0, 0.5])
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for k in range(1, 3001):
        th, m, v = mlp.adam_step(th, th - c, m, v, k, lr=0.01)
    assert np.max(np.abs(th - c)) < 1e-3


def test_judge_on_the_quartic():
    # alpha T^4 + T - s with alpha = 1, s = 2 has the root T = 1
    assert mlp.judge(np.array([1.0]), 1.0, 2.0, 1e-10)[0]
    assert not mlp.judge(np.array([1.0 + 1e-8]), 1.0, 2.0, 1e-10)[0]
    # alpha = 0: the root is s
    assert mlp.judge(np.array([0.25]), 0.0, 0.25, 0.0)[0]


def test_training_lowers_the_loss_on_a_smooth_target():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(256, mlp.N_IN))
    t = np.tanh(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]
    theta = rng.normal(0, 1.0, mlp.N_PARAM) * np.concatenate(
        [np.full(320, 1 / math.sqrt(5)), np.zeros(64), np.full(4096, 1 / 8), np.zeros(64), np.full(64, 1 / 8),
         [0.0]])
    L0 = mlp.loss(theta, X, t)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    for k in range(1, 301):
        _, g = mlp.loss_and_grad(theta, X, t)
        theta, m, v = mlp.adam_step(theta, g, m, v, k, lr=3e-3)
    assert mlp.loss(theta, X, t) < 0.2 * L0
