"""FP64 reference of the learned Newton initial guess (test infrastructure).

A small multilayer perceptron maps local state to a starting value for the
scalar temperature equation (4.13)/(5.5), which Newton then polishes:

  features   f = log10 of (rho*, T^n, sigma0 (T^n)^-m, eps, dt)   (5 inputs)
  normalise  x = (f - mu_f) / sd_f
  network    z1 = W1 x + b1,  h1 = gelu(z1)     (64)
             z2 = W2 h1 + b2, h2 = gelu(z2)     (64)
             y  = W3 . h2 + b3                  (1)
  output     T0 = T^n exp(mu_t + sd_t y)        (y predicts log(T^{n+1}/T^n))
  gelu(x)    = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2   (exact form)
  loss       mean over the batch of (y - (log(T^{n+1}/T^n) - mu_t) / sd_t)^2
  optimiser  Adam (Kingma & Ba 2015) with bias correction.

Inference uses the weights rounded to bfloat16 (round to nearest even) and
accumulates in a wider type; `bf16_round` gives the rounded values so that
the FP64 reference can evaluate exactly the network the GPU evaluates.

The parameter vector is flat: W1 (64x5, row-major: W1[i, f] at 5 i + f),
b1 (64), W2 (64x64, W2[i, j] at 64 i + j, i the output unit), b2 (64),
W3 (64), b3 (1): 4609 values.  The normalisation vector holds
mu_f (5), sd_f (5), mu_t, sd_t: 12 values.

Pins (tests/test_oracle_mlp.py): the backward pass against central finite
differences of the forward pass, gelu against tabulated values of the normal
distribution, bf16 rounding against hand-worked bit patterns, Adam against
its closed form on a quadratic, and the Newton judge against the textbook
properties of the quartic.
"""
import math

import numpy as np
from scipy.special import erf

N_IN = 5
N_HID = 64
N_PARAM = N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_HID + 1
N_NORM = 2 * N_IN + 2


def features(rho_star, Tn, sigma0, m, eps, dt):
    """log10 of the five inputs, float64 (the GPU rounds these to binary32)."""
    rho_star = np.asarray(rho_star, dtype=np.float64)
    Tn = np.asarray(Tn, dtype=np.float64)
    sigma_eff = np.asarray(sigma0, dtype=np.float64) * Tn ** (-m)
    n = rho_star.size
    F = np.empty((n, N_IN))
    F[:, 0] = np.log10(np.maximum(np.abs(rho_star), 1e-300))
    F[:, 1] = np.log10(Tn)
    F[:, 2] = np.log10(sigma_eff)
    F[:, 3] = np.log10(np.full(n, eps))
    F[:, 4] = np.log10(np.full(n, dt))
    return F


def target(Tn, Tnew):
    """Training target: log(T^{n+1} / T^n)."""
    return np.log(np.asarray(Tnew, dtype=np.float64) / np.asarray(Tn, dtype=np.float64))


def unpack(theta):
    th = np.asarray(theta, dtype=np.float64)
    assert th.size == N_PARAM
    o = 0
    W1 = th[o:o + N_HID * N_IN].reshape(N_HID, N_IN); o += N_HID * N_IN
    b1 = th[o:o + N_HID]; o += N_HID
    W2 = th[o:o + N_HID * N_HID].reshape(N_HID, N_HID); o += N_HID * N_HID
    b2 = th[o:o + N_HID]; o += N_HID
    W3 = th[o:o + N_HID]; o += N_HID
    b3 = th[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, W3, [b3]]).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_prime(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def normalise(F, norm):
    norm = np.asarray(norm, dtype=np.float64)
    return (np.asarray(F, dtype=np.float64) - norm[:N_IN]) / norm[N_IN:2 * N_IN]


def forward(theta, X):
    """Network output y for normalised inputs X (n x 5), and the cache of the
    intermediate values used by the backward pass."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    y = h2 @ W3 + b3
    return y, (X, z1, h1, z2, h2)


def loss(theta, X, t):
    y, _ = forward(theta, X)
    return float(np.mean((y - t) ** 2))


def loss_and_grad(theta, X, t):
    """Mean squared error and its gradient with respect to every parameter
    (chain rule through the two gelu layers)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (X, z1, h1, z2, h2) = forward(theta, X)
    n = y.size
    dy = 2.0 * (y - t) / n                      # dL/dy
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    dz2 = np.outer(dy, W3) * gelu_prime(z2)     # dL/dz2
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_prime(z1)           # dL/dz1
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return float(np.mean((y - t) ** 2)), pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(theta, grad, m, v, k, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number k >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** k)
    vhat = v / (1.0 - beta2 ** k)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def bf16_round(x):
    """Round binary32 values to bfloat16 (round to nearest, ties to even);
    returned as float64 holding the exact bfloat16 values."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out


def predict_guess(theta_bf16, norm, F, Tn):
    """T0 from the network whose parameters are the given (bfloat16-valued)
    numbers; FP64 arithmetic."""
    norm = np.asarray(norm, dtype=np.float64)
    y, _ = forward(theta_bf16, normalise(F, norm))
    return np.asarray(Tn, dtype=np.float64) * np.exp(norm[2 * N_IN] + norm[2 * N_IN + 1] * y)


def judge(T0, alpha, s, tol):
    """Accept a starting value for alpha T^4 + T - s = 0 outright when its
    normalised residual is at most tol (the caller then skips Newton)."""
    res = alpha * T0 ** 4 + T0 - s
    return np.abs(res) <= tol * np.maximum(np.abs(s), 1e-300)
