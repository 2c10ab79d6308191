"""Plain FP64 CPU oracle of the warm-start perceptron.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
kernels.

Why a network at all: Algorithm 1 (Section 2) starts from an initial guess of
the coefficients and Section 3's step works from any starting residual, so a
guess that is already close to the answer saves sweeps.  For a parametric
family of systems the guess is predicted from the family parameters p by a
multilayer perceptron.  The paper defines no network; this one is:

    z1 = W1 x + b1,  h1 = gelu(z1)
    z2 = W2 h1 + b2, h2 = gelu(z2)
    o  = W3 h2 + b3
    gelu(z) = z * Phi(z) = 0.5 z (1 + erf(z / sqrt 2))   (exact, not tanh)
    L = sum_{b,k} (o_bk - t_bk)^2 / (batch * n_out)        (mean squared error)

trained by Adam (Kingma and Ba, "Adam: a method for stochastic
optimization", 2015, Algorithm 1; beta1 0.9, beta2 0.999, eps 1e-8, with both
bias corrections).

Parameter vector, the same flat layout the library uses: W1[h1][in], b1[h1],
W2[h2][h1], b2[h2], W3[out][h2], b3[out]; row o of a weight matrix holds the
weights into output unit o.  Inputs x are rows [batch][in].

Output scaling (standardised targets): mu_k and sd_k are the mean and the
sample standard deviation of output k over the training targets; the
network is trained on (t - mu)/sd and answers sd * o + mu.

Initial parameters: parameter k of the flat vector is value k of the
SplitMix64 stream started at the seed (Steele, Lea and Flood, 2014),
u = top 53 bits / 2^53, w = (2u - 1) * (1 / sqrt(fan_in)) of its layer,
rounded to FP32.

Gradients are the chain rule written out (backpropagation):
    dL/do  = 2 (o - t) / (batch * n_out)
    dW3 = dO^T h2, db3 = sum_b dO, dH2 = dO W3
    dZ2 = dH2 * gelu'(z2), gelu'(z) = Phi(z) + z phi(z)
    dW2 = dZ2^T h1, db2 = sum_b dZ2, dH1 = dZ2 W2, dZ1 = dH1 * gelu'(z1)
    dW1 = dZ1^T x, db1 = sum_b dZ1.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

__all__ = ["num_params", "unpack", "gelu", "gelu_prime", "forward", "loss", "grads", "adam_step",
           "output_scaling", "forward_scaled", "grads_scaled", "splitmix64", "init_params"]


def num_params(shape) -> int:
    n_in, h1, h2, n_out = shape
    return h1 * n_in + h1 + h2 * h1 + h2 + n_out * h2 + n_out


def unpack(flat, shape):
    """Views (W1, b1, W2, b2, W3, b3) into the flat FP64 parameter vector."""
    n_in, h1, h2, n_out = shape
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.shape == (num_params(shape),)
    out, o = [], 0
    for rows, cols in ((h1, n_in), (h2, h1), (n_out, h2)):
        out.append(flat[o: o + rows * cols].reshape(rows, cols))
        o += rows * cols
        out.append(flat[o: o + rows])
        o += rows
    return tuple(out)


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    z = np.asarray(z, dtype=np.float64)
    cdf = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def forward(flat, shape, x, cache=False):
    """Network output o (batch, n_out); with ``cache`` also (z1, h1, z2, h2)."""
    W1, b1, W2, b2, W3, b3 = unpack(flat, shape)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    o = h2 @ W3.T + b3
    return (o, (z1, h1, z2, h2)) if cache else o


def loss(o, t):
    o = np.asarray(o, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    return float(np.sum((o - t) ** 2) / o.size)


def grads(flat, shape, x, t):
    """(dL/dflat in the flat layout, L) at the given parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(flat, shape)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    o, (z1, h1, z2, h2) = forward(flat, shape, x, cache=True)
    dO = 2.0 * (o - t) / o.size
    dW3 = dO.T @ h2
    db3 = dO.sum(axis=0)
    dZ2 = (dO @ W3) * gelu_prime(z2)
    dW2 = dZ2.T @ h1
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * gelu_prime(z1)
    dW1 = dZ1.T @ x
    db1 = dZ1.sum(axis=0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])
    return g, loss(o, t)


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step number ``step`` (1-based); returns (p, m, v)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def output_scaling(T):
    """(mu, sd): per-column mean and sample standard deviation of T (rows are
    samples), sd at least 1e-12 and 1 for a single row."""
    T = np.asarray(T, dtype=np.float64)
    mu = T.mean(axis=0)
    sd = T.std(axis=0, ddof=1) if T.shape[0] > 1 else np.ones(T.shape[1])
    return mu, np.maximum(sd, 1e-12)


def forward_scaled(flat, shape, x, mu, sd):
    """sd * o + mu: the network's answer in target units."""
    return np.asarray(sd, np.float64) * forward(flat, shape, x) + np.asarray(mu, np.float64)


def grads_scaled(flat, shape, x, t, mu, sd):
    """Gradient and loss of the network trained on standardised targets."""
    t = (np.asarray(t, np.float64) - np.asarray(mu, np.float64)) / np.asarray(sd, np.float64)
    return grads(flat, shape, x, t)


_M64 = (1 << 64) - 1


def splitmix64(seed, k):
    """Value k (0-based) of the SplitMix64 stream started at ``seed``: state
    seed + (k+1)·0x9E3779B97F4A7C15, then the finaliser (xor-shift 30,
    multiply 0xBF58476D1CE4E5B9, xor-shift 27, multiply 0x94D049BB133111EB,
    xor-shift 31), all modulo 2^64.  k may be an integer array."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + (k + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def init_params(shape, seed):
    """Initial flat parameter vector (FP64 values of the FP32 the library stores)."""
    n_in, h1, h2, n_out = shape
    out, k0 = [], 0
    for fan, rows in ((n_in, h1), (h1, h2), (h2, n_out)):
        cnt = rows * fan + rows
        u = (splitmix64(seed, np.arange(k0, k0 + cnt)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        bound = 1.0 / math.sqrt(fan)
        out.append(((2.0 * u - 1.0) * bound).astype(np.float32).astype(np.float64))
        k0 += cnt
    return np.concatenate(out)
