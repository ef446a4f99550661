"""Float64 reference of the partition router's network (test infrastructure only).

The router is a small multilayer perceptron d -> H -> H -> P with ReLU
activations and a softmax over P coarse partitions, trained with the
cross-entropy against a soft target: each training cell's target puts
weight 1/m on the partition of each of its m exact nearest neighbours
(repeats add up).  Everything here is plain numpy in float64: forward,
loss, backward by the chain rule written out layer by layer, and an Adam
step.  Weights are stored like the GPU's: W[l] has shape (fan_out, fan_in).

Only tests (and the smoke check) use this module.
"""

from __future__ import annotations

import numpy as np


def init_params(d: int, hidden: int, parts: int, seed: int = 0):
    """Seeded uniform(+-sqrt(6 / (fan_in + fan_out))) weights, zero biases."""
    rng = np.random.default_rng(seed)
    shapes = [(hidden, d), (hidden, hidden), (parts, hidden)]
    params = []
    for fo, fi in shapes:
        lim = np.sqrt(6.0 / (fi + fo))
        params.append(rng.uniform(-lim, lim, size=(fo, fi)))
        params.append(np.zeros(fo))
    return params


def soft_targets(label_parts: np.ndarray, parts: int) -> np.ndarray:
    """Dense targets: row i has weight 1/m on each listed partition."""
    n, m = label_parts.shape
    t = np.zeros((n, parts))
    for j in range(m):
        np.add.at(t, (np.arange(n), label_parts[:, j]), 1.0 / m)
    return t


def forward(params, X):
    """Returns the activations needed by the backward pass and the logits."""
    W1, b1, W2, b2, W3, b3 = params
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return (X, a1, h1, a2, h2), z


def log_softmax(z):
    zmax = z.max(axis=1, keepdims=True)
    lse = zmax + np.log(np.exp(z - zmax).sum(axis=1, keepdims=True))
    return z - lse


def loss(params, X, targets):
    """Mean over rows of -sum_p t_p log softmax(z)_p."""
    _, z = forward(params, X)
    return float(-(targets * log_softmax(z)).sum(axis=1).mean())


def backward(params, X, targets):
    """Gradients of ``loss`` with respect to (W1, b1, W2, b2, W3, b3)."""
    W1, b1, W2, b2, W3, b3 = params
    (x, a1, h1, a2, h2), z = forward(params, X)
    n = X.shape[0]
    p = np.exp(log_softmax(z))
    dz = (p - targets) / n                  # d loss / d z
    dW3 = dz.T @ h2
    db3 = dz.sum(axis=0)
    dh2 = dz @ W3
    da2 = dh2 * (a2 > 0)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (a1 > 0)
    dW1 = da1.T @ x
    db1 = da1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3]


def adam_step(params, grads, state, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); ``state`` is a list of (m, v) pairs."""
    out = []
    for i, (w, g) in enumerate(zip(params, grads)):
        m, v = state[i]
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        state[i] = (m, v)
        mhat = m / (1 - beta1 ** step)
        vhat = v / (1 - beta2 ** step)
        out.append(w - lr * mhat / (np.sqrt(vhat) + eps))
    return out


def top_partitions(params, X, probes: int):
    """Top-``probes`` partitions per row (descending probability, lower index
    on ties) and the softmax mass they hold."""
    _, z = forward(params, X)
    p = np.exp(log_softmax(z))
    order = np.lexsort((np.broadcast_to(np.arange(z.shape[1]), z.shape), -z), axis=1)[:, :probes]
    mass = np.take_along_axis(p, order, axis=1).sum(axis=1)
    return order, mass


def bf16_round(x):
    """Round to the nearest bfloat16 value (ties to even), returned in float64.

    bfloat16 keeps the float32 sign, exponent and top 7 mantissa bits; the
    float32 value is rounded first (round to nearest even), then the low 16
    bits with ties to even.
    """
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    lsb = (u >> 16) & 1
    r = np.where(finite, (u + 0x7FFF + lsb) >> 16, u >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(params, X, rounding=True):
    """Forward pass with the roundings of the BF16 matrix-core kernels:
    inputs, weights and hidden activations rounded to bfloat16, biases and
    logits kept exact.  ``rounding=False`` makes it ``forward``."""
    rnd = bf16_round if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = params
    x = rnd(X)
    h1 = rnd(np.maximum(x @ rnd(W1).T + b1, 0.0))
    h2 = rnd(np.maximum(h1 @ rnd(W2).T + b2, 0.0))
    z = h2 @ rnd(W3).T + b3
    return (x, h1, h2), z


def backward_bf16(params, X, targets, rounding=True):
    """Gradients with the roundings of the BF16 kernels: the output error
    (softmax - target) / n and the back-propagated hidden errors are rounded
    to bfloat16 before they enter the next product; weight gradients are
    exact sums of those rounded factors.  ``rounding=False`` gives
    ``backward``."""
    rnd = bf16_round if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = params
    (x, h1, h2), z = forward_bf16(params, X, rounding)
    n = X.shape[0]
    dz = rnd((np.exp(log_softmax(z)) - targets) / n)
    dW3 = dz.T @ h2
    db3 = dz.sum(axis=0)
    dh2 = rnd((dz @ rnd(W3)) * (h2 > 0))
    dW2 = dh2.T @ h1
    db2 = dh2.sum(axis=0)
    dh1 = rnd((dh2 @ rnd(W2)) * (h1 > 0))
    dW1 = dh1.T @ x
    db1 = dh1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3]
