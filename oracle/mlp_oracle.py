"""FP64 NumPy oracle for the learned screening network.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). The screening network is
not part of the paper's method; it is the learned pre-screen that runs on the
FK control points (the paper cites a network on control points as prior art
for fast collision-cost estimates, Section I-B). The GPU library computes the
same network with its own BF16 kernels; this module gives the float64
reference for the forward pass, the backward pass and the optimiser step.

Network: x (B, 3M) control points -> standardise -> Linear(3M, H1) -> ReLU ->
Linear(H1, H2) -> ReLU -> Linear(H2, 1) -> logit z.
Loss: binary cross-entropy on logits, target t = (y + 1) / 2, averaged over B.
Optimiser: Adam (Kingma & Ba 2015) with bias correction.

The screening network's precision is BF16 operands with FP32 accumulation:
the standardised inputs, the weight matrices and the activations or
gradients that enter a matrix product are bfloat16 values. ``forward_bf16``
and ``backward_bf16`` are the same computation with those values rounded to
the nearest bfloat16 at exactly those points (everything else FP64), so that
a comparison with an implementation of that precision is left with its FP32
accumulation error only. With ``rnd`` the identity they are ``forward`` and
``backward`` step for step.
"""
from __future__ import annotations

import numpy as np


def standardise(x, mu, sd):
    return (np.asarray(x, np.float64) - mu) / sd


def forward(params, x, mu, sd):
    """Returns logits z (B,) and the cache needed by ``backward``."""
    W1, b1, W2, b2, w3, b3 = (np.asarray(p, np.float64) for p in params)
    xs = standardise(x, mu, sd)
    a1 = xs @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    return z, (xs, a1, h1, a2, h2)


def bce_loss(z, y):
    """Mean over the batch of softplus(z) - t z, with t = (y + 1) / 2."""
    t = (np.asarray(y, np.float64) + 1.0) * 0.5
    z = np.asarray(z, np.float64)
    softplus = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))
    return float(np.mean(softplus - t * z))


def backward(params, cache, z, y):
    """Gradients of ``bce_loss`` w.r.t. (W1, b1, W2, b2, w3, b3)."""
    W1, b1, W2, b2, w3, b3 = (np.asarray(p, np.float64) for p in params)
    xs, a1, h1, a2, h2 = cache
    B = z.shape[0]
    t = (np.asarray(y, np.float64) + 1.0) * 0.5
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = (sig - t) / B
    gw3 = h2.T @ dz
    gb3 = np.array(np.sum(dz))
    dh2 = np.outer(dz, w3)
    da2 = dh2 * (a2 > 0.0)
    gW2 = h1.T @ da2
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2.T
    da1 = dh1 * (a1 > 0.0)
    gW1 = xs.T @ da1
    gb1 = da1.sum(axis=0)
    return [gW1, gb1, gW2, gb2, gw3, gb3]


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1). Returns new params, m, v."""
    new_p, new_m, new_v = [], [], []
    for p, g, mi, vi in zip(params, grads, m, v):
        p = np.asarray(p, np.float64)
        g = np.asarray(g, np.float64)
        mi = beta1 * np.asarray(mi, np.float64) + (1.0 - beta1) * g
        vi = beta2 * np.asarray(vi, np.float64) + (1.0 - beta2) * g * g
        mhat = mi / (1.0 - beta1 ** step)
        vhat = vi / (1.0 - beta2 ** step)
        new_p.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        new_m.append(mi)
        new_v.append(vi)
    return new_p, new_m, new_v


def bf16_round(x):
    """Nearest bfloat16 value of x (8 significant bits, ties to the even significand), float64 in and out.
    bfloat16 keeps float32's exponent range; the values here stay far from its limits."""
    m, e = np.frexp(np.asarray(x, np.float64))  # x = m 2^e with 0.5 <= |m| < 1 (m = 0 for x = 0)
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)  # rint rounds halves to even


def forward_bf16(params, x, mu, sd, rnd=bf16_round):
    """``forward`` with the operands of both matrix products rounded by ``rnd``: the standardised inputs,
    W1, the layer-1 activations and W2. Returns z and the cache for ``backward_bf16``."""
    W1, b1, W2, b2, w3, b3 = (np.asarray(p, np.float64) for p in params)
    xs = standardise(x, mu, sd)
    xq = rnd(xs)
    a1 = xq @ rnd(W1) + b1
    h1q = rnd(np.maximum(a1, 0.0))
    a2 = h1q @ rnd(W2) + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    return z, (xs, xq, a1, h1q, a2, h2)


def backward_bf16(params, cache, z, y, rnd=bf16_round):
    """``backward`` with the operands of its matrix products rounded by ``rnd``: the layer-2 and layer-1
    pre-activation gradients (the bias gradients sum the unrounded values) and W2."""
    W1, b1, W2, b2, w3, b3 = (np.asarray(p, np.float64) for p in params)
    xs, xq, a1, h1q, a2, h2 = cache
    B = z.shape[0]
    t = (np.asarray(y, np.float64) + 1.0) * 0.5
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = (sig - t) / B
    gw3 = h2.T @ dz
    gb3 = np.array(np.sum(dz))
    da2 = np.outer(dz, w3) * (a2 > 0.0)
    da2q = rnd(da2)
    gW2 = h1q.T @ da2q
    gb2 = da2.sum(axis=0)
    dh1 = da2q @ rnd(W2).T
    da1 = dh1 * (a1 > 0.0)
    da1q = rnd(da1)
    gW1 = xq.T @ da1q
    gb1 = da1.sum(axis=0)
    return [gW1, gb1, gW2, gb2, gw3, gb3]
