"""Per-element bounds on the device screening network against the oracle's BF16 forms.

The device computes the network with BF16 matrix-product operands and FP32 everywhere else. The oracle's
forward_bf16 / backward_bf16 round to bfloat16 at the same points and compute everything else in FP64, so the
two differ only by
  - FP32 arithmetic: a sum of K terms in FP32 is within (K + 2) 2^-24 of the exact sum of their magnitudes
    (products of two bf16 values are exact in the FP32 accumulator; the +2 covers a bias add and the final
    rounding), and an elementwise FP32 step carries a few units of 2^-24 of its value;
  - rounding to bfloat16 of a value that the two sides hold slightly differently: when the oracle's value v
    and every value within the bound E of it round to the same bfloat16 number, both sides round to that
    number exactly; otherwise the device may take the neighbouring one, at most one bfloat16 step (2^-7 of
    the magnitude) away;
  - ReLU masks: where the oracle's pre-activation lies within its bound of zero the device may take the other
    branch. A forward ReLU is 1-Lipschitz (no extra error); in the backward pass the masked gradient may then
    be missing or present entirely, so its bound is its full magnitude there;
  - the logistic function, whose slope over [z - E, z + E] is at most its slope at the point of that interval
    nearest 0.
The helpers propagate these absolute bounds layer by layer from the oracle's FP64 intermediates. A final factor
`safety` (1.25) covers the products of bounds (second-order terms) that the first-order terms leave out.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp_oracle as mo

U32 = 2.0 ** -24
BF16_STEP = 2.0 ** -7  # distance between neighbouring bfloat16 values, relative to the magnitude


def _acc(K):
    """FP32 summation bound over K terms, relative to the sum of their magnitudes."""
    return (K + 2) * U32


def _rounded(v, E, lo=None, hi=None):
    """Bound on |bf16(v_device) - bf16(v)| for v_device in [lo, hi] (default v -+ E): zero where the whole
    interval rounds to one bfloat16 number, one bfloat16 step of the interval's largest magnitude otherwise."""
    lo = v - E if lo is None else lo
    hi = v + E if hi is None else hi
    same = mo.bf16_round(lo) == mo.bf16_round(hi)
    return np.where(same, 0.0, BF16_STEP * (np.abs(v) + E) + E)


def _sigmoid_slope_max(z, E):
    near = np.where(np.abs(z) <= E, 0.0, np.abs(z) - E)
    s = 1.0 / (1.0 + np.exp(-near))
    return s * (1.0 - s)


def forward_bounds(params, cache, z, E_params=None):
    """Bounds on the device's logits and the intermediates the backward bounds need, for one batch.

    params: FP64 [W1, b1, W2, b2, w3, b3]; cache, z: oracle.forward_bf16 on the same rows. E_params (same
    shapes, default zeros) bounds how far the device's own parameters may lie from params (after optimiser
    steps taken separately on the two sides)."""
    W1, b1, W2, b2, w3, b3 = params
    eW1, eb1, eW2, eb2, ew3, eb3 = E_params if E_params is not None else [np.zeros_like(p) for p in params]
    xs, xq, a1, h1q, a2, h2 = cache
    W1q, W2q = mo.bf16_round(W1), mo.bf16_round(W2)
    E_W1q, E_W2q = _rounded(W1, eW1), _rounded(W2, eW2)
    d, H = W1.shape
    # standardisation in FP32: a subtraction and a division
    E_xs = 3 * U32 * np.abs(xs)
    E_xq = _rounded(xs, E_xs)
    aW1q, aW2q = np.abs(W1q) + E_W1q, np.abs(W2q) + E_W2q
    E_a1 = (E_xq @ aW1q + np.abs(xq) @ E_W1q + eb1
            + _acc(d) * ((np.abs(xq) + E_xq) @ aW1q + np.abs(b1) + eb1))
    # the device's ReLU output lies in [relu(a1 - E), relu(a1 + E)]
    E_h1q = _rounded(np.maximum(a1, 0.0), E_a1, np.maximum(a1 - E_a1, 0.0), np.maximum(a1 + E_a1, 0.0))
    E_a2 = (E_h1q @ aW2q + np.abs(h1q) @ E_W2q + eb2
            + _acc(H) * ((np.abs(h1q) + E_h1q) @ aW2q + np.abs(b2) + eb2))
    E_h2 = E_a2
    # the head sums four partial dot products of 64 columns, then adds b3
    aw3 = np.abs(w3) + ew3
    E_z = (E_h2 @ aw3 + np.abs(h2) @ ew3 + float(eb3)
           + _acc(H + 4) * ((np.abs(h2) + E_h2) @ aw3 + abs(float(b3)) + float(eb3)))
    return dict(E_xq=E_xq, E_a1=E_a1, E_h1q=E_h1q, E_a2=E_a2, E_h2=E_h2, E_z=E_z, W2q=W2q, E_W2q=E_W2q,
                E_w3=ew3)


def gradient_bounds(params, cache, z, y, fb, splits=64, safety=1.25):
    """Bounds on the device's six gradients of the mean BCE (the order of oracle.backward_bf16)."""
    W1, b1, W2, b2, w3, b3 = params
    xs, xq, a1, h1q, a2, h2 = cache
    E_xq, E_a1, E_h1q, E_a2, E_h2, E_z = (fb[k] for k in ("E_xq", "E_a1", "E_h1q", "E_a2", "E_h2", "E_z"))
    E_W2q, E_w3 = fb["E_W2q"], fb["E_w3"]
    aW2q = np.abs(fb["W2q"]) + E_W2q
    aw3 = np.abs(w3) + E_w3
    B = z.shape[0]
    H = W2.shape[0]
    t = (np.asarray(y, np.float64) + 1.0) * 0.5
    dz = (1.0 / (1.0 + np.exp(-z)) - t) / B
    adz = np.abs(dz)
    # FP32 exp, add, reciprocal-division and subtraction: a few units of 2^-24 of sigmoid (<= 1)
    E_dz = (_sigmoid_slope_max(z, E_z) * E_z + 8 * U32) / B + 2 * U32 * adz
    ah2 = np.abs(h2)
    KB = B + splits  # the column sums add their 64 chunk partials in a second pass
    E_gw3 = E_h2.T @ adz + (ah2 + E_h2).T @ E_dz + _acc(KB) * ((ah2 + E_h2).T @ (adz + E_dz))
    E_gb3 = np.sum(E_dz) + _acc(KB) * np.sum(adz + E_dz)
    # layer 2: dZ2 = [a2 > 0] dz w3 in FP32, then rounded to bf16 for both products
    dZ2 = (a2 > 0) * np.outer(dz, w3)
    adZ2 = np.abs(dZ2)
    sure2 = np.abs(a2) > E_a2
    # a certainly inactive unit gives exactly 0 on both sides
    E_dZ2 = np.where(sure2, (a2 > 0) * (np.outer(E_dz, aw3) + np.outer(adz, E_w3) + U32 * adZ2),
                     np.outer(adz + E_dz, aw3))
    dZ2q = mo.bf16_round(dZ2)
    E_dZ2q = np.where(sure2, _rounded(dZ2, E_dZ2), (1 + BF16_STEP) * (adZ2 + E_dZ2))
    adZ2q = np.abs(dZ2q)
    ah1q = np.abs(h1q)
    E_gW2 = E_h1q.T @ adZ2q + (ah1q + E_h1q).T @ E_dZ2q + _acc(KB) * ((ah1q + E_h1q).T @ (adZ2q + E_dZ2q))
    E_gb2 = np.sum(E_dZ2, axis=0) + _acc(KB) * np.sum(adZ2 + E_dZ2, axis=0)
    # layer 1: dH1 = dZ2q W2q^T (FP32), dZ1 = [a1 > 0] dH1, rounded to bf16 for the weight gradient
    dH1 = dZ2q @ fb["W2q"].T
    adH1 = np.abs(dH1)
    E_dH1 = E_dZ2q @ aW2q.T + adZ2q @ E_W2q.T + _acc(H) * ((adZ2q + E_dZ2q) @ aW2q.T)
    sure1 = np.abs(a1) > E_a1
    dZ1 = (a1 > 0) * dH1
    adZ1 = np.abs(dZ1)
    E_dZ1 = np.where(sure1, (a1 > 0) * E_dH1, adH1 + E_dH1)
    dZ1q = mo.bf16_round(dZ1)
    E_dZ1q = np.where(sure1, _rounded(dZ1, E_dZ1), (1 + BF16_STEP) * (adZ1 + E_dZ1))
    adZ1q = np.abs(dZ1q)
    axq = np.abs(xq)
    E_gW1 = E_xq.T @ adZ1q + (axq + E_xq).T @ E_dZ1q + _acc(KB) * ((axq + E_xq).T @ (adZ1q + E_dZ1q))
    E_gb1 = np.sum(E_dZ1, axis=0) + _acc(KB) * np.sum(adZ1 + E_dZ1, axis=0)
    out = [E_gW1, E_gb1, E_gW2, E_gb2, E_gw3, np.array(E_gb3)]
    info = dict(uncertain_relu1=int(np.sum(~sure1)), uncertain_relu2=int(np.sum(~sure2)),
                bf16_ties_h1=int(np.sum(E_h1q > 0)), bf16_ties_dZ2=int(np.sum(E_dZ2q > 0)),
                bf16_ties_dZ1=int(np.sum(E_dZ1q > 0)))
    return [safety * e for e in out], info


def adam_direction_bound(g_ref, E_g, eps=1e-8):
    """Largest change of s(g) = g / (|g| + eps) -- the first Adam step's direction, since then
    m_hat = g and v_hat = g^2 -- over every g within E_g of g_ref (s is increasing, so the ends of the
    interval decide)."""
    s = lambda x: x / (np.abs(x) + eps)
    s0 = s(g_ref)
    return np.maximum(np.abs(s(g_ref + E_g) - s0), np.abs(s(g_ref - E_g) - s0))


def adam_ratio_cap(t, beta1, beta2):
    """Largest |m_hat / sqrt(v_hat)| that any gradient sequence can give at step t (Cauchy-Schwarz on
    m_t = (1 - b1) sum_j b1^j g_(t-j) against v_t = (1 - b2) sum_j b2^j g_(t-j)^2)."""
    r = sum((beta1 * beta1 / beta2) ** j for j in range(t))
    return (1 - beta1) / (1 - beta1 ** t) / np.sqrt((1 - beta2) / (1 - beta2 ** t)) * np.sqrt(r)


def adam_ratio_bound(mh, Emh, vh, Evh, eps=1e-8, cap=np.inf):
    """Largest change of m_hat / (sqrt(v_hat) + eps) over m_hat within Emh of mh and v_hat >= 0 within Evh of
    vh (monotone in each argument, so the four corners decide), and never more than 2 cap when both ratios
    are at most cap in magnitude."""
    r0 = mh / (np.sqrt(vh) + eps)
    worst = np.zeros_like(r0)
    for m_ in (mh - Emh, mh + Emh):
        for v_ in (np.maximum(vh - Evh, 0.0), vh + Evh):
            worst = np.maximum(worst, np.abs(m_ / (np.sqrt(v_) + eps) - r0))
    return np.minimum(worst, 2 * cap)
