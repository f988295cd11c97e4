"""Pins of the FP64 screening-network oracle: central finite differences for
the gradients and the closed form of Adam's first step."""
import numpy as np

from oracle import mlp_oracle as mo


def _params(g, d_in=6, h1=5, h2=4):
    return [g.standard_normal((d_in, h1)) * 0.5, g.standard_normal(h1) * 0.1, g.standard_normal((h1, h2)) * 0.5,
            g.standard_normal(h2) * 0.1, g.standard_normal(h2) * 0.5, np.array(0.05)]


def test_gradients_match_finite_differences():
    g = np.random.default_rng(0)
    params = _params(g)
    x = g.standard_normal((9, 6))
    y = np.where(g.random(9) < 0.5, 1, -1)
    mu, sd = x.mean(axis=0), x.std(axis=0) + 0.5

    def loss(ps):
        z, _ = mo.forward(ps, x, mu, sd)
        return mo.bce_loss(z, y)

    z, cache = mo.forward(params, x, mu, sd)
    grads = mo.backward(params, cache, z, y)
    h = 1e-6
    for k, p in enumerate(params):
        p = np.asarray(p, np.float64)
        num = np.zeros_like(p)
        it = np.nditer(p, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            plus = [np.array(q, copy=True) for q in params]
            minus = [np.array(q, copy=True) for q in params]
            plus[k][idx] += h
            minus[k][idx] -= h
            num[idx] = (loss(plus) - loss(minus)) / (2 * h)
        err = np.linalg.norm(num - grads[k]) / max(np.linalg.norm(num), 1e-12)
        assert err < 1e-6, (k, err)


def test_bce_closed_form():
    # z = 0: loss log 2 for either label; large positive z with label +1: ~0
    assert abs(mo.bce_loss(np.zeros(4), np.array([1, -1, 1, -1])) - np.log(2.0)) < 1e-15
    assert mo.bce_loss(np.array([40.0]), np.array([1])) < 1e-16


def test_adam_first_step_closed_form():
    """After one step from zero moments the bias-corrected ratio is g/|g|, so each weight moves by lr*sign(g)
    (up to eps)."""
    g = np.random.default_rng(1)
    p = [g.standard_normal((3, 2))]
    grad = [g.standard_normal((3, 2))]
    new, m, v = mo.adam_step(p, grad, [np.zeros((3, 2))], [np.zeros((3, 2))], step=1, lr=1e-2)
    np.testing.assert_allclose(new[0], p[0] - 1e-2 * np.sign(grad[0]), atol=1e-8)
    np.testing.assert_allclose(m[0], 0.1 * grad[0])
    np.testing.assert_allclose(v[0], 0.001 * grad[0] ** 2)


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        return json.load(fh)


def test_forward_tiny_network_by_hand():
    """Standardisation, both hidden layers and the head against a network worked by hand
    (golden/mlp_tiny_forward.json): every hidden unit is active in one sample and inactive in the other."""
    gd = _golden("mlp_tiny_forward.json")
    params = [np.array(gd[k], np.float64) for k in ("W1", "b1", "W2", "b2", "w3")] + [np.array(gd["b3"])]
    z, (xs, a1, h1, a2, h2) = mo.forward(params, np.array(gd["x"]), np.array(gd["mu"]), np.array(gd["sd"]))
    np.testing.assert_array_equal(xs, np.array(gd["xs"]))
    np.testing.assert_array_equal(a1, np.array(gd["a1"]))
    np.testing.assert_array_equal(a2, np.array(gd["a2"]))
    np.testing.assert_array_equal(h1, np.maximum(np.array(gd["a1"]), 0.0))
    np.testing.assert_array_equal(h2, np.maximum(np.array(gd["a2"]), 0.0))
    np.testing.assert_array_equal(z, np.array(gd["z"]))


def test_adam_three_steps_by_hand():
    """Three Adam steps with a varying gradient against exact fractions (golden/adam_three_steps.json):
    the moments, both bias corrections (1 - beta^t at t = 1, 2, 3) and the weight after each step."""
    from fractions import Fraction

    gd = _golden("adam_three_steps.json")
    p = [np.array([gd["p0"]])]
    m = [np.zeros(1)]
    v = [np.zeros(1)]
    for k, (g, st) in enumerate(zip(gd["grads"], gd["steps"])):
        p, m, v = mo.adam_step(p, [np.array([g])], m, v, step=st["t"], lr=gd["lr"], beta1=gd["beta1"],
                               beta2=gd["beta2"], eps=gd["eps"])
        assert abs(m[0][0] - float(Fraction(st["m"]))) <= 1e-15 * abs(float(Fraction(st["m"])))
        assert abs(v[0][0] - float(Fraction(st["v"]))) <= 1e-15 * abs(float(Fraction(st["v"])))
        assert abs(p[0][0] - gd["p"][k]) <= 1e-15, (st["t"], p[0][0], gd["p"][k])


def test_adam_constant_gradient_moves_by_lr():
    """With a constant gradient g the bias-corrected moments are exactly g and g^2 at every step, so each step
    moves every weight by lr |g| / (|g| + eps); a wrong bias-correction power breaks this from step 2 on."""
    g = np.array([[0.3, -1.7], [2.5, -0.01]])
    p = [np.zeros((2, 2))]
    m = [np.zeros((2, 2))]
    v = [np.zeros((2, 2))]
    for t in range(1, 6):
        p, m, v = mo.adam_step(p, [g], m, v, step=t, lr=1e-2)
        np.testing.assert_allclose(p[0], -t * 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_round_by_hand():
    """Nearest bfloat16 (8 significant bits, ties to the even significand) on values worked by hand."""
    cases = [
        (1.0 + 2.0 ** -8, 1.0),                        # halfway between 1 and 1 + 2^-7: the even one, 1
        (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),        # halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
        (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # just above halfway: up
        (255.5, 256.0),                                # 255 (odd) and 256 (even, next binade): 256
        (255.25, 255.0),                               # below halfway: down
        (-3.0, -3.0), (0.0, 0.0),
        (-(1.0 + 2.0 ** -8), -1.0),
        (0.1, 0.10009765625),                          # 0.1 = 1.6 * 2^-4 -> 205/128 * 2^-4 = 0.10009765625
    ]
    for x, want in cases:
        assert mo.bf16_round(x) == want, (x, mo.bf16_round(x), want)
    # any value: the result has 8 significant bits and no other such value is nearer
    g = np.random.default_rng(3)
    x = g.standard_normal(2000) * np.exp2(g.integers(-20, 20, 2000))
    r = mo.bf16_round(x)
    m, e = np.frexp(r)
    assert np.all(np.ldexp(m, 8) == np.rint(np.ldexp(m, 8)))
    ulp = np.ldexp(1.0, np.frexp(x)[1] - 8)
    assert np.all(np.abs(r - x) <= 0.5 * ulp)


def test_bf16_forms_reduce_to_the_pinned_forms():
    """With the rounding replaced by the identity, forward_bf16 / backward_bf16 are forward / backward step for
    step (bit-identical), so the BF16 forms add exactly the rounding points and nothing else; on the hand-worked
    network, whose values are all bfloat16 numbers, forward_bf16 gives the hand-worked logits exactly."""
    g = np.random.default_rng(2)
    params = _params(g)
    x = g.standard_normal((9, 6))
    y = np.where(g.random(9) < 0.5, 1, -1)
    mu, sd = x.mean(axis=0), x.std(axis=0) + 0.5
    ident = lambda v: np.asarray(v, np.float64)
    z, cache = mo.forward(params, x, mu, sd)
    zq, cq = mo.forward_bf16(params, x, mu, sd, rnd=ident)
    np.testing.assert_array_equal(z, zq)
    for a, b in zip(mo.backward(params, cache, z, y), mo.backward_bf16(params, cq, zq, y, rnd=ident)):
        np.testing.assert_array_equal(a, b)
    # the rounding does act: the rounded forms differ from the FP64 forms on general values
    zr, cr = mo.forward_bf16(params, x, mu, sd)
    assert np.max(np.abs(zr - z)) > 0
    gd = _golden("mlp_tiny_forward.json")
    ps = [np.array(gd[k], np.float64) for k in ("W1", "b1", "W2", "b2", "w3")] + [np.array(gd["b3"])]
    zt, _ = mo.forward_bf16(ps, np.array(gd["x"]), np.array(gd["mu"]), np.array(gd["sd"]))
    np.testing.assert_array_equal(zt, np.array(gd["z"]))
