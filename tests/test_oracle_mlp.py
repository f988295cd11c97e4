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
