"""Pins of the oracle's kernels (Section II-B Eq. 3, Section III-A Eq. 4 and
Claim 1) and of the model score (Section III-B)."""
import json
import os
from fractions import Fraction

import numpy as np

from paper_1910_06451_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dh(oracle_mod, arm):
    return oracle_mod.dh_table(arm.a, arm.alpha, arm.d, arm.theta, arm.joint_type)


def test_k_rq_values(oracle_mod):
    x = np.array([0.3, -0.2, 0.9])
    assert oracle_mod.k_rq(x, x, 10.0) == 1.0
    # gamma = 2, d^2 = 1 -> (1 + 1)^-2 = 1/4 exactly; d^2 = 2 -> 1/9
    assert oracle_mod.k_rq([0, 0, 0], [1, 0, 0], 2.0) == 0.25
    assert abs(oracle_mod.k_rq([0, 0, 0], [1, 1, 0], 2.0) - 1.0 / 9.0) < 1e-16
    # second order, not a Gaussian: at gamma/2 d^2 = 3 the value is 1/16, far above exp(-3)
    assert abs(oracle_mod.k_rq([0.0], [np.sqrt(3.0)], 2.0) - 0.0625) < 1e-15


def test_k_fk_two_link_golden(oracle_mod):
    g = json.load(open(os.path.join(GOLDEN, "two_link_kfk.json")))
    for frames, key in ((g["frames_distal"], "k_fk_distal"), (g["frames_with_base"], "k_fk_with_base")):
        arm = wl.two_link(frames)
        dh = _dh(oracle_mod, arm)
        Px = oracle_mod.control_points(dh, arm.frames, np.array(g["x"]))
        Pxp = oracle_mod.control_points(dh, arm.frames, np.array(g["xp"]))
        assert abs(oracle_mod.k_fk(Px, Pxp, g["gamma"]) - g[key]) < 1e-15
    arm = wl.two_link(g["frames_distal"])
    np.testing.assert_allclose(oracle_mod.control_points(_dh(oracle_mod, arm), arm.frames, np.array(g["xp"])),
                               np.array(g["control_points_xp"]), atol=1e-15)


def test_gram_symmetric_unit_diagonal_psd(oracle_mod):
    arm = wl.arm_7dof()
    dh = _dh(oracle_mod, arm)
    q = wl.configs("gram_psd", 60, 7)
    P = oracle_mod.control_points(dh, arm.frames, q)
    K = oracle_mod.gram(P, 10.0)
    np.testing.assert_array_equal(K, K.T)
    np.testing.assert_array_equal(np.diag(K), 1.0)
    assert np.all(K > 0) and np.all(K <= 1.0)
    np.linalg.cholesky(K)  # PD for distinct configurations (Claim 1)
    # the base point never moves, so every entry is at least 1/M
    assert K.min() >= 1.0 / arm.M - 1e-15


def test_claim1_construction(oracle_mod):
    g = json.load(open(os.path.join(GOLDEN, "claim1_construction.json")))
    arm = wl.two_link((1, 2))
    P = oracle_mod.control_points(_dh(oracle_mod, arm), arm.frames, np.array(g["q"]))
    np.testing.assert_allclose(P[:, 0], np.array(g["elbow_points"], float), atol=1e-15)
    np.testing.assert_allclose(P[:, 1], np.array(g["end_points"], float), atol=1e-15)
    K1 = np.array([[float(Fraction(v)) for v in r] for r in g["K_elbow"]])
    K2 = np.array([[float(Fraction(v)) for v in r] for r in g["K_end"]])
    np.testing.assert_allclose(oracle_mod.gram_summand(P, 2.0, 0), K1, atol=1e-15)
    np.testing.assert_allclose(oracle_mod.gram_summand(P, 2.0, 1), K2, atol=1e-15)
    K = oracle_mod.gram(P, 2.0)
    np.testing.assert_allclose(K, 0.5 * (K1 + K2), atol=1e-15)
    assert np.linalg.matrix_rank(K1, tol=1e-10) == g["rank_elbow"]
    assert np.linalg.matrix_rank(K2, tol=1e-10) == g["rank_end"]
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > 0.1  # PD although both summands are singular
    np.linalg.cholesky(K)


def test_score_definition_pins(oracle_mod):
    g = json.load(open(os.path.join(GOLDEN, "two_link_kfk.json")))
    arm = wl.two_link(g["frames_distal"])
    dh = _dh(oracle_mod, arm)
    # one support with weight 1: f is the kernel value itself
    f = oracle_mod.score(dh, arm.frames, np.array([g["x"]]), [1.0], g["gamma"], np.array([g["xp"]]))
    assert abs(f[0] - g["k_fk_distal"]) < 1e-15
    # linear in alpha, additive over supports, zero for an empty model
    sq = np.array([g["x"], g["xp"]])
    f2 = oracle_mod.score(dh, arm.frames, sq, [2.0, -3.0], g["gamma"], np.array([g["xp"]]))
    assert abs(f2[0] - (2.0 * g["k_fk_distal"] - 3.0)) < 1e-15
    f0 = oracle_mod.score(dh, arm.frames, np.zeros((0, 2)), np.zeros(0), g["gamma"], np.array([g["xp"]]))
    assert f0[0] == 0.0


def test_score_matches_points_path(oracle_mod):
    arm = wl.arm_7dof()
    dh = _dh(oracle_mod, arm)
    sq, al = wl.model("score_pts", 50, 7)
    q = wl.configs("score_pts/q", 40, 7)
    f = oracle_mod.score(dh, arm.frames, sq, al, 10.0, q)
    Ps = oracle_mod.control_points(dh, arm.frames, sq)
    Pq = oracle_mod.control_points(dh, arm.frames, q)
    K = np.array([[oracle_mod.k_fk(Ps[i], Pq[j], 10.0) for i in range(50)] for j in range(40)])
    np.testing.assert_allclose(f, K @ al.astype(np.float64), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle_mod.score_points(Ps, al, 10.0, Pq), f, rtol=0, atol=0)


def test_predict_sign_rule(oracle_mod):
    np.testing.assert_array_equal(oracle_mod.predict([-1e-30, 0.0, 2.0]), [-1, 1, 1])


def test_points_kernel_on_configurations(oracle_mod):
    """Eq. 4 generalised to M points of D coordinates, used with M = 1 and the joint vector (D = n) for the
    kernel on configurations. Pinned by properties a dropped coordinate, a wrong index or a misplaced gamma
    would break: rigid motions and coordinate permutations of both vectors leave it unchanged, zero
    coordinates past the third reduce it to the 3-D control-point kernel, (x, gamma) -> (c x, gamma / c^2)
    leaves it unchanged, and its Gram matrix has a unit diagonal and is positive definite."""
    g = np.random.default_rng(5)
    x, xp = g.uniform(-np.pi, np.pi, 7), g.uniform(-np.pi, np.pi, 7)
    k = oracle_mod.k_pts(x[None], xp[None], 0.7)
    d2 = float(np.sum((x - xp) ** 2))
    assert abs(k - oracle_mod.k_rq(np.zeros(1), np.array([np.sqrt(d2)]), 0.7)) < 1e-15  # depends on |x - x'| only
    Q, _ = np.linalg.qr(g.standard_normal((7, 7)))
    b = g.standard_normal(7)
    assert abs(oracle_mod.k_pts((Q @ x + b)[None], (Q @ xp + b)[None], 0.7) - k) < 1e-13
    perm = g.permutation(7)
    assert abs(oracle_mod.k_pts(x[perm][None], xp[perm][None], 0.7) - k) < 1e-15
    assert abs(oracle_mod.k_pts(3.0 * x[None], 3.0 * xp[None], 0.7 / 9.0) - k) < 1e-14
    # zero padding: a D = 7 point with coordinates 3..6 equal is the 3-D kernel of its first three
    x3, xp3 = x.copy(), xp.copy()
    x3[3:] = xp3[3:] = 0.25
    assert abs(oracle_mod.k_pts(x3[None], xp3[None], 0.7) - oracle_mod.k_fk(x3[None, :3], xp3[None, :3], 0.7)) < 1e-16
    # M points of D coordinates average the per-point kernels (Eq. 4's 1/M)
    P1, P2 = g.standard_normal((3, 5)), g.standard_normal((3, 5))
    avg = np.mean([oracle_mod.k_pts(P1[m][None], P2[m][None], 0.7) for m in range(3)])
    assert abs(oracle_mod.k_pts(P1, P2, 0.7) - avg) < 1e-16
    X = g.uniform(-np.pi, np.pi, (40, 1, 7))
    K = oracle_mod.gram(X, 0.5)
    np.testing.assert_array_equal(K, K.T)
    np.testing.assert_array_equal(np.diag(K), 1.0)
    np.linalg.cholesky(K)
    # the model sum over supports
    alpha = g.standard_normal(40)
    f = oracle_mod.rbf_score(X[:, 0], alpha, 0.5, X[:5, 0])
    np.testing.assert_allclose(f, K[:5] @ alpha, rtol=0, atol=1e-13)
