"""Pins of the oracle's Fastron update (Section III-B, Eq. 5-9, Algorithm 1,
Claim 2): hand-executed trajectories, special cases with known answers and
per-step invariants that follow from the update rules."""
import json
import os

import numpy as np
import pytest

from paper_1910_06451_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _points(oracle_mod, arm, q):
    dh = oracle_mod.dh_table(arm.a, arm.alpha, arm.d, arm.theta, arm.joint_type)
    return oracle_mod.control_points(dh, arm.frames, q)


@pytest.mark.parametrize("case_idx", [0, 1])
def test_worked_trajectory(oracle_mod, case_idx):
    g = json.load(open(os.path.join(GOLDEN, "fastron_worked.json")))
    case = g["cases"][case_idx]
    P = _points(oracle_mod, wl.two_link((1, 2)), np.array(g["x"]))
    out = oracle_mod.fastron_update(P, g["y"], g["gamma"], beta=case["beta"], trace=True)
    assert out["converged"]
    acts = {1: "add", 2: "remove"}
    steps = [[acts[a], int(i), float(d)] for a, i, d in zip(out["trace_action"], out["trace_index"],
                                                            out["trace_dalpha"])]
    assert len(steps) == len(case["steps"])
    for got, want in zip(steps, case["steps"]):
        assert got[0] == want[0] and got[1] == want[1]
        assert abs(got[2] - want[2]) < 1e-15
    np.testing.assert_allclose(out["alpha"], case["alpha"], atol=1e-15)
    np.testing.assert_allclose(out["F"], case["F"], atol=1e-15)
    np.testing.assert_array_equal(out["support"], [0, 1])


def test_all_free_labels_give_one_support(oracle_mod):
    """Every K_FK entry is positive, so one negative support classifies every free sample."""
    arm = wl.arm_3dof()
    q = wl.configs("allfree", 200, 3)
    P = _points(oracle_mod, arm, q)
    out = oracle_mod.fastron_update(P, -np.ones(200, dtype=int), 10.0)
    assert out["converged"]
    np.testing.assert_array_equal(out["support"], [0])
    assert out["alpha"][0] == -1.0
    assert np.all(out["F"] < 0)


def test_identity_kernel_limit(oracle_mod):
    """With gamma so large that every off-diagonal entry underflows to 0 and no shared control point,
    K = I exactly: each point is added once with alpha_i = b_i y_i, nothing is removed, every point is support.
    (With K only close to I, removals legitimately fire on the tiny off-diagonal tails.)"""
    arm = wl.arm_3dof()
    arm.frames = np.array([1, 2, 3], dtype=np.int32)  # drop the fixed base point
    q = wl.configs("klimit", 64, 3)
    P = _points(oracle_mod, arm, q)
    y = np.where(wl.rng("klimit/y").random(64) < 0.4, 1, -1)
    beta = 3.0
    out = oracle_mod.fastron_update(P, y, 1e300, beta=beta)
    np.testing.assert_array_equal(oracle_mod.gram(P, 1e300), np.eye(64))
    assert out["converged"]
    b = np.where(y > 0, beta, 1.0)
    np.testing.assert_array_equal(out["alpha"], b * y)
    assert out["support"].shape[0] == 64


def _random_problem(oracle_mod, name, N, gamma=10.0, frac_pos=0.35):
    arm = wl.arm_3dof()
    q = wl.configs(name, N, 3)
    P = _points(oracle_mod, arm, q)
    # labels from a smooth random field over the end-effector position, so that classes are spatially coherent
    c = wl.rng(name + "/c").uniform(-0.6, 0.6, size=(3, 3))
    d = np.min(np.linalg.norm(P[:, -1][:, None, :2] - c[None, :, :2], axis=2), axis=1)
    y = np.where(d < np.quantile(d, frac_pos), 1, -1)
    return P, y, gamma


@pytest.mark.parametrize("beta", [1.0, 2.0])
def test_per_step_invariants(oracle_mod, beta):
    """Replay the trace against the exact Gram matrix:
    F = K alpha; y_i alpha_i >= 0; after an add F_i = b_i y_i and L drops by exactly dalpha^2/2 >= 1/2
    (Claim 2); after a removal the removed point keeps a positive margin; at break every margin is positive."""
    P, y, gamma = _random_problem(oracle_mod, "inv%d" % int(beta), 150)
    out = oracle_mod.fastron_update(P, y, gamma, beta=beta, trace=True)
    assert out["converged"]
    K = oracle_mod.gram(P, gamma)
    b = np.where(y > 0, beta, 1.0)
    alpha = np.zeros(150)
    L_prev = 0.0
    n_remove = 0
    for act, i, da in zip(out["trace_action"], out["trace_index"], out["trace_dalpha"]):
        alpha[i] += da
        if act == oracle_mod.ACT_REMOVE:
            assert alpha[i] == 0.0 or abs(alpha[i]) < 1e-12
            alpha[i] = 0.0
            n_remove += 1
        F = K @ alpha
        assert np.all(y * alpha >= -1e-12)
        L = 0.5 * alpha @ K @ alpha - (y * b) @ alpha
        if act == oracle_mod.ACT_ADD:
            assert abs(F[i] - b[i] * y[i]) < 1e-10
            assert abs((L - L_prev) + 0.5 * da * da) < 1e-9
            assert da * da >= 1.0 - 1e-12
        else:
            assert y[i] * F[i] > 0
        L_prev = L
    np.testing.assert_allclose(out["alpha"], alpha, atol=1e-10)
    np.testing.assert_allclose(out["F"], K @ out["alpha"], atol=1e-9)
    assert np.all(y * out["F"] > 0)
    assert abs(oracle_mod.loss(P, y, gamma, beta, out["alpha"]) - L_prev) < 1e-8
    np.testing.assert_array_equal(out["support"], np.flatnonzero(out["alpha"]))


def test_removal_branch_fires(oracle_mod):
    """Over several seeds at least one run removes a redundant support point."""
    removed = 0
    for s in range(6):
        P, y, gamma = _random_problem(oracle_mod, "rm%d" % s, 200, gamma=3.0, frac_pos=0.5)
        out = oracle_mod.fastron_update(P, y, gamma, trace=True)
        removed += int(np.sum(out["trace_action"] == oracle_mod.ACT_REMOVE))
    assert removed > 0


def test_support_cap_and_iteration_cap(oracle_mod):
    P, y, gamma = _random_problem(oracle_mod, "caps", 150)
    full = oracle_mod.fastron_update(P, y, gamma)
    assert full["support"].shape[0] > 3
    capped = oracle_mod.fastron_update(P, y, gamma, s_max=3)
    assert capped["support"].shape[0] <= 3
    # the cap can stop the loop while samples are still misclassified (Algorithm 1 falls through to break)
    short = oracle_mod.fastron_update(P, y, gamma, iter_max=2)
    assert not short["converged"] and short["updates"] == 2


def test_warm_start_continues(oracle_mod):
    """loadPreviousModel: resuming from a partial run reaches the same model as one uninterrupted run."""
    P, y, gamma = _random_problem(oracle_mod, "warm", 120)
    full = oracle_mod.fastron_update(P, y, gamma)
    part = oracle_mod.fastron_update(P, y, gamma, iter_max=7)
    rest = oracle_mod.fastron_update(P, y, gamma, alpha=part["alpha"], F=part["F"])
    np.testing.assert_allclose(rest["alpha"], full["alpha"], atol=1e-12)
    np.testing.assert_array_equal(rest["support"], full["support"])


def test_configuration_kernel_training_claim2(oracle_mod):
    """Algorithm 1 with the kernel on configurations (M = 1, D = n): at convergence every margin is positive
    (Claim 2), F equals K alpha with that kernel, and the support set is exactly the nonzero weights."""
    g = np.random.default_rng(3)
    X = g.uniform(-np.pi, np.pi, (300, 7))
    y = np.where(np.sin(X[:, 0]) + 0.5 * np.cos(X[:, 1] + X[:, 2]) > 0.2, 1, -1)
    out = oracle_mod.fastron_update(X[:, None, :], y, 0.5, beta=1.0)
    assert out["converged"]
    K = oracle_mod.gram(X[:, None, :], 0.5)
    np.testing.assert_allclose(out["F"], K @ out["alpha"], rtol=0, atol=1e-9)
    assert np.all(y * out["F"] > 0)
    np.testing.assert_array_equal(out["support"], np.flatnonzero(out["alpha"]))


def test_active_update(oracle_mod):
    """The update after two-stage active learning (Section III-B). Pins: the assembled set is the support
    set, support + noise rows and the exploration rows; F0 on the support rows equals K_SS alpha from the
    Gram matrix; the update converges with every margin positive (Claim 2) and keeps the rows' labels; with
    no new samples and unchanged obstacles a converged model comes back unchanged after zero updates."""
    arm = wl.arm_3dof()
    dh = oracle_mod.dh_table(arm.a, arm.alpha, arm.d, arm.theta, arm.joint_type)
    g = np.random.default_rng(11)
    lo, hi = wl.cubes("al_cubes", 5, 0.15)
    q = wl.configs("al_train", 400, 3)
    y, _ = oracle_mod.capsule_box_labels(dh, q.astype(np.float64), arm.radius, lo, hi)
    P = oracle_mod.control_points(dh, arm.frames, q.astype(np.float64)).astype(np.float32).astype(np.float64)
    base = oracle_mod.fastron_update(P, y, 10.0)
    assert base["converged"]
    sup = base["support"]
    sq, al = q[sup], base["alpha"][sup]
    # no new samples, same obstacles: nothing to change
    same = oracle_mod.active_update(dh, arm.frames, sq, al, 10.0, np.zeros((0, 3)), 0, np.zeros((0, 3)),
                                    arm.radius, lo, hi)
    assert same["updates"] == 0 and same["converged"]
    np.testing.assert_array_equal(same["alpha"], al)
    # moved obstacles, 2 samples near each support point, 150 uniform samples
    lo2, hi2 = lo + 0.05, hi + 0.05
    noise = (0.1 * g.standard_normal((2 * len(sup), 3))).astype(np.float32)
    explore = g.uniform(-np.pi, np.pi, (150, 3)).astype(np.float32)
    out = oracle_mod.active_update(dh, arm.frames, sq, al, 10.0, noise, 2, explore, arm.radius, lo2, hi2)
    X = out["X"]
    S = len(sup)
    assert X.shape == (3 * S + 150, 3)
    np.testing.assert_array_equal(X[:S], sq)
    np.testing.assert_array_equal(X[S:3 * S], (np.repeat(sq, 2, axis=0) + noise).astype(np.float32))
    np.testing.assert_array_equal(X[3 * S:], explore)
    Ps = oracle_mod.control_points(dh, arm.frames, sq.astype(np.float64)).astype(np.float32).astype(np.float64)
    # supports whose label flipped with the move start from weight 0, the others keep theirs
    y_new, _ = oracle_mod.capsule_box_labels(dh, sq.astype(np.float64), arm.radius, lo2, hi2)
    flipped = np.sign(al) != y_new
    assert flipped.any() and not flipped.all()
    np.testing.assert_array_equal(out["relabelled"], np.nonzero(flipped)[0])
    a_kept = np.where(flipped, 0.0, al)
    np.testing.assert_array_equal(out["alpha0"][:S], a_kept)
    np.testing.assert_array_equal(out["alpha0"][S:], 0.0)
    np.testing.assert_allclose(out["F0"][:S], oracle_mod.gram(Ps, 10.0) @ a_kept, rtol=0, atol=1e-12)
    assert out["converged"]
    PX = oracle_mod.control_points(dh, arm.frames, X.astype(np.float64)).astype(np.float32).astype(np.float64)
    K = oracle_mod.gram(PX, 10.0)
    np.testing.assert_allclose(out["F"], K @ out["alpha"], rtol=0, atol=1e-9)
    assert np.all(out["y"] * out["F"] > 0)
