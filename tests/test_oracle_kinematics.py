"""Pins of the FP64 oracle's kinematics (Section II-A, Eq. 1-2) against facts
that do not come from the oracle itself: hand-derived planar closed forms,
the textbook factorisation of a D-H link into elementary motions, and
geometric invariants of rigid chains."""
import json
import math
import os

import numpy as np
import pytest

from paper_1910_06451_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rz(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[c, -s, 0, 0], [s, c, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1.0]])


def _rx(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[1, 0, 0, 0], [0, c, -s, 0], [0, s, c, 0], [0, 0, 0, 1.0]])


def _tz(d):
    T = np.eye(4)
    T[2, 3] = d
    return T


def _tx(a):
    T = np.eye(4)
    T[0, 3] = a
    return T


def test_dh_link_equals_elementary_product(oracle_mod):
    """Eq. 1 is the standard D-H link: Rot_z(theta) Trans_z(d) Trans_x(a) Rot_x(alpha)."""
    g = np.random.default_rng(1)
    for _ in range(50):
        th, al, a, d = g.uniform(-4, 4), g.uniform(-4, 4), g.uniform(-1, 1), g.uniform(-1, 1)
        A = oracle_mod.dh_link(th, al, a, d)
        ref = _rz(th) @ _tz(d) @ _tx(a) @ _rx(al)
        np.testing.assert_allclose(A, ref, atol=1e-15)


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "planar_fk.json")))["cases"])
def test_planar_golden(oracle_mod, case):
    a = np.array(case["a"])
    n = a.shape[0]
    dh = oracle_mod.dh_table(a, np.zeros(n), np.zeros(n))
    P = oracle_mod.control_points(dh, np.arange(n + 1), np.array(case["q"]))
    np.testing.assert_allclose(P, np.array(case["origins"]), atol=1e-15)


def test_planar_closed_form_random(oracle_mod):
    g = np.random.default_rng(2)
    for n in (1, 2, 3, 5):
        a = g.uniform(0.1, 1.0, size=n)
        dh = oracle_mod.dh_table(a, np.zeros(n), np.zeros(n))
        q = g.uniform(-np.pi, np.pi, size=(20, n))
        P = oracle_mod.control_points(dh, np.arange(n + 1), q)
        cum = np.cumsum(q, axis=1)
        ref = np.zeros((20, n + 1, 3))
        ref[:, 1:, 0] = np.cumsum(a * np.cos(cum), axis=1)
        ref[:, 1:, 1] = np.cumsum(a * np.sin(cum), axis=1)
        np.testing.assert_allclose(P, ref, atol=1e-14)


def test_link_length_and_rotation_invariants(oracle_mod):
    """Consecutive origins are sqrt(a_i^2 + d_i^2) apart; rotation blocks are proper orthonormal."""
    g = np.random.default_rng(3)
    n = 7
    a = g.uniform(0.2, 0.4, n)
    d = g.uniform(-0.3, 0.3, n)
    alpha = g.choice([0.0, np.pi / 2, -np.pi / 2, 0.3], n)
    dh = oracle_mod.dh_table(a, alpha, d, theta=g.uniform(-1, 1, n))
    for q in g.uniform(-np.pi, np.pi, size=(30, n)):
        T = oracle_mod.frames(dh, q)
        o = T[:, :3, 3]
        np.testing.assert_allclose(np.linalg.norm(np.diff(o, axis=0), axis=1), np.sqrt(a * a + d * d), atol=1e-14)
        for R in T[:, :3, :3]:
            np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
            assert abs(np.linalg.det(R) - 1.0) < 1e-13


def test_prismatic_joint_moves_along_z(oracle_mod):
    """A prismatic joint adds its variable to d (Section II-A): the origin moves along z_{i-1}."""
    dh = oracle_mod.dh_table([0.5], [0.0], [0.2], theta=[0.0], joint_type=[1])
    P = oracle_mod.control_points(dh, [1], np.array([[0.3]]))
    np.testing.assert_allclose(P[0, 0], [0.5, 0.0, 0.5], atol=1e-15)


def test_base_transform_and_offset(oracle_mod):
    """wA_0 shifts every point; T_m offsets are expressed in frame j_m."""
    dh = oracle_mod.dh_table([1.0], [0.0], [0.0])
    base = np.eye(4)
    base[:3, 3] = [0.1, -0.2, 0.3]
    q = np.array([np.pi / 2])
    P0 = oracle_mod.control_points(dh, [1], q)
    Pb = oracle_mod.control_points(dh, [1], q, base=base)
    np.testing.assert_allclose(Pb[0] - P0[0], [0.1, -0.2, 0.3], atol=1e-15)
    # frame 1 origin at (0, 1, 0) with its x axis along world y: an offset of 0.5 along x_1 lands at (0, 1.5, 0)
    Po = oracle_mod.control_points(dh, [1], q, offset=[[0.5, 0.0, 0.0]])
    np.testing.assert_allclose(Po[0], [0.0, 1.5, 0.0], atol=1e-15)


def test_7dof_workload_shape(oracle_mod):
    arm = wl.arm_7dof()
    assert arm.n == 7 and arm.M == 8
    assert np.all((arm.a >= 0.2) & (arm.a <= 0.4))
    assert set(np.round(arm.alpha, 12)).issubset({0.0, round(np.pi / 2, 12), round(-np.pi / 2, 12)})
    dh = oracle_mod.dh_table(arm.a, arm.alpha, arm.d)
    q = wl.configs("shape", 100, 7)
    P = oracle_mod.control_points(dh, arm.frames, q)
    # frame 0 never moves; the end effector stays within the reach sum(a)
    np.testing.assert_array_equal(P[:, 0], 0.0)
    assert np.all(np.linalg.norm(P[:, -1], axis=1) <= arm.a.sum() + 1e-12)


def test_control_point_frames_drop_exactly_the_coincident_origins(oracle_mod):
    """Section III-A placement: a frame is dropped iff its origin coincides with the preceding one for
    every configuration. Checked against FK itself on random configurations."""
    g = wl.rng("oracle/placement")
    a = np.array([0.3, 0.0, 0.2, 0.0, 0.0, 0.25])
    d = np.array([0.0, 0.0, 0.1, 0.0, 0.15, 0.0])
    types = np.array([0, 0, 0, 1, 0, 0])  # joint 4 prismatic with a = d = 0: it moves, so it keeps a point
    alpha = np.array([0.0, np.pi / 2, -np.pi / 2, np.pi / 2, 0.0, -np.pi / 2])
    dh = oracle_mod.dh_table(a, alpha, d, None, types)
    kept = list(oracle_mod.control_point_frames(dh, include_base=True))
    assert kept == [0, 1, 3, 4, 5, 6]
    assert list(oracle_mod.control_point_frames(dh)) == [1, 3, 4, 5, 6]
    for _ in range(20):
        q = g.uniform(-np.pi, np.pi, 6)
        T = oracle_mod.frames(dh, q)
        o = T[:, :3, 3]
        gaps = np.linalg.norm(o[1:] - o[:-1], axis=1)  # gap between origin i and i-1, i = 1..n
        for i in range(1, 7):
            if i in kept:
                assert gaps[i - 1] > 1e-3
            else:
                assert gaps[i - 1] <= 1e-15
