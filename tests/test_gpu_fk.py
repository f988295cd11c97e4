"""Parity of the HIP forward kinematics (Section II-A, Eq. 1-2) with the FP64 oracle."""
import numpy as np
import pytest
import torch

from paper_1910_06451_amd import api, workloads as wl
from conftest import announce, oracle_dh

pytestmark = pytest.mark.gpu


def _ulp32(x):
    return np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)


@pytest.mark.parametrize("arm_name,N", [("3dof", 10_037), ("7dof", 10_037), ("7dof", 1), ("3dof", 255)])
def test_fk_points_parity(oracle_mod, dev, arm_name, N):
    arm = wl.arm_3dof() if arm_name == "3dof" else wl.arm_7dof()
    q = wl.configs(f"fk_{arm_name}_{N}", N, arm.n)
    announce(f"fk_points {arm_name} N={N}")
    P = api.fk_points(arm, torch.from_numpy(q).to(dev)).cpu().numpy().astype(np.float64)
    ref = oracle_mod.control_points(oracle_dh(oracle_mod, arm), arm.frames, q.astype(np.float64))
    err = np.abs(P - ref)
    if arm.n >= 7:
        # FP64 chain: only the final rounding to float32 remains (within one float32 ulp)
        assert np.all(err <= _ulp32(ref) + 1e-30), err.max()
    else:
        # FP32 chain over <= 3 joints with |p| <= 0.9 m
        assert err.max() <= 2e-6, err.max()


def test_fk_points_general_chain(oracle_mod, dev):
    """Prismatic joints, angle offsets, a base transform and point offsets."""
    arm = wl.Arm(a=np.array([0.3, 0.0, 0.25, 0.2]), alpha=np.array([np.pi / 2, -np.pi / 2, 0.0, np.pi / 2]),
                 d=np.array([0.1, 0.2, 0.0, 0.05]), theta=np.array([0.1, -0.2, 0.3, 0.0]),
                 joint_type=np.array([0, 1, 0, 0], dtype=np.int32), frames=np.array([1, 2, 4, 4, 0], dtype=np.int32),
                 offsets=np.array([[0, 0, 0], [0.1, 0, 0], [0, 0.05, 0.02], [0, 0, 0], [0.3, 0.1, 0.2]]))
    base = np.eye(4)
    base[:3, :3] = [[0, -1, 0], [1, 0, 0], [0, 0, 1]]
    base[:3, 3] = [0.5, -0.25, 0.1]
    arm.base = base
    q = wl.configs("fk_general", 3001, 4, lo=-1.5, hi=1.5)
    announce("fk_points general chain")
    P = api.fk_points(arm, torch.from_numpy(q).to(dev)).cpu().numpy()
    ref = oracle_mod.control_points(oracle_dh(oracle_mod, arm), arm.frames, q.astype(np.float64),
                                    offset=arm.offsets, base=base)
    assert np.abs(P - ref).max() <= 3e-6


def test_fk_points_empty(dev):
    arm = wl.arm_7dof()
    P = api.fk_points(arm, torch.zeros((0, 7), dtype=torch.float32, device=dev))
    assert P.shape == (0, 8, 3)


@pytest.mark.parametrize("n,prismatic", [(8, (2, 5)), (16, ()), (7, (6,))])
def test_fk_points_long_general_chains(oracle_mod, dev, n, prismatic):
    """Chains of 7 to 16 joints run the FP64 chain with every joint's sine and cosine computed up front: angle
    offsets, prismatic joints, a base transform, repeated frames, the base frame and point offsets; each
    coordinate within one float32 ulp of the oracle's FP64 result."""
    g = wl.rng(f"fk_long_{n}")
    frames = np.concatenate([[0], np.arange(max(1, n - 12), n + 1), [n, n // 2]]).astype(np.int32)  # <= 16 points
    arm = wl.Arm(a=g.uniform(0.05, 0.2, n), alpha=g.choice(np.array([0.0, np.pi / 2, -np.pi / 2]), size=n),
                 d=g.uniform(-0.1, 0.1, n), theta=g.uniform(-0.5, 0.5, n),
                 joint_type=np.isin(np.arange(n), prismatic).astype(np.int32), frames=frames,
                 offsets=g.uniform(-0.05, 0.05, (frames.shape[0], 3)))
    base = np.eye(4)
    base[:3, :3] = [[0, 0, 1], [1, 0, 0], [0, 1, 0]]
    base[:3, 3] = [0.2, -0.1, 0.3]
    arm.base = base
    q = wl.configs(f"fk_long_{n}/q", 4099, n, lo=-3.0, hi=3.0)
    announce(f"fk_points long chain n={n} prismatic={prismatic}")
    P = api.fk_points(arm, torch.from_numpy(q).to(dev)).cpu().numpy().astype(np.float64)
    ref = oracle_mod.control_points(oracle_dh(oracle_mod, arm), arm.frames, q.astype(np.float64),
                                    offset=arm.offsets, base=base)
    err = np.abs(P - ref)
    assert np.all(err <= _ulp32(ref) + 1e-30), err.max()


def test_fk_points_large_joint_values(oracle_mod, dev):
    """Joint values beyond the range of the branch-free angle reduction (|theta| > 1e5) take the library sine
    and cosine; ordinary lanes of the same wave keep the fast path."""
    arm = wl.arm_7dof()
    q = wl.configs("fk_large/q", 1000, arm.n)
    q[::7, 3] = np.float32(3.0e5)
    q[1::11, 0] = np.float32(-1.0e7)
    q[2::13, 6] = np.float32(9.99e4)  # just inside the fast range
    announce("fk_points large joint values")
    P = api.fk_points(arm, torch.from_numpy(q).to(dev)).cpu().numpy().astype(np.float64)
    ref = oracle_mod.control_points(oracle_dh(oracle_mod, arm), arm.frames, q.astype(np.float64))
    err = np.abs(P - ref)
    assert np.all(err <= _ulp32(ref) + 1e-30), err.max()
