"""Parity of the device geometric labeller with the oracle's checker.

Both decide 'distance <= radius' in FP64, with different algorithms (the
oracle minimises the piecewise quadratic exactly, the device bisects the
derivative), so labels must agree bit for bit except where the clearance is
within rounding of zero. The label-only mode (early exit at the first touching
pair) must give the same labels as the mode that also returns the clearance."""
import numpy as np
import pytest
import torch

from paper_1910_06451_amd import api, workloads as wl
from conftest import announce, oracle_dh

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("arm_name,N,n_cubes", [("3dof", 20000, 5), ("7dof", 100003, 20), ("7dof", 17, 0)])
def test_labels_match_oracle(oracle_mod, dev, arm_name, N, n_cubes):
    arm = wl.arm_3dof() if arm_name == "3dof" else wl.arm_7dof()
    q = wl.configs(f"label_{arm_name}", N, arm.n)
    if arm_name == "3dof":
        # cubes straddling the arm's plane so that both labels occur
        g = wl.rng("label3/cubes")
        c = np.concatenate([g.uniform(-0.7, 0.7, (n_cubes, 2)), g.uniform(-0.05, 0.05, (n_cubes, 1))], axis=1)
        lo, hi = c - 0.075, c + 0.075
    else:
        lo, hi = wl.cubes(f"label_{arm_name}/cubes", n_cubes, 0.1, 0.25)
    announce(f"label {arm_name} N={N} cubes={n_cubes}")
    lab, clr = api.label_capsule_box(arm, torch.from_numpy(q).to(dev), arm.radius, lo, hi)
    lab, clr = lab.cpu().numpy(), clr.cpu().numpy()
    # labels alone: the kernel stops at a configuration's first touching pair; same decisions
    lab_only, _ = api.label_capsule_box(arm, torch.from_numpy(q).to(dev), arm.radius, lo, hi, want_clearance=False)
    np.testing.assert_array_equal(lab_only.cpu().numpy(), lab)
    ref, ref_clr = oracle_mod.capsule_box_labels(oracle_dh(oracle_mod, arm), q.astype(np.float64), arm.radius, lo,
                                                 hi)
    near = np.abs(ref_clr) < 1e-9
    np.testing.assert_array_equal(lab[~near], ref[~near])
    if n_cubes:
        assert np.abs(clr - ref_clr).max() <= 1e-6
        print(dict(collision_rate=float(np.mean(ref == 1)), near_boundary=int(near.sum())))
    else:
        assert np.all(lab == -1)


def _prismatic_chain():
    g = wl.rng("label_chain6")
    n = 6
    jt = np.zeros(n, dtype=np.int32)
    jt[[1, 4]] = 1
    return wl.Arm(a=g.uniform(0.1, 0.25, n), alpha=g.choice(np.array([0.0, np.pi / 2, -np.pi / 2]), size=n),
                  d=g.uniform(-0.1, 0.1, n), theta=g.uniform(-0.5, 0.5, n), joint_type=jt,
                  frames=np.arange(n + 1, dtype=np.int32))


@pytest.mark.parametrize("case", ["cubes_and_point_box", "enclosing_box"])
def test_labels_general_chain(oracle_mod, dev, case):
    """A 6-joint chain with two prismatic joints (joint values as lengths), a ragged batch; random cubes plus a
    degenerate box (lo = hi, a single point), or one box enclosing the whole reach (every configuration
    collides, every clearance negative)."""
    arm = _prismatic_chain()
    q = wl.configs(f"label_chain6/{case}", 1001, arm.n, lo=-1.0, hi=1.0)
    if case == "cubes_and_point_box":
        lo, hi = wl.cubes("label_chain6/cubes", 8, 0.1, 0.25)
        p = np.array([[0.15, 0.05, 0.1]])
        lo, hi = np.concatenate([lo, p]), np.concatenate([hi, p])
    else:
        lo, hi = np.full((1, 3), -10.0), np.full((1, 3), 10.0)
    announce(f"label prismatic chain {case}")
    lab, clr = api.label_capsule_box(arm, torch.from_numpy(q).to(dev), arm.radius, lo, hi)
    lab, clr = lab.cpu().numpy(), clr.cpu().numpy()
    lab_only, _ = api.label_capsule_box(arm, torch.from_numpy(q).to(dev), arm.radius, lo, hi, want_clearance=False)
    np.testing.assert_array_equal(lab_only.cpu().numpy(), lab)
    ref, ref_clr = oracle_mod.capsule_box_labels(oracle_dh(oracle_mod, arm), q.astype(np.float64), arm.radius, lo,
                                                 hi)
    near = np.abs(ref_clr) < 1e-9
    np.testing.assert_array_equal(lab[~near], ref[~near])
    assert np.abs(clr - ref_clr).max() <= 1e-6
    if case == "enclosing_box":
        assert np.all(lab == 1) and np.all(clr < 0)
    print(dict(case=case, collision_rate=float(np.mean(ref == 1)), near_boundary=int(near.sum())))
