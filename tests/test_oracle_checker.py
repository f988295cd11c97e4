"""Pins of the oracle's geometric labeller (capsule links vs axis-aligned
boxes; it stands in for the ground-truth checker of Section IV) against hand
cases and brute-force sphere sampling."""
import numpy as np

from paper_1910_06451_amd import workloads as wl


def test_segment_box_hand_cases(oracle_mod):
    d2 = oracle_mod.segment_box_dist2
    assert abs(d2([-1, 0, 0], [1, 0, 0], [-0.1, 0.5, -0.1], [0.1, 0.7, 0.1]) - 0.25) < 1e-15
    assert d2([-1, 0.6, 0], [1, 0.6, 0], [-0.1, 0.5, -0.1], [0.1, 0.7, 0.1]) == 0.0
    assert abs(d2([2, 2, 2], [3, 3, 3], [0, 0, 0], [1, 1, 1]) - 3.0) < 1e-15
    assert abs(d2([2, -1, 0.5], [2, 2, 0.5], [0, 0, 0], [1, 1, 1]) - 1.0) < 1e-15
    assert abs(d2([0.5, 0.5, 3], [0.5, 0.5, 3], [0, 0, 0], [1, 1, 1]) - 4.0) < 1e-15  # zero-length link
    # a diagonal segment passing a box edge: closest approach from the edge x=1,y=1 to the line x+y=3 (z inside)
    assert abs(d2([3, 0, 0.5], [0, 3, 0.5], [0, 0, 0], [1, 1, 1]) - 0.5) < 1e-15


def _sample_dist(A, B, lo, hi, h):
    L = np.linalg.norm(B - A)
    k = max(2, int(np.ceil(L / h)) + 1)
    t = np.linspace(0.0, 1.0, k)
    p = A[None, :] + t[:, None] * (B - A)[None, :]
    e = np.maximum(np.maximum(lo - p, 0.0), p - hi)
    return np.sqrt(np.min(np.sum(e * e, axis=1))), L / (k - 1)


def test_segment_box_vs_dense_sampling(oracle_mod):
    g = np.random.default_rng(7)
    for _ in range(300):
        A, B = g.uniform(-1, 1, 3), g.uniform(-1, 1, 3)
        c, s = g.uniform(-0.5, 0.5, 3), g.uniform(0.05, 0.4, 3)
        lo, hi = c - s, c + s
        exact = np.sqrt(oracle_mod.segment_box_dist2(A, B, lo, hi))
        ds, step = _sample_dist(A, B, lo, hi, 1e-4)
        assert exact <= ds + 1e-12
        assert ds <= exact + 0.5 * step + 1e-12


def test_labels_vs_brute_force_grid(oracle_mod):
    """3-DOF planar arm on a 24^3 grid against cubes that straddle its plane: sphere sampling with spacing
    h <= r/20 brackets the exact distance, so labels must agree wherever the bracket is decisive."""
    arm = wl.arm_3dof()
    dh = oracle_mod.dh_table(arm.a, arm.alpha, arm.d)
    g1 = np.linspace(-np.pi, np.pi, 24, endpoint=False)
    q = np.stack(np.meshgrid(g1, g1, g1, indexing="ij"), axis=-1).reshape(-1, 3)
    g = wl.rng("checker_grid")
    centres = np.concatenate([g.uniform(-0.7, 0.7, (4, 2)), g.uniform(-0.05, 0.05, (4, 1))], axis=1)
    lo, hi = centres - 0.075, centres + 0.075
    r = arm.radius
    lab, clr = oracle_mod.capsule_box_labels(dh, q, r, lo, hi)
    T = oracle_mod.frames(dh, q[0])  # shape check of the frame API
    assert T.shape == (4, 4, 4)
    decisive = 0
    hits = 0
    for j in range(q.shape[0]):
        o = oracle_mod.frames(dh, q[j])[:, :3, 3]
        best_s, best_step = np.inf, 0.0
        for i in range(1, 4):
            for b in range(lo.shape[0]):
                ds, step = _sample_dist(o[i - 1], o[i], lo[b], hi[b], r / 20.0)
                if ds < best_s:
                    best_s, best_step = ds, step
        exact = clr[j] + r
        assert exact <= best_s + 1e-12 and best_s <= exact + 0.5 * best_step + 1e-12
        if best_s <= r:
            assert lab[j] == 1
            decisive += 1
            hits += 1
        elif best_s - 0.5 * best_step > r:
            assert lab[j] == -1
            decisive += 1
    assert decisive > 0.99 * q.shape[0]
    assert 0 < hits < q.shape[0]
