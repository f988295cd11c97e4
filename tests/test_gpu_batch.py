"""Batched form: many environments (one arm, uneven support sets and query
batches) scored in one persistent launch must give exactly the single-model
result for each environment, and, through it, the oracle's within the FP32
error bound. Graph replays are checked against the eager result each time."""
import numpy as np
import pytest
import torch

from paper_1910_06451_amd import api, workloads as wl
from conftest import announce, oracle_dh
from test_gpu_score import check_scores, error_bound

pytestmark = pytest.mark.gpu


def _envs(name, S_counts, Q_counts, n):
    sq = wl.configs(name + "/s", int(np.sum(S_counts)), n)
    al = wl.weights(name + "/a", int(np.sum(S_counts)))
    q = wl.configs(name + "/q", int(np.sum(Q_counts)), n)
    return sq, al, q


def _per_env_reference(arm, S_counts, Q_counts, sq, al, q, gamma, dev, envs):
    so = np.concatenate([[0], np.cumsum(S_counts)])
    qo = np.concatenate([[0], np.cumsum(Q_counts)])
    out = {}
    for e in envs:
        s_d = torch.from_numpy(sq[so[e]:so[e + 1]]).to(dev)
        a_d = torch.from_numpy(al[so[e]:so[e + 1]]).to(dev)
        q_d = torch.from_numpy(q[qo[e]:qo[e + 1]]).to(dev)
        model = api.support_prep(arm, s_d, a_d, gamma)
        out[e] = api.fk_score_prepared(arm, model, q_d)
    return out, so, qo


def test_batch_matches_single_model_and_oracle(oracle_mod, dev):
    arm = wl.arm_7dof()
    gamma = 10.0
    S_counts = np.array([1, 17, 200, 833, 0, 64, 2000, 5, 350, 4096, 999, 16])
    Q_counts = np.array([100, 1, 640, 333, 50, 0, 1000, 64, 65, 129, 17, 300])
    sq, al, q = _envs("batch_small", S_counts, Q_counts, 7)
    announce("batch small E=12")
    b = api.Batch(arm, S_counts, Q_counts, gamma)
    b.prepare(torch.from_numpy(sq).to(dev), torch.from_numpy(al).to(dev))
    q_d = torch.from_numpy(q).to(dev)
    f, lab = b.score(q_d)
    ref, so, qo = _per_env_reference(arm, S_counts, Q_counts, sq, al, q, gamma, dev, range(len(S_counts)))
    for e, (fr, lr) in ref.items():
        assert torch.equal(f[qo[e]:qo[e + 1]], fr), e
        assert torch.equal(lab[qo[e]:qo[e + 1]], lr), e
    # empty model -> f = 0
    assert torch.all(f[qo[4]:qo[5]] == 0)
    # oracle on a sample from every non-empty environment
    dh = oracle_dh(oracle_mod, arm)
    fn, ln = f.cpu().numpy(), lab.cpu().numpy()
    for e in range(len(S_counts)):
        if Q_counts[e] == 0 or S_counts[e] == 0:
            continue
        idx = np.arange(qo[e], qo[e + 1])[:40]
        s64 = sq[so[e]:so[e + 1]].astype(np.float64)
        r = oracle_mod.score(dh, arm.frames, s64, al[so[e]:so[e + 1]].astype(np.float64), gamma,
                             q[idx].astype(np.float64))
        tol = error_bound(oracle_mod.control_points(dh, arm.frames, s64), al[so[e]:so[e + 1]], gamma,
                          oracle_mod.control_points(dh, arm.frames, q[idx].astype(np.float64)))
        check_scores(fn[idx], ln[idx], r, tol, min_agree=0.97)
    b.close()


def test_batch_autotune_and_graph_replay(dev):
    arm = wl.arm_7dof()
    gamma = 10.0
    envs = wl.batched_envs(E=16, q_lo=500, q_hi=3000)
    sq, al, q = _envs("batch_graph", envs.support_counts, envs.query_counts, 7)
    b = api.Batch(arm, envs.support_counts, envs.query_counts, gamma)
    b.prepare(torch.from_numpy(sq).to(dev), torch.from_numpy(al).to(dev))
    q_d = torch.from_numpy(q).to(dev)
    announce("batch eager")
    f0, l0 = b.score(q_d)
    f0, l0 = f0.clone(), l0.clone()
    announce("batch autotune")
    tq = b.autotune(q_d)
    assert tq in (16, 32, 64)
    f1, l1 = b.score(q_d)
    assert torch.equal(f1, f0) and torch.equal(l1, l0)
    side = torch.cuda.Stream()
    f_g = torch.empty_like(f0)
    l_g = torch.empty_like(l0)
    q_g = q_d.clone()
    announce("batch graph capture")
    with torch.cuda.stream(side):
        b.capture(q_g, (f_g, l_g))
    torch.cuda.synchronize()
    q2 = torch.from_numpy(wl.configs("batch_graph/q2", q.shape[0], 7)).to(dev)
    for rep in range(4):
        src = q_d if rep % 2 == 0 else q2
        q_g.copy_(src)  # eager work between replays
        expect_f, expect_l = b.score(src)
        expect_f, expect_l = expect_f.clone(), expect_l.clone()
        torch.cuda.synchronize()
        announce(f"batch graph replay {rep}")
        with torch.cuda.stream(side):
            b.replay()
        side.synchronize()
        assert torch.equal(f_g, expect_f), rep
        assert torch.equal(l_g, expect_l), rep
    # a new launch shape rebuilds the work items and drops the captured graph (which holds the old kernel and
    # item count): replay refuses until the caller captures again, and the new capture replays exactly
    cur = b.shape["queries_per_item"]
    b.set_shape(*((16, 4, 0, 100) if cur != 16 else (32, 8, 0, 75)))
    assert b.shape["queries_per_item"] != cur
    with pytest.raises(api.nat.FastronError, match="no captured graph"):
        b.replay()
    announce("batch graph recapture after a new shape")
    with torch.cuda.stream(side):
        b.capture(q_g, (f_g, l_g))
    torch.cuda.synchronize()
    q_g.copy_(q2)
    expect_f, expect_l = b.score(q2)
    expect_f, expect_l = expect_f.clone(), expect_l.clone()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        b.replay()
    side.synchronize()
    assert torch.equal(f_g, expect_f) and torch.equal(l_g, expect_l)
    b.close()


def test_batch_full_scale(oracle_mod, dev):
    """256 environments, lognormal support sets over [200, 8000], 1,000-100,000 queries each."""
    arm = wl.arm_7dof()
    gamma = 10.0
    envs = wl.batched_envs()
    sq, al, q = _envs("batch_full", envs.support_counts, envs.query_counts, 7)
    b = api.Batch(arm, envs.support_counts, envs.query_counts, gamma)
    b.prepare(torch.from_numpy(sq).to(dev), torch.from_numpy(al).to(dev))
    q_d = torch.from_numpy(q).to(dev)
    announce(f"batch full E=256 N={q.shape[0]}")
    f, lab = b.score(q_d)
    pick = [0, int(np.argmax(envs.support_counts)), int(np.argmin(envs.support_counts)), 255]
    ref, so, qo = _per_env_reference(arm, envs.support_counts, envs.query_counts, sq, al, q, gamma, dev, pick)
    for e, (fr, lr) in ref.items():
        assert torch.equal(f[qo[e]:qo[e + 1]], fr), e
        assert torch.equal(lab[qo[e]:qo[e + 1]], lr), e
    assert torch.isfinite(f).all()
    # the oracle on a sample of the largest and the smallest environment
    dh = oracle_dh(oracle_mod, arm)
    fn, ln = f.cpu().numpy(), lab.cpu().numpy()
    for e in pick[1:3]:
        s64 = sq[so[e]:so[e + 1]].astype(np.float64)
        idx = np.arange(qo[e], qo[e + 1])[::max(1, int(envs.query_counts[e]) // 200)]
        r = oracle_mod.score(dh, arm.frames, s64, al[so[e]:so[e + 1]].astype(np.float64), gamma,
                             q[idx].astype(np.float64))
        tol = error_bound(oracle_mod.control_points(dh, arm.frames, s64), al[so[e]:so[e + 1]], gamma,
                          oracle_mod.control_points(dh, arm.frames, q[idx].astype(np.float64)))
        check_scores(fn[idx], ln[idx], r, tol, min_agree=0.99)
    b.close()


def test_every_launch_shape_gives_the_same_result(dev):
    """Every launch shape the autotuner chooses from (queries per item x waves per workgroup x paired MFMAs x
    grid share) scores each environment exactly as the single-model path; autotune keeps one of them, and a
    second batch of the same kind (same moving points, support-size bucket and device) reuses it without
    timing."""
    arm = wl.arm_7dof()
    gamma = 10.0
    S_counts = np.array([300, 17, 1200, 0, 64, 2000, 5, 750])
    Q_counts = np.array([700, 1, 64, 50, 0, 1000, 129, 333])
    sq, al, q = _envs("batch_shapes", S_counts, Q_counts, 7)
    b = api.Batch(arm, S_counts, Q_counts, gamma)
    b.prepare(torch.from_numpy(sq).to(dev), torch.from_numpy(al).to(dev))
    q_d = torch.from_numpy(q).to(dev)
    ref, so, qo = _per_env_reference(arm, S_counts, Q_counts, sq, al, q, gamma, dev, range(len(S_counts)))
    shapes = [(16 * qb, w, p, occ) for qb in (1, 2, 4) for w in (4, 8) for p in ((0, 1) if qb >= 2 else (0,))
              for occ in (100, 75)]
    assert len(shapes) == 20
    for sh in shapes:
        announce(f"batch shape {sh}")
        b.set_shape(*sh)
        f, lab = b.score(q_d)
        for e, (fr, lr) in ref.items():
            assert torch.equal(f[qo[e]:qo[e + 1]], fr), (sh, e)
            assert torch.equal(lab[qo[e]:qo[e + 1]], lr), (sh, e)
    announce("batch autotune (timed)")
    b.autotune(q_d)
    first = b.shape
    assert first["from_cache"] == 0
    assert (first["queries_per_item"], first["waves_per_group"], first["paired"], first["grid_pct"]) in shapes
    f, lab = b.score(q_d)
    for e, (fr, lr) in ref.items():
        assert torch.equal(f[qo[e]:qo[e + 1]], fr), e
    announce("batch autotune (same kind: cached)")
    b2 = api.Batch(arm, S_counts, Q_counts, gamma)
    b2.prepare(torch.from_numpy(sq).to(dev), torch.from_numpy(al).to(dev))
    b2.autotune(q_d)
    second = b2.shape
    assert second["from_cache"] == 1
    assert {k: v for k, v in second.items() if k != "from_cache"} == {k: v for k, v in first.items()
                                                                       if k != "from_cache"}
    print(dict(tuned=first))
    b.close()
    b2.close()
