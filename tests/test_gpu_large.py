"""Arrays past 2^31 elements: FK (Section II-A, Eq. 1-2), the Gram column (Section III-A Eq. 4) and the fused
score (Section III-B model) on inputs whose last elements lie beyond 2^31 - 1 float32 elements.

Every kernel takes element offsets in 64 bits; an offset formed in 32 bits would wrap and read or write another
row. The big inputs repeat a ragged seeded block of R rows on the device (row j holds block row j mod R), so
each sampled output, the last rows and those around the 2^31 boundary included, is checked against the oracle
and must equal, bit for bit, the output of its block row computed in the same launch."""
import numpy as np
import pytest
import torch

from paper_1910_06451_amd import api, workloads as wl
from conftest import announce, oracle_dh
from test_gpu_fk import _ulp32
from test_gpu_score import check_scores, error_bound

pytestmark = pytest.mark.gpu

R = 1_000_003  # rows of the repeated block (ragged against every tile and workgroup size)


def _repeated(name, N, n, dev):
    base = wl.configs(name, R, n)
    reps = -(-N // R)
    return base, torch.from_numpy(base).to(dev).repeat(reps, 1)[:N]


def _sample(name, N, boundary):
    g = wl.rng(name + "/sample")
    idx = np.concatenate([g.choice(N, 300, replace=False), np.arange(N - 64, N),
                          np.arange(boundary - 32, boundary + 32), [0, R - 1, R]])
    return np.unique(idx)


def test_fk_points_and_gram_column_past_2g(oracle_mod, dev):
    """90,000,000 configurations of the 7-DOF arm: 2.16e9 control-point coordinates (8 points x 3 per row), row
    89,478,486 onwards entirely past 2^31; the Gram column against a point in that range, over all of them."""
    arm = wl.arm_7dof()
    N, w = 90_000_000, 3 * arm.M
    base, q = _repeated("large/fk", N, arm.n, dev)
    announce(f"fk_points 7dof N={N}")
    P = api.fk_points(arm, q)
    torch.cuda.synchronize()
    del q
    first_past = -(-(2 ** 31) // w)
    assert (N - 1) * w + w - 1 > 2 ** 31 - 1 and first_past < N
    idx = _sample("large/fk", N, first_past)
    got = P[torch.from_numpy(idx).to(dev)].cpu().numpy()
    own = P[torch.from_numpy(idx % R).to(dev)].cpu().numpy()
    np.testing.assert_array_equal(got, own)
    dh = oracle_dh(oracle_mod, arm)
    ref = oracle_mod.control_points(dh, arm.frames, base[idx % R].astype(np.float64))
    err = np.abs(got.astype(np.float64) - ref)
    assert np.all(err <= _ulp32(ref) + 1e-30), err.max()

    # Gram column and F update against the last point (its own coordinates past 2^31 as well)
    i = N - 5
    announce(f"gram_update N={N} i={i}")
    F = torch.zeros(N, dtype=torch.float32, device=dev)
    kcol = api.gram_update_points(P, 10.0, i, 0.5, F=F)
    torch.cuda.synchronize()
    kc, Fs = kcol[torch.from_numpy(idx).to(dev)].cpu().numpy(), F[torch.from_numpy(idx).to(dev)].cpu().numpy()
    np.testing.assert_array_equal(kc, kcol[torch.from_numpy(idx % R).to(dev)].cpu().numpy())
    P32 = got.reshape(-1, arm.M, 3).astype(np.float64)
    Pi = P[i].cpu().numpy().astype(np.float64)
    kref = np.array([oracle_mod.k_fk(P32[r], Pi, 10.0) for r in range(len(idx))])
    assert np.abs(kc - kref).max() <= 1e-6
    assert float(kcol[i]) == 1.0
    np.testing.assert_array_equal(Fs, (0.5 * kc.astype(np.float64)).astype(np.float32))
    del P, kcol, F
    torch.cuda.empty_cache()


def test_score_past_2g(oracle_mod, dev):
    """310,000,000 queries of the 7-DOF arm in one launch: 2.17e9 joint values, query 306,783,379 onwards past
    2^31; S = 64 supports (four tiles), gamma = 10; the FP32 form and the BF16 SPLIT3 form (FP32 bound)."""
    arm = wl.arm_7dof()
    N, S, gamma = 310_000_000, 64, 10.0
    sq, al = wl.model("large/score", S, arm.n)
    base, q = _repeated("large/score/q", N, arm.n, dev)
    first_past = -(-(2 ** 31) // arm.n)
    assert N * arm.n > 2 ** 31 - 1 and first_past < N
    sq_d, al_d = torch.from_numpy(sq).to(dev), torch.from_numpy(al).to(dev)
    idx = _sample("large/score", N, first_past)
    ti, to = torch.from_numpy(idx).to(dev), torch.from_numpy(idx % R).to(dev)
    dh = oracle_dh(oracle_mod, arm)
    qs = base[idx % R].astype(np.float64)
    ref = oracle_mod.score(dh, arm.frames, sq.astype(np.float64), al.astype(np.float64), gamma, qs)
    tol = error_bound(oracle_mod.control_points(dh, arm.frames, sq.astype(np.float64)), al, gamma,
                      oracle_mod.control_points(dh, arm.frames, qs))
    for name in ("fp32", "bf16 split3"):
        announce(f"fk_score 7dof {name} S={S} N={N}")
        if name == "fp32":
            f, lab = api.fk_score(arm, sq_d, al_d, gamma, q)
        else:
            model = api.support_prep(arm, sq_d, al_d, gamma)
            f, lab = api.fk_score_prepared(arm, model, q, flags=api.SCORE_BF16 | api.BF16_SPLIT3)
        torch.cuda.synchronize()
        fg, lg = f[ti].cpu().numpy(), lab[ti].cpu().numpy()
        np.testing.assert_array_equal(fg, f[to].cpu().numpy())
        np.testing.assert_array_equal(lg, lab[to].cpu().numpy())
        stats = check_scores(fg, lg, ref, tol, min_agree=0.99)
        print(name, stats)
        del f, lab
    del q
    torch.cuda.empty_cache()
