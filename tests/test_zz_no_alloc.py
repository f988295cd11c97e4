"""The scoring entry point that allocates nothing (fastron_fk_score_noalloc): through the C ABI, its f and
labels equal fastron_fk_score's bit for bit on the same inputs, over consecutive calls that reuse the static
buffer (the second and third smaller than the first, so stale contents of a larger model would show), and both
stay within the FP32 error bound of the FP64 oracle on sampled queries. A support set too large for the buffer
is refused before any device work."""
import numpy as np
import pytest
import torch

from paper_1910_06451_amd import _native as nat, api, workloads as wl
from conftest import announce, oracle_dh
from test_gpu_score import check_scores, error_bound

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("calls", [[(4000, 20_011, api.SCORE_FP32), (517, 3001, api.SCORE_FP32),
                                    (33, 130, api.SCORE_BF16 | api.BF16_SPLIT3)]])
def test_noalloc_matches_fk_score(oracle_mod, dev, calls):
    arm = wl.arm_7dof()
    dh = oracle_dh(oracle_mod, arm)
    gamma = 10.0
    for k, (S, N, flags) in enumerate(calls):
        sq, al = wl.model(f"noalloc/{k}", S, arm.n)
        q = wl.configs(f"noalloc/{k}/q", N, arm.n)
        sq_d, al_d, q_d = (torch.from_numpy(x).to(dev) for x in (sq, al, q))
        announce(f"fk_score_noalloc call {k}: S={S} N={N} flags={flags:#x}")
        f_na, l_na = api.fk_score_noalloc(arm, sq_d, al_d, gamma, q_d, flags=flags)
        announce(f"fk_score call {k}: S={S} N={N} flags={flags:#x}")
        f_ref, l_ref = api.fk_score(arm, sq_d, al_d, gamma, q_d, flags=flags)
        torch.cuda.synchronize()
        assert torch.equal(f_na, f_ref)
        assert torch.equal(l_na, l_ref)
        if flags == api.SCORE_FP32:
            idx = np.unique(np.concatenate([wl.rng(f"noalloc/{k}/sample").choice(N, min(N, 400), replace=False),
                                            [0, N - 1]]))
            ref = oracle_mod.score(dh, arm.frames, sq.astype(np.float64), al.astype(np.float64), gamma,
                                   q[idx].astype(np.float64))
            tol = error_bound(oracle_mod.control_points(dh, arm.frames, sq.astype(np.float64)), al, gamma,
                              oracle_mod.control_points(dh, arm.frames, q[idx].astype(np.float64)))
            print(check_scores(f_na.cpu().numpy()[idx], l_na.cpu().numpy()[idx], ref, tol))


def test_noalloc_refuses_oversized_model(dev):
    arm = wl.arm_7dof()
    cap = nat.lib().fastron_model_bytes(1, 8)
    S = 1
    while nat.lib().fastron_model_bytes(S, 8) <= 16 << 20:
        S += 16
    assert cap > 0
    sq = torch.zeros(S, arm.n, dtype=torch.float32, device=dev)
    al = torch.zeros(S, dtype=torch.float32, device=dev)
    q = torch.zeros(8, arm.n, dtype=torch.float32, device=dev)
    with pytest.raises(nat.FastronError) as ei:
        api.fk_score_noalloc(arm, sq, al, 10.0, q)
    assert ei.value.status == nat.FASTRON_EINVAL
    assert "static buffer" in str(ei.value)
