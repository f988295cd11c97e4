"""Learned screening network: the device forward pass and gradients against
the FP64 oracle (same weights, same standardised inputs), training progress,
and the exact semantics of the tau-margin fallback to the Fastron score."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as mo
from paper_1910_06451_amd import api, workloads as wl
from conftest import announce, oracle_dh

pytestmark = pytest.mark.gpu


def _data(oracle_mod, N, name, n_cubes=20):
    arm = wl.arm_7dof()
    dh = oracle_dh(oracle_mod, arm)
    q = wl.configs(name, N, 7)
    lo, hi = wl.cubes("bench7/cubes", n_cubes, 0.1, 0.25)
    y, _ = oracle_mod.capsule_box_labels(dh, q.astype(np.float64), arm.radius, lo, hi)
    P = oracle_mod.control_points(dh, arm.frames, q.astype(np.float64)).astype(np.float32)
    return arm, q, P, y.astype(np.int8)


def test_forward_and_gradients_match_oracle(oracle_mod, dev):
    arm, q, P, y = _data(oracle_mod, 700, "mlp_grad")
    d_in = 24
    params = wl.mlp_init(d_in, 256, name="mlp_grad_init")
    X = P.reshape(-1, d_in).astype(np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd[sd < 1e-6] = 1.0
    mu32, sd32 = mu.astype(np.float32), sd.astype(np.float32)
    net = api.MLP(d_in, 256, max_rows=1024)
    net.set_params(torch.from_numpy(params).to(dev), torch.from_numpy(mu32).to(dev), torch.from_numpy(sd32).to(dev))
    P_d = torch.from_numpy(P).to(dev)
    announce("mlp forward")
    z = net.forward(P_d).cpu().numpy().astype(np.float64)
    announce("mlp gradients")
    loss = net.gradients(P_d, torch.from_numpy(y).to(dev))
    _, g, _, _ = net.get_params(dev)
    g = g.cpu().numpy().astype(np.float64)
    ps = [p.astype(np.float64) for p in wl.split_mlp_params(params, d_in)]
    z_ref, cache = mo.forward(ps, X, mu32.astype(np.float64), sd32.astype(np.float64))
    g_ref = mo.backward(ps, cache, z_ref, y)
    # BF16 operands: relative errors of order 2^-8 per product, averaged over 256-wide sums
    rel_z = np.linalg.norm(z - z_ref) / np.linalg.norm(z_ref)
    assert rel_z < 2e-2, rel_z
    assert abs(loss - mo.bce_loss(z_ref, y)) < 2e-2 * abs(mo.bce_loss(z_ref, y)) + 1e-3
    gs = wl.split_mlp_params(g, d_in)
    for k, (a, b) in enumerate(zip(gs, g_ref)):
        rel = np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-12)
        assert rel < 2e-2, (k, rel)
    net.close()


def test_training_learns(oracle_mod, dev):
    arm, q, P, y = _data(oracle_mod, 60000, "mlp_train")
    d_in = 24
    Ptr, ytr = torch.from_numpy(P[:50000]).to(dev), torch.from_numpy(y[:50000]).to(dev)
    Pte, yte = torch.from_numpy(P[50000:]).to(dev), y[50000:]
    net = api.MLP(d_in, 256, max_rows=4096)
    net.set_params(torch.from_numpy(wl.mlp_init(d_in, 256, name="mlp_train_init")).to(dev))
    net.fit_standardisation(Ptr)
    losses = []
    for ep in range(6):
        perm = torch.from_numpy(wl.rng(f"mlp_train/perm{ep}").permutation(50000).astype(np.int32)).to(dev)
        announce(f"mlp epoch {ep}")
        losses.append(net.train_epoch(Ptr, ytr, perm, batch=4096, lr=2e-3))
    z = net.forward(Pte).cpu().numpy()
    acc = np.mean(np.where(z >= 0, 1, -1) == yte)
    majority = max(np.mean(yte == 1), np.mean(yte == -1))
    print(dict(losses=losses, acc=float(acc), majority=float(majority)))
    assert losses[-1] < losses[0] * 0.8
    assert acc > majority + 0.05
    net.close()


@pytest.mark.parametrize("N", [1, 63, 3001])
def test_fused_screen_logits(oracle_mod, dev, N):
    """The fused screening pass (FK + both layers + head in one persistent kernel) against the staged GEMM
    forward on the same control points, and against the FP64 oracle; ragged sizes (one query, less than a
    wave, several tiles plus a partial one)."""
    arm = wl.arm_7dof()
    dh = oracle_dh(oracle_mod, arm)
    q = wl.configs(f"fused_screen/{N}", N, 7)
    q_d = torch.from_numpy(q).to(dev)
    P_d = api.fk_points(arm, q_d)
    params = wl.mlp_init(24, 256, name="fused_screen_init")
    params[24 * 256:24 * 256 + 256] = wl.rng("fused_screen/b1").normal(0, 0.1, 256)  # nonzero biases
    params[-257:-1] = wl.rng("fused_screen/w3").normal(0, 0.2, 256)
    P_stats = api.fk_points(arm, torch.from_numpy(wl.configs("fused_screen/stats", 4096, 7)).to(dev))
    net = api.MLP(24, 256, max_rows=4096)
    net.set_params(torch.from_numpy(params).to(dev))
    net.fit_standardisation(P_stats)
    sq, al = wl.model("fused_screen_model", 64, 7)
    model = api.support_prep(arm, torch.from_numpy(sq).to(dev), torch.from_numpy(al).to(dev), 10.0)
    announce(f"fused screen N={N}")
    lab, z, fb, nf = net.screen(arm, model, q_d, 0.0)
    announce(f"staged forward N={N}")
    z_st = net.forward(P_d)
    z, z_st = z.cpu().numpy().astype(np.float64), z_st.cpu().numpy().astype(np.float64)
    diff = np.linalg.norm(z - z_st) / max(np.linalg.norm(z_st), 1e-30)
    _, _, mu, sd = net.get_params(dev)
    ps = [p_.astype(np.float64) for p_ in wl.split_mlp_params(params, 24)]
    X = oracle_mod.control_points(dh, arm.frames, q.astype(np.float64)).reshape(N, 24)
    z_ref, _ = mo.forward(ps, X, mu.cpu().numpy().astype(np.float64), sd.cpu().numpy().astype(np.float64))
    rel = np.linalg.norm(z - z_ref) / max(np.linalg.norm(z_ref), 1e-30)
    print(dict(N=N, rel_vs_staged=float(diff), rel_vs_oracle=float(rel), max_abs_vs_staged=float(np.abs(z - z_st).max())))
    assert diff < 1e-3, diff
    assert rel < 2e-2, rel
    assert nf == 0
    assert np.array_equal(lab.cpu().numpy(), np.where(z >= 0, 1, -1).astype(np.int8))
    net.close()


@pytest.mark.parametrize("hidden", [256, 128])
def test_screen_semantics(oracle_mod, dev, hidden):
    """hidden = 256 runs the fused screening kernel, hidden = 128 the staged GEMM path."""
    arm = wl.arm_7dof()
    gamma = 10.0
    sq, al = wl.model("mlp_screen_model", 500, 7)
    q = wl.configs("mlp_screen/q", 3001, 7)
    sq_d, al_d, q_d = (torch.from_numpy(x).to(dev) for x in (sq, al, q))
    model = api.support_prep(arm, sq_d, al_d, gamma)
    _, plain = api.fk_score_prepared(arm, model, q_d)
    net = api.MLP(24, hidden, max_rows=1024)
    net.set_params(torch.from_numpy(wl.mlp_init(24, hidden, name="mlp_screen_init")).to(dev))
    net.fit_standardisation(api.fk_points(arm, q_d))
    announce(f"screen hidden={hidden} tau=0")
    lab0, z0, fb0, n0 = net.screen(arm, model, q_d, 0.0)
    assert n0 == 0 and int(fb0.sum()) == 0
    assert torch.equal(lab0, torch.where(z0 >= 0, 1, -1).to(torch.int8))
    announce("screen tau=inf")
    labi, zi, fbi, ni = net.screen(arm, model, q_d, 1e30)
    assert ni == 3001 and torch.equal(labi, plain)
    tau = float(torch.median(z0.abs()))
    announce("screen tau=median")
    lab, z, fb, nf = net.screen(arm, model, q_d, tau)
    expect_fb = (z.abs() < tau)
    assert torch.equal(fb.bool(), expect_fb) and nf == int(expect_fb.sum())
    assert torch.equal(lab[~expect_fb], torch.where(z[~expect_fb] >= 0, 1, -1).to(torch.int8))
    assert torch.equal(lab[expect_fb], plain[expect_fb])
    torch.testing.assert_close(z, z0, rtol=0, atol=0)
    net.close()


def test_screening_gain(oracle_mod, dev):
    """What the network adds to the plain method: on 400,000 queries of the 20-cube environment, the screened
    labels agree with the geometric labels at least as well as the plain Fastron model's, while only the
    uncertain fraction of queries pays for the Fastron score."""
    import time

    arm = wl.arm_7dof()
    lo, hi = wl.cubes("bench7/cubes", 20, 0.1, 0.25)
    q_tr = torch.from_numpy(wl.configs("gain/train", 300_000, 7)).to(dev)
    y_tr, _ = api.label_capsule_box(arm, q_tr, arm.radius, lo, hi, want_clearance=False)
    P_tr = api.fk_points(arm, q_tr)
    net = api.MLP(24, 256, max_rows=8192)
    net.set_params(torch.from_numpy(wl.mlp_init(24, 256, name="gain/init")).to(dev))
    net.fit_standardisation(P_tr)
    for ep in range(5):
        perm = torch.from_numpy(wl.rng(f"gain/perm{ep}").permutation(300_000).astype(np.int32)).to(dev)
        announce(f"gain: mlp epoch {ep}")
        net.train_epoch(P_tr, y_tr, perm, batch=8192, lr=2e-3)
    q20 = torch.from_numpy(wl.configs("gain/fastron", 20_000, 7)).to(dev)
    y20, _ = api.label_capsule_box(arm, q20, arm.radius, lo, hi, want_clearance=False)
    announce("gain: fastron fallback model")
    fit = api.train_points(api.fk_points(arm, q20), y20, 30.0, s_max=2000)
    sup = fit["support"].long()
    model = api.support_prep(arm, q20[sup].contiguous(), fit["alpha"][sup].contiguous(), 30.0)
    q = torch.from_numpy(wl.configs("gain/q", 400_000, 7)).to(dev)
    truth, _ = api.label_capsule_box(arm, q, arm.radius, lo, hi, want_clearance=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, plain = api.fk_score_prepared(arm, model, q, want_f=False)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    acc_plain = float((plain == truth).float().mean())
    announce("gain: screen tau=1")
    t0 = time.perf_counter()
    lab, z, fb, nfb = net.screen(arm, model, q, 1.0)
    t_screen = time.perf_counter() - t0
    acc_screen = float((lab == truth).float().mean())
    print(dict(acc_plain=acc_plain, acc_screen=acc_screen, fallback=nfb / 400_000, t_plain=t_plain,
               t_screen=t_screen, support=int(sup.numel())))
    assert acc_screen >= acc_plain - 0.01
    assert nfb < 0.6 * 400_000
    net.close()


def test_train_epoch_rejects_bad_order(dev):
    """The binding refuses an order array of the wrong length; an in-range-length order holding an index
    outside [0, N) is caught by the input kernel's guard and reported as FASTRON_EINVAL."""
    from paper_1910_06451_amd import _native

    arm = wl.arm_7dof()
    q = torch.from_numpy(wl.configs("bad_order", 300, 7)).to(dev)
    P = api.fk_points(arm, q)
    y = torch.ones(300, dtype=torch.int8, device=dev)
    net = api.MLP(24, 256, max_rows=256)
    net.set_params(torch.from_numpy(wl.mlp_init(24, 256, name="bad_order")).to(dev))
    with pytest.raises(ValueError):
        net.train_epoch(P, y, torch.arange(299, dtype=torch.int32, device=dev), batch=128)
    order = torch.arange(300, dtype=torch.int32, device=dev)
    order[7] = 300
    announce("mlp bad order index")
    with pytest.raises(_native.FastronError) as ei:
        net.train_epoch(P, y, order, batch=128)
    assert ei.value.status == _native.FASTRON_EINVAL
    net.close()


def test_screen_full_size_sampled(oracle_mod, dev):
    """The screening form's launch at full size (4,194,304 queries through the fused kernel, tau = 1 so that
    a fallback list forms): sampled logits against the FP64 oracle forward pass, labels of confident queries
    = sign(logit), labels of fallback queries = the Fastron label, fallback count = |logit| < tau."""
    arm = wl.arm_7dof()
    dh = oracle_dh(oracle_mod, arm)
    N = 4_194_304
    q = wl.configs("bench7/screen_q", N, arm.n)
    q_d = torch.from_numpy(q).to(dev)
    params = wl.mlp_init(24, 256, name="screen_full_init")
    net = api.MLP(24, 256, max_rows=8192)
    net.set_params(torch.from_numpy(params).to(dev))
    net.fit_standardisation(api.fk_points(arm, q_d[:65536].contiguous()))
    sq, al = wl.model("screen_full_model", 500, 7)
    model = api.support_prep(arm, torch.from_numpy(sq).to(dev), torch.from_numpy(al).to(dev), 10.0)
    announce("screen full size N=4194304 tau=1")
    lab, z, fb, nf = net.screen(arm, model, q_d, 1.0)
    zc = z.cpu().numpy()
    fbc = fb.cpu().numpy().astype(bool)
    assert nf == int(fbc.sum()) and np.array_equal(fbc, np.abs(zc) < 1.0)
    labc = lab.cpu().numpy()
    assert np.array_equal(labc[~fbc], np.where(zc[~fbc] >= 0, 1, -1).astype(np.int8))
    _, plain = api.fk_score_prepared(arm, model, q_d, want_f=False)
    assert np.array_equal(labc[fbc], plain.cpu().numpy()[fbc])
    idx = np.unique(np.concatenate([wl.rng("screen_full/sample").choice(N, 2000, replace=False), [0, N - 1]]))
    _, _, mu, sd = net.get_params(dev)
    ps = [p_.astype(np.float64) for p_ in wl.split_mlp_params(params, 24)]
    X = oracle_mod.control_points(dh, arm.frames, q[idx].astype(np.float64)).reshape(idx.size, 24)
    z_ref, _ = mo.forward(ps, X, mu.cpu().numpy().astype(np.float64), sd.cpu().numpy().astype(np.float64))
    rel = np.linalg.norm(zc[idx] - z_ref) / np.linalg.norm(z_ref)
    print(dict(fallback=nf / N, rel_vs_oracle=float(rel)))
    assert rel < 2e-2
    net.close()
