"""Learned screening network: the device forward pass and gradients against
the FP64 oracle (same weights, same standardised inputs), training progress,
and the exact semantics of the tau-margin fallback to the Fastron score."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as mo
import mlp_bounds as mb
from paper_1910_06451_amd import api, workloads as wl
from conftest import announce, oracle_dh

pytestmark = pytest.mark.gpu


def _arm9():
    """A 9-joint chain with a point on every frame: 10 points, 30 input features (the widest the three-kernel
    training step takes is 32)."""
    g = wl.rng("mlp_arm9")
    n = 9
    return wl.Arm(a=g.uniform(0.1, 0.25, size=n), alpha=g.choice(np.array([0.0, np.pi / 2, -np.pi / 2]), size=n),
                  d=np.zeros(n), theta=np.zeros(n), joint_type=np.zeros(n, dtype=np.int32),
                  frames=np.arange(n + 1, dtype=np.int32))


def _data(oracle_mod, N, name, n_cubes=20, arm=None):
    arm = arm if arm is not None else wl.arm_7dof()
    dh = oracle_dh(oracle_mod, arm)
    q = wl.configs(name, N, arm.n)
    lo, hi = wl.cubes("bench7/cubes", n_cubes, 0.1, 0.25)
    y, _ = oracle_mod.capsule_box_labels(dh, q.astype(np.float64), arm.radius, lo, hi)
    P = oracle_mod.control_points(dh, arm.frames, q.astype(np.float64)).astype(np.float32)
    return arm, q, P, y.astype(np.int8)


def _grad_setup(oracle_mod, dev, N, name, max_rows, H=256, arm=None):
    arm, q, P, y = _data(oracle_mod, N, name, arm=arm)
    d_in = 3 * arm.M
    params = wl.mlp_init(d_in, H, name=f"{name}_init")
    g = wl.rng(f"{name}/biases")
    params[d_in * H:d_in * H + H] = g.normal(0, 0.1, H)                   # b1
    o2 = d_in * H + H + H * H
    params[o2:o2 + H] = g.normal(0, 0.1, H)                               # b2
    params[-1] = 0.2                                                      # b3
    X = P.reshape(-1, d_in).astype(np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd[sd < 1e-6] = 1.0
    mu32, sd32 = mu.astype(np.float32), sd.astype(np.float32)
    net = api.MLP(d_in, H, max_rows=max_rows)
    net.set_params(torch.from_numpy(params).to(dev), torch.from_numpy(mu32).to(dev), torch.from_numpy(sd32).to(dev))
    ps = [p_.astype(np.float64) for p_ in wl.split_mlp_params(params, d_in, H)]
    return net, P, X, y, params, ps, mu32.astype(np.float64), sd32.astype(np.float64)


def _oracle_grads(ps, X, y, mu, sd, E_params=None):
    """The oracle's BF16 forms (bfloat16 rounding at the device's matrix-product operands, FP64 otherwise) and
    the per-element bounds on the device's logits and gradients against them (tests/mlp_bounds.py)."""
    z, cache = mo.forward_bf16(ps, X, mu, sd)
    g = mo.backward_bf16(ps, cache, z, y)
    fb = mb.forward_bounds(ps, cache, z, E_params)
    Eg, info = mb.gradient_bounds(ps, cache, z, y, fb)
    return z, g, fb, Eg, info


NAMES = ["gW1", "gb1", "gW2", "gb2", "gw3", "gb3"]


def ADAM_F32(lr):
    """The optimiser's hyperparameters as the library holds them (FP32 values), for the oracle's adam_step."""
    f = lambda x: float(np.float32(x))
    return dict(lr=f(lr), beta1=f(0.9), beta2=f(0.999), eps=f(1e-8))


def _forward_and_gradients(oracle_mod, dev, H, name, arm=None):
    net, P, X, y, params, ps, mu, sd = _grad_setup(oracle_mod, dev, 700, name, 1024, H, arm=arm)
    d_in = X.shape[1]
    P_d = torch.from_numpy(P).to(dev)
    announce(f"mlp forward d_in={d_in} H={H}")
    z = net.forward(P_d).cpu().numpy().astype(np.float64)
    announce(f"mlp gradients d_in={d_in} H={H}")
    loss = net.gradients(P_d, torch.from_numpy(y).to(dev))
    _, g, _, _ = net.get_params(dev)
    g = g.cpu().numpy().astype(np.float64)
    z_ref, g_ref, fb, Eg, info = _oracle_grads(ps, X, y, mu, sd)
    Ez = 1.25 * fb["E_z"]
    report = dict(info, d_in=d_in, z_ratio=float(np.max(np.abs(z - z_ref) / Ez)))
    assert np.all(np.abs(z - z_ref) <= Ez), np.max(np.abs(z - z_ref) / Ez)
    loss_ref = mo.bce_loss(z_ref, y)
    # BCE is 1-Lipschitz in z; the loss is summed in FP32 over 256-row blocks, then in FP64 on the host
    assert abs(loss - loss_ref) <= float(np.mean(Ez)) + 1e-5 * (abs(loss_ref) + 1.0)
    z64, c64 = mo.forward(ps, X, mu, sd)
    g64 = mo.backward(ps, c64, z64, y)
    report["logits_rel_l2_vs_fp64"] = float(np.linalg.norm(z - z64) / np.linalg.norm(z64))
    gs = wl.split_mlp_params(g, d_in, H)
    for k, (a, b, e) in enumerate(zip(gs, g_ref, Eg)):
        err = np.abs(np.ravel(a) - np.ravel(b))
        e = np.ravel(e)
        ratio = np.divide(err, e, out=np.zeros_like(err), where=e > 0)
        nz = np.abs(np.ravel(b)) > 0
        report[NAMES[k]] = dict(max_ratio=float(np.max(ratio)), median_bound_over_abs=float(
            np.median(e[nz] / np.abs(np.ravel(b))[nz])), rel_l2_vs_fp64=float(
            np.linalg.norm(np.ravel(a) - np.ravel(g64[k])) / max(np.linalg.norm(np.ravel(g64[k])), 1e-30)))
        assert np.all(err <= e), (NAMES[k], float(np.max(ratio)))
    print(report)
    net.close()


@pytest.mark.parametrize("H", [256, 128])
def test_forward_and_gradients_match_oracle(oracle_mod, dev, H):
    """Forward logits, loss and all six gradients of one batch against the oracle, element by element: the
    oracle's BF16 forms round to bfloat16 where the device does, and every difference must lie within the bound
    propagated from the device's FP32 arithmetic, the bfloat16 roundings that this arithmetic can tip and the
    ReLU decisions it can flip (tests/mlp_bounds.py). Nonzero biases, so that every bias path carries weight.
    Also reported: the relative L2 distance to the unrounded FP64 network. Hidden width 256 runs the
    three-kernel training step, 128 the staged GEMM path."""
    _forward_and_gradients(oracle_mod, dev, H, "mlp_grad")


@pytest.mark.parametrize("which", ["3dof", "9joint"])
def test_forward_and_gradients_other_input_widths(oracle_mod, dev, which):
    """The same element-by-element check at the other input widths of the three-kernel training step: 12
    features (the 3-DOF arm's 4 points) and 30 (a 9-joint chain's 10 points), where the zero padding of the
    32-wide layer-1 operand and the standardisation's feature bound matter."""
    arm = wl.arm_3dof() if which == "3dof" else _arm9()
    _forward_and_gradients(oracle_mod, dev, 256, f"mlp_grad_{which}", arm=arm)


@pytest.mark.parametrize("H", [256, 128])
def test_adam_first_step_matches_oracle(oracle_mod, dev, H):
    """One batch of train_epoch (a fixed row order, lr = 1e-3) against the oracle's forward -> backward ->
    adam_step, element by element: at step 1, m = (1 - beta1) g, v = (1 - beta2) g^2 and the update is
    lr g / (|g| + eps), so each bound follows from the gradient's bound."""
    net, P, X, y, params, ps, mu, sd = _grad_setup(oracle_mod, dev, 1000, "mlp_adam1", 1024, H)
    order = wl.rng("mlp_adam1/order").permutation(1000).astype(np.int32)
    lr = 1e-3
    announce("mlp one Adam step")
    net.train_epoch(torch.from_numpy(P).to(dev), torch.from_numpy(y).to(dev), torch.from_numpy(order).to(dev),
                    batch=1000, lr=lr)
    p1, _, _, _ = net.get_params(dev)
    m1, v1, step = net.adam_state(dev)
    assert step == 1
    p1, m1, v1 = (t.cpu().numpy().astype(np.float64) for t in (p1, m1, v1))
    _, g_ref, _, Eg, _ = _oracle_grads(ps, X[order], y[order], mu, sd)
    zeros = [np.zeros_like(x) for x in ps]
    new_p, new_m, new_v = mo.adam_step(ps, g_ref, zeros, zeros, 1, **ADAM_F32(lr))
    cat = lambda xs: np.concatenate([np.ravel(x) for x in xs])
    g_r, E, p_r, m_r, v_r, p0 = cat(g_ref), cat(Eg), cat(new_p), cat(new_m), cat(new_v), cat(ps)
    Em = 0.1 * E + 4 * mb.U32 * np.abs(m_r)
    Ev = 1e-3 * (2 * np.abs(g_r) * E + E * E) + 8 * mb.U32 * np.abs(v_r)
    Ep = lr * mb.adam_direction_bound(g_r, E) + 2 * mb.U32 * (np.abs(p0) + lr) + 16 * mb.U32 * lr
    for name, dv, rv, eb in (("m", m1, m_r, Em), ("v", v1, v_r, Ev), ("params", p1, p_r, Ep)):
        err = np.abs(dv - rv)
        ratio = np.divide(err, eb, out=np.zeros_like(err), where=eb > 0)
        print(name, "max error / bound", float(np.max(ratio)), "elements with bound < 1% of value",
              float(np.mean(eb < 0.01 * np.abs(rv))))
        assert np.all(err <= eb), (name, float(np.max(ratio)), int(np.argmax(ratio)))
    # the update moved (almost) every weight by lr: a wrong learning rate or sign would show here
    assert np.mean(np.abs(np.abs(p1 - p0) - lr) < 0.01 * lr) > 0.9
    net.close()


def test_adam_three_steps_match_oracle(oracle_mod, dev):
    """Three Adam steps against the oracle, element by element. Steps 1 and 2 (one train_epoch call over two
    batches) use lr = 1e-12, too small to change any FP32 weight above 1e-4 in magnitude, so the moments build
    up while the device and the oracle keep the same parameters; step 3 (a second call, the step count carries
    over) uses lr = 1e-3. Compared: m and v after step 3 and the step-3 displacement / lr, which is
    m_hat / (sqrt(v_hat) + eps) with the bias corrections 1 - beta^3: a wrong power or a step count that
    restarts changes it by tens of percent where its bound is a few percent."""
    B = 512
    net, P, X, y, params, ps, mu, sd = _grad_setup(oracle_mod, dev, 3 * B, "mlp_adam3", B)
    lr12, lr3 = 1e-12, 1e-3
    o12 = wl.rng("mlp_adam3/order12").permutation(2 * B).astype(np.int32)
    o3 = wl.rng("mlp_adam3/order3").permutation(B).astype(np.int32)
    announce("mlp Adam steps 1-2")
    net.train_epoch(torch.from_numpy(P[:2 * B]).to(dev), torch.from_numpy(y[:2 * B]).to(dev),
                    torch.from_numpy(o12).to(dev), batch=B, lr=lr12)
    announce("mlp Adam step 3")
    net.train_epoch(torch.from_numpy(P[2 * B:]).to(dev), torch.from_numpy(y[2 * B:]).to(dev),
                    torch.from_numpy(o3).to(dev), batch=B, lr=lr3)
    p3, _, _, _ = net.get_params(dev)
    m3, v3, step = net.adam_state(dev)
    assert step == 3
    cat = lambda xs: np.concatenate([np.ravel(x) for x in xs])
    p3, m3, v3 = (t.cpu().numpy().astype(np.float64) for t in (p3, m3, v3))
    hp = ADAM_F32(lr12)
    b1, b2, eps = hp["beta1"], hp["beta2"], hp["eps"]
    shapes = [np.shape(x) for x in ps]
    offs = np.cumsum([int(np.prod(sh)) for sh in shapes])[:-1]
    split = lambda flat: [a.reshape(sh) for a, sh in zip(np.split(flat, offs), shapes)]
    p, m, v = ps, [np.zeros_like(x) for x in ps], [np.zeros_like(x) for x in ps]
    n = p3.size
    Em, Ev = np.zeros(n), np.zeros(n)
    mag_m, mag_v = np.zeros(n), np.zeros(n)   # sums of the magnitudes that the FP32 moment updates round
    X12, y12 = X[:2 * B][o12], y[:2 * B][o12]
    batches = [(X12[:B], y12[:B], lr12), (X12[B:], y12[B:], lr12), (X[2 * B:][o3], y[2 * B:][o3], lr3)]
    drift = np.zeros(n)  # how far the device's weights may be from the oracle's before each step
    for k, (Xk, yk, lr) in enumerate(batches):
        _, g_k, _, Eg, _ = _oracle_grads(p, Xk, yk, mu, sd, split(drift))
        p, m, v = mo.adam_step(p, g_k, m, v, k + 1, **ADAM_F32(lr))
        g, E = cat(g_k), cat(Eg)
        mag_m = b1 * mag_m + (1 - b1) * (np.abs(g) + E)
        mag_v = b2 * mag_v + (1 - b2) * (np.abs(g) + E) ** 2
        Em = b1 * Em + (1 - b1) * E + 3 * mb.U32 * mag_m
        Ev = b2 * Ev + (1 - b2) * (2 * np.abs(g) * E + E * E) + 4 * mb.U32 * mag_v
        # each side moves by at most lr * cap; the device also rounds its weights to FP32
        drift = drift + 2 * lr * mb.adam_ratio_cap(k + 1, b1, b2) + 2 * mb.U32 * np.abs(cat(p))
    c1, c2 = 1 / (1 - b1 ** 3), 1 / (1 - b2 ** 3)
    E_ratio = mb.adam_ratio_bound(cat(m) * c1, (Em + 2 * mb.U32 * mag_m) * c1, cat(v) * c2,
                                  (Ev + 2 * mb.U32 * mag_v) * c2, eps, cap=mb.adam_ratio_cap(3, b1, b2))
    p0, m_r, v_r = cat(ps), cat(m), cat(v)
    disp_dev, disp_ref = (p3 - p0) / lr3, (cat(p) - p0) / lr3
    # steps 1-2 (at most 2 lr12 cap each side), FP32 arithmetic of the update and the rounding of the write
    Ed = E_ratio + 16 * mb.U32 + 4 * lr12 * 3.2 / lr3 + 2 * mb.U32 * (np.abs(p0) + 4 * lr3) / lr3
    for name, dv, rv, eb in (("m", m3, m_r, Em), ("v", v3, v_r, Ev), ("displacement", disp_dev, disp_ref, Ed)):
        err = np.abs(dv - rv)
        ratio = np.divide(err, eb, out=np.zeros_like(err), where=eb > 0)
        print(name, "max error / bound", float(np.max(ratio)), "median bound", float(np.median(eb)),
              "elements with bound < 5% of value", float(np.mean(eb < 0.05 * np.abs(rv))))
        assert np.all(err <= eb), (name, float(np.max(ratio)), int(np.argmax(ratio)))
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


@pytest.mark.parametrize("which,N", [("7dof", 1), ("7dof", 63), ("7dof", 3001), ("3dof", 3001)],
                         ids=["7dof-1", "7dof-63", "7dof-3001", "3dof-3001"])
def test_fused_screen_logits(oracle_mod, dev, which, N):
    """The fused screening pass (FK + both layers + head in one persistent kernel) against the staged GEMM
    forward on the same control points, and against the FP64 oracle; ragged sizes (one query, less than a
    wave, several tiles plus a partial one), 24 input features (7-DOF arm) and 12 (3-DOF arm, FP32 chain)."""
    arm = wl.arm_7dof() if which == "7dof" else wl.arm_3dof()
    d_in = 3 * arm.M
    dh = oracle_dh(oracle_mod, arm)
    q = wl.configs(f"fused_screen/{which}/{N}", N, arm.n)
    q_d = torch.from_numpy(q).to(dev)
    P_d = api.fk_points(arm, q_d)
    params = wl.mlp_init(d_in, 256, name=f"fused_screen_init_{which}")
    params[d_in * 256:d_in * 256 + 256] = wl.rng(f"fused_screen/b1/{which}").normal(0, 0.1, 256)  # nonzero biases
    params[-257:-1] = wl.rng(f"fused_screen/w3/{which}").normal(0, 0.2, 256)
    P_stats = api.fk_points(arm, torch.from_numpy(wl.configs(f"fused_screen/stats/{which}", 4096, arm.n)).to(dev))
    net = api.MLP(d_in, 256, max_rows=4096)
    net.set_params(torch.from_numpy(params).to(dev))
    net.fit_standardisation(P_stats)
    sq, al = wl.model(f"fused_screen_model_{which}", 64, arm.n)
    model = api.support_prep(arm, torch.from_numpy(sq).to(dev), torch.from_numpy(al).to(dev), 10.0)
    announce(f"fused screen {which} N={N}")
    lab, z, fb, nf = net.screen(arm, model, q_d, 0.0)
    announce(f"staged forward {which} N={N}")
    z_st = net.forward(P_d)
    z, z_st = z.cpu().numpy().astype(np.float64), z_st.cpu().numpy().astype(np.float64)
    diff = np.linalg.norm(z - z_st) / max(np.linalg.norm(z_st), 1e-30)
    _, _, mu, sd = net.get_params(dev)
    ps = [p_.astype(np.float64) for p_ in wl.split_mlp_params(params, d_in)]
    X = oracle_mod.control_points(dh, arm.frames, q.astype(np.float64)).reshape(N, d_in)
    z_ref, _ = mo.forward(ps, X, mu.cpu().numpy().astype(np.float64), sd.cpu().numpy().astype(np.float64))
    rel = np.linalg.norm(z - z_ref) / max(np.linalg.norm(z_ref), 1e-30)
    print(dict(which=which, N=N, rel_vs_staged=float(diff), rel_vs_oracle=float(rel),
               max_abs_vs_staged=float(np.abs(z - z_st).max())))
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
    """What the network adds to the plain method, on 400,000 queries of the 20-cube environment: at tau = 0.5
    and tau = 1 the screened labels agree with the geometric labels better than the plain Fastron model's, and
    the screened pass (FK + network + the Fastron score of the uncertain queries only) takes less device time
    than scoring every query with the Fastron model (HIP events, median of 5)."""
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

    def event_ms(fn, reps=5):
        fn()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        return float(np.median(times))

    announce("gain: plain Fastron score")
    _, plain = api.fk_score_prepared(arm, model, q, want_f=False)
    acc_plain = float((plain == truth).float().mean())
    t_plain = event_ms(lambda: api.fk_score_prepared(arm, model, q, want_f=False))
    res = dict(acc_plain=acc_plain, t_plain_ms=t_plain, support=int(sup.numel()))
    for tau in (0.5, 1.0):
        announce(f"gain: screen tau={tau}")
        lab, z, fb, nfb = net.screen(arm, model, q, tau)
        acc = float((lab == truth).float().mean())
        t = event_ms(lambda: net.screen(arm, model, q, tau))
        res[f"tau{tau}"] = dict(acc=acc, fallback=nfb / 400_000, ms=t)
        assert acc > acc_plain, (tau, acc, acc_plain)
        assert nfb < 0.6 * 400_000
    print(res)
    assert res["tau0.5"]["ms"] < t_plain, res
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
