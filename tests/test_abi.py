"""The C ABI without a GPU: the library loads, exports exactly the entry
points that include/fastron_fk.h declares, the header compiles as C and C++,
and host-side validation rejects bad arguments before any device work.
Also checks the library's control-point placement rule (host code, Section
III-A) against the oracle's."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1910_06451_amd import _native as nat
from paper_1910_06451_amd import workloads as wl
from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "fastron_fk.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fastron_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(nat.LIB_PATH):
        from paper_1910_06451_amd import build

        build.build()
    return nat.lib()


def test_header_declares_what_the_binding_marshals():
    assert declared_functions() == sorted(nat.EXPORTED)


@pytest.mark.parametrize("lang,std", [("c", "-std=c99"), ("c++", "-std=c++17")])
def test_header_compiles(tmp_path, lang, std):
    src = tmp_path / ("t.c" if lang == "c" else "t.cpp")
    src.write_text('#include "fastron_fk.h"\nint main(void) { return (int)FASTRON_OK; }\n')
    cc = "gcc" if lang == "c" else "g++"
    subprocess.run([cc, std, "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.dirname(HEADER),
                    "-fsyntax-only", str(src)], check=True)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", nat.LIB_PATH], check=True, capture_output=True,
                         text=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if re.search(r" T fastron_", ln)})
    assert exported == declared_functions()


def test_host_only_entry_points(lib):
    assert lib.fastron_version().decode().startswith("fastron-fk")
    assert lib.fastron_tune_get(b"train.threads") in (256, 512, 1024)
    assert lib.fastron_tune_get(b"no.such.key") == -1
    assert lib.fastron_tune_set(b"no.such.key", 1) == nat.FASTRON_EINVAL
    assert "no.such.key" in nat.last_error()
    assert lib.fastron_tune_set(b"train.threads", 300) == nat.FASTRON_EINVAL
    # wave form of Algorithm 1: waves per workgroup (power of two up to 16), first-poll delay (-1 adaptive)
    assert lib.fastron_tune_get(b"train.waves") == 8
    assert lib.fastron_tune_get(b"train.poll_delay") == -1
    assert lib.fastron_tune_set(b"train.waves", 6) == nat.FASTRON_EINVAL
    assert lib.fastron_tune_set(b"train.waves", 32) == nat.FASTRON_EINVAL
    assert lib.fastron_tune_set(b"train.poll_delay", -2) == nat.FASTRON_EINVAL
    assert lib.fastron_tune_set(b"train.poll_delay", 65) == nat.FASTRON_EINVAL
    assert lib.fastron_tune_set(b"train.poll_delay", 12) == nat.FASTRON_OK
    assert lib.fastron_tune_set(b"train.poll_delay", -1) == nat.FASTRON_OK
    # one workgroup for a set that fits 16 waves (1) or the grid rule alone (0)
    assert lib.fastron_tune_get(b"train.single_group") == 1
    assert lib.fastron_tune_set(b"train.single_group", 2) == nat.FASTRON_EINVAL
    assert lib.fastron_tune_set(b"train.single_group", 0) == nat.FASTRON_OK
    assert lib.fastron_tune_set(b"train.single_group", 1) == nat.FASTRON_OK
    assert lib.fastron_model_bytes(-1, 8) == -1
    assert lib.fastron_model_bytes(4000, 17) == -1
    assert lib.fastron_model_bytes(4000, 8) > 4000 * 8 * 4


def test_validation_before_device_work(lib):
    arm = wl.arm_7dof()
    hc = nat.HostChain(arm)
    ch, cp = ctypes.byref(hc.chain), ctypes.byref(hc.cpoints)
    vp = ctypes.c_void_p
    # N == 0 is a no-op that needs no device
    assert lib.fastron_fk_points(ch, cp, None, 0, None, None) == nat.FASTRON_OK
    assert nat.last_error() == ""
    assert lib.fastron_fk_points(None, cp, None, 0, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_fk_points(ch, cp, None, -1, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_fk_points(ch, cp, None, 5, None, None) == nat.FASTRON_EINVAL
    bad = nat.CPoints(1, (ctypes.c_int32 * 1)(8), None)  # frame 8 > n = 7
    assert lib.fastron_fk_points(ch, ctypes.byref(bad), None, 0, None, None) == nat.FASTRON_EINVAL
    many = nat.CPoints(17, (ctypes.c_int32 * 17)(*([1] * 17)), None)
    assert lib.fastron_fk_points(ch, ctypes.byref(many), None, 0, None, None) == nat.FASTRON_EINVAL
    zero_n = nat.Chain(0, hc.chain.a, hc.chain.alpha, hc.chain.d, None, None, None)
    assert lib.fastron_fk_points(ctypes.byref(zero_n), cp, None, 0, None, None) == nat.FASTRON_EINVAL
    ns, up = ctypes.c_int64(0), ctypes.c_int64(0)
    fake = vp(256)  # never dereferenced: validation fails first
    args = lambda beta, s_max, gamma=10.0: (fake, fake, 100, 8, gamma, beta, 10, s_max, fake, fake, fake,
                                            ctypes.byref(ns), ctypes.byref(up), None, None, 0, None)
    assert lib.fastron_train_points(*args(0.5, 10)) == nat.FASTRON_EINVAL  # beta < 1 (Eq. 5)
    assert "beta" in nat.last_error()
    assert lib.fastron_train_points(*args(1.0, 0)) == nat.FASTRON_EINVAL  # s_max < 1
    assert lib.fastron_train_points(*args(1.0, 10, gamma=0.0)) == nat.FASTRON_EINVAL
    assert lib.fastron_train_points(*args(1.0, 10, gamma=float("nan"))) == nat.FASTRON_EINVAL
    assert lib.fastron_gram_update_points(fake, 100, 8, 10.0, 100, 1.0, fake, None, None) == nat.FASTRON_EINVAL
    # the configuration forms validate the chain and every argument before their FK scratch is allocated
    xargs = lambda beta, s_max, gamma=10.0, chain=ch: (chain, cp, fake, fake, 100, gamma, beta, 10, s_max, fake,
                                                       fake, fake, ctypes.byref(ns), ctypes.byref(up), None, None,
                                                       0, None)
    assert lib.fastron_train(*xargs(0.5, 10)) == nat.FASTRON_EINVAL
    assert "beta" in nat.last_error()
    assert lib.fastron_train(*xargs(1.0, 0)) == nat.FASTRON_EINVAL
    assert lib.fastron_train_f64(*xargs(1.0, 10, gamma=0.0)) == nat.FASTRON_EINVAL
    assert lib.fastron_train(*xargs(1.0, 10, chain=None)) == nat.FASTRON_EINVAL
    assert lib.fastron_train(ch, cp, None, fake, 100, 10.0, 1.0, 10, 10, fake, fake, fake, ctypes.byref(ns),
                             ctypes.byref(up), None, None, 0, None) == nat.FASTRON_EINVAL  # X NULL
    assert lib.fastron_gram_update(ch, cp, fake, 100, 10.0, 100, 1.0, fake, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_gram_update(ch, cp, fake, 100, 10.0, 5, 1.0, None, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_gram_update(None, cp, fake, 100, 10.0, 5, 1.0, fake, None, None) == nat.FASTRON_EINVAL
    # the kernel on configurations
    assert lib.fastron_rbf_score(None, None, 0, 7, 1.0, None, 0, None, None, None) == nat.FASTRON_OK  # N = 0
    assert lib.fastron_rbf_score(fake, fake, 10, 0, 1.0, fake, 10, fake, None, None) == nat.FASTRON_EINVAL  # n < 1
    assert lib.fastron_rbf_score(fake, fake, 10, 17, 1.0, fake, 10, fake, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_rbf_score(fake, fake, 10, 7, -1.0, fake, 10, fake, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_rbf_score(None, None, 10, 7, 1.0, fake, 10, fake, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_rbf_score(fake, fake, 10, 7, 1.0, fake, 10, None, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_rbf_train(fake, fake, 100, 0, 1.0, 1.0, 10, 10, fake, fake, fake, ctypes.byref(ns),
                                 ctypes.byref(up), None) == nat.FASTRON_EINVAL
    assert lib.fastron_rbf_train(fake, fake, 100, 7, 1.0, 0.5, 10, 10, fake, fake, fake, ctypes.byref(ns),
                                 ctypes.byref(up), None) == nat.FASTRON_EINVAL  # beta < 1
    assert lib.fastron_rbf_train_f64(fake, fake, 100, 7, 0.0, 1.0, 10, 10, fake, fake, fake, ctypes.byref(ns),
                                     ctypes.byref(up), None, None, 0, None) == nat.FASTRON_EINVAL
    # the scoring form that allocates nothing refuses a model too large for its static buffer up front
    S_big = 1
    while lib.fastron_model_bytes(S_big, 8) <= 16 << 20:
        S_big += 16
    assert lib.fastron_fk_score_noalloc(ch, cp, fake, fake, S_big, 10.0, fake, 10, fake, None, 0,
                                        None) == nat.FASTRON_EINVAL
    assert "static buffer" in nat.last_error()
    assert lib.fastron_fk_score_noalloc(ch, cp, fake, fake, 100, 0.0, fake, 10, fake, None, 0,
                                        None) == nat.FASTRON_EINVAL
    assert lib.fastron_fk_score_noalloc(ch, cp, None, None, 0, 10.0, None, 0, None, None, 0,
                                        None) == nat.FASTRON_OK  # N = 0
    # the batched form's launch shape: only the tuned candidates are accepted (checked before any device work)
    assert lib.fastron_batch_set_shape(None, 32, 4, 0, 100, None) == nat.FASTRON_EINVAL
    assert lib.fastron_batch_get_shape(None, None, None, None, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_active_relabel(None, 0, None, None) == nat.FASTRON_OK  # S = 0
    assert lib.fastron_active_relabel(None, 5, None, None) == nat.FASTRON_EINVAL
    # active-learning assembly
    assert lib.fastron_active_samples(None, None, 0, 7, None, 0, None, 0, None, None, None) == nat.FASTRON_OK
    assert lib.fastron_active_samples(fake, fake, 10, 7, None, 2, None, 0, fake, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_active_samples(fake, fake, 10, 7, fake, 2, None, 5, fake, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_active_samples(fake, fake, 10, 7, fake, 2, fake, 5, None, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_active_samples(fake, fake, -1, 7, fake, 2, fake, 5, fake, None, None) == nat.FASTRON_EINVAL
    # one launch spans at most 2^32 - 1 work-items per grid dimension: 2^32 - 256 configurations (256 per
    # workgroup of 256), 2^31 - 128 queries for the FK-kernel score (128 per workgroup of 256)
    big = 2 ** 32 - 255
    assert lib.fastron_fk_points(ch, cp, fake, big, fake, None) == nat.FASTRON_EINVAL
    assert "2^32 - 256" in nat.last_error()
    assert lib.fastron_label_capsule_box(ch, fake, big, 0.04, fake, 1, fake, None, None) == nat.FASTRON_EINVAL
    assert lib.fastron_rbf_score(fake, fake, 10, 7, 1.0, fake, big, fake, None, None) == nat.FASTRON_EINVAL
    model = nat.Model(100, hc.cpoints.M, 10.0, fake, lib.fastron_model_bytes(100, hc.cpoints.M))
    assert lib.fastron_fk_score_prepared(ch, cp, ctypes.byref(model), fake, 2 ** 31 - 127, fake, None, 0,
                                         None) == nat.FASTRON_EINVAL
    assert "2^31 - 128" in nat.last_error()
    assert lib.fastron_fk_score(ch, cp, fake, fake, 100, 10.0, fake, 2 ** 31 - 127, fake, None, 0,
                                None) == nat.FASTRON_EINVAL


def _frames_lib(lib, a, d, types, include_base):
    n = len(a)
    a = np.asarray(a, np.float64)
    d = np.asarray(d, np.float64)
    z = np.zeros(n)
    t = np.asarray(types, np.int32)
    dp = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    chain = nat.Chain(n, dp(a), dp(z), dp(d), None, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None)
    out = (ctypes.c_int32 * (n + 1))()
    M = ctypes.c_int32(0)
    assert lib.fastron_control_point_frames(ctypes.byref(chain), int(include_base), out, ctypes.byref(M)) == 0
    return list(out[:M.value])


def test_control_point_frames_match_oracle(lib, oracle_mod):
    # hand case: joint 2 is revolute with a = d = 0 (dropped); joint 4 is prismatic with a = d = 0 (kept)
    a, d, types = [0.3, 0.0, 0.2, 0.0], [0.0, 0.0, 0.1, 0.0], [0, 0, 0, 1]
    assert _frames_lib(lib, a, d, types, True) == [0, 1, 3, 4]
    assert _frames_lib(lib, a, d, types, False) == [1, 3, 4]
    g = wl.rng("abi/frames")
    for _ in range(50):
        n = int(g.integers(1, 17))
        a = np.where(g.random(n) < 0.4, 0.0, g.uniform(0.1, 0.5, n))
        d = np.where(g.random(n) < 0.5, 0.0, g.uniform(-0.3, 0.3, n))
        types = (g.random(n) < 0.2).astype(np.int32)
        for inc in (False, True):
            ref = oracle_mod.control_point_frames(oracle_mod.dh_table(a, np.zeros(n), d, None, types), inc)
            assert _frames_lib(lib, a, d, types, inc) == list(ref)


def test_constructor_validation(lib):
    """Batch and network constructors reject bad arguments before touching a device."""
    arm = wl.arm_7dof()
    hc = nat.HostChain(arm)
    h = ctypes.c_void_p()
    so = (ctypes.c_int64 * 3)(0, 10, 5)  # decreasing
    qo = (ctypes.c_int64 * 3)(0, 4, 8)
    assert lib.fastron_batch_create(ctypes.byref(hc.chain), ctypes.byref(hc.cpoints), 2, so, qo, 10.0,
                                    ctypes.byref(h)) == nat.FASTRON_EINVAL
    assert "decreases" in nat.last_error()
    so_ok = (ctypes.c_int64 * 3)(0, 10, 15)
    assert lib.fastron_batch_create(ctypes.byref(hc.chain), ctypes.byref(hc.cpoints), 2, so_ok, qo, -1.0,
                                    ctypes.byref(h)) == nat.FASTRON_EINVAL
    assert lib.fastron_batch_create(ctypes.byref(hc.chain), ctypes.byref(hc.cpoints), 0, so_ok, qo, 10.0,
                                    ctypes.byref(h)) == nat.FASTRON_EINVAL
    assert not h.value
    for d_in, hidden, rows in ((0, 256, 16), (24, 17, 16), (24, 256, 0), (49, 256, 16)):
        assert lib.fastron_mlp_create(d_in, hidden, rows, ctypes.byref(h)) == nat.FASTRON_EINVAL, (d_in, hidden, rows)
    assert lib.fastron_mlp_screen_workspace_bytes(-1, 7) == -1
    assert lib.fastron_mlp_param_count(None) == -1


def test_score_form_choice(lib):
    """Host-side choice between the running-fraction and the saturated-reciprocal sums. For the 7-DOF arm
    (revolute, d = 0) the reach bound is R = sum_i a_i, so T = 1.01 (1 + 2 gamma R^2) can be worked out by
    hand: the fraction is taken iff T <= 2^16 (2^8 for plain BF16) and 2 Mm log2(T) <= 120 with Mm = 7."""
    from paper_1910_06451_amd import api

    arm = wl.arm_7dof()
    R = float(np.sum(np.hypot(arm.a, arm.d)))

    def expect(gamma, t_limit):
        T = 1.01 * (1.0 + 2.0 * gamma * R * R)
        return T <= t_limit and 2 * 7 * np.log2(T) <= 120.0

    for gamma in (0.01, 1.0, 10.0, 40.0, 100.0, 1e4):
        assert api.score_rational(arm, gamma) == expect(gamma, 65536.0), gamma
        assert api.score_rational(arm, gamma, api.SCORE_BF16 | api.BF16_SPLIT3) == expect(gamma, 65536.0), gamma
        assert api.score_rational(arm, gamma, api.SCORE_BF16) == expect(gamma, 256.0), gamma
        assert api.score_rational(arm, gamma, api.SCORE_VALU) == expect(gamma, 65536.0), gamma
    # the cases that separate the limits
    assert api.score_rational(arm, 10.0) and api.score_rational(arm, 10.0, api.SCORE_BF16)
    assert api.score_rational(arm, 40.0) and not api.score_rational(arm, 40.0, api.SCORE_BF16)
    assert not api.score_rational(arm, 100.0)
    # a prismatic joint before a moving point: no finite reach bound
    pr = wl.Arm(a=arm.a, alpha=arm.alpha, d=arm.d, theta=arm.theta,
                joint_type=np.array([0, 0, 1, 0, 0, 0, 0], dtype=np.int32), frames=arm.frames)
    assert not api.score_rational(pr, 10.0)
    # ... but one after the last moving point does not matter
    pr_tail = wl.Arm(a=arm.a, alpha=arm.alpha, d=arm.d, theta=arm.theta,
                     joint_type=np.array([0, 0, 0, 0, 0, 0, 1], dtype=np.int32),
                     frames=np.arange(7, dtype=np.int32))
    assert api.score_rational(pr_tail, 10.0)
    # a base transform adds its translation to the reach and scales it by the norm of its matrix (a
    # rotation: exactly 1): with R = |p_base| + s sum_i a_i, gamma = 28 separates the cases
    import types

    def with_base(Bm, p):
        T4 = np.eye(4)
        T4[:3, :3], T4[:3, 3] = Bm, p
        return types.SimpleNamespace(a=arm.a, alpha=arm.alpha, d=arm.d, theta=arm.theta, joint_type=arm.joint_type,
                                     frames=arm.frames, offsets=None, base=T4)

    def t_ok(Rr, gamma):
        T = 1.01 * (1.0 + 2.0 * gamma * Rr * Rr)
        return T <= 65536.0 and 14 * np.log2(T) <= 120.0

    cz, sz, cx, sx = np.cos(0.7), np.sin(0.7), np.cos(0.3), np.sin(0.3)
    rot = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]]) @ np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    p = np.array([0.3, -0.2, 0.5])
    assert t_ok(R, 28.0) and not t_ok(np.linalg.norm(p) + R, 28.0) and t_ok(np.linalg.norm(p) + R, 25.0)
    assert api.score_rational(arm, 28.0)
    assert not api.score_rational(with_base(rot, p), 28.0)
    assert api.score_rational(with_base(rot, p), 25.0)
    assert api.score_rational(with_base(rot, np.zeros(3)), 28.0)  # a pure rotation leaves the bound alone
    assert not t_ok(np.linalg.norm(p) + 2 * R, 10.0)
    assert not api.score_rational(with_base(2 * np.eye(3), p), 10.0)  # a scaling base matrix counts
    # the tuning key switches the form off
    try:
        api.tune_set("score.rational", 0)
        assert not api.score_rational(arm, 10.0)
    finally:
        api.tune_set("score.rational", 1)
    assert lib.fastron_score_rational(None, None, ctypes.c_float(10.0), 0) == nat.FASTRON_EINVAL
    with pytest.raises(Exception):
        api.score_rational(arm, -1.0)
    with pytest.raises(Exception):
        api.score_rational(arm, 10.0, 0x40)


def test_label_binding_rejects_inverted_boxes():
    """The labeller's bounding-box culling assumes lo <= hi on every axis; the binding checks the host-side
    corners before any device work (the C entry point cannot read the device array on the host)."""
    import torch
    from paper_1910_06451_amd import api
    arm = wl.arm_7dof()
    q = torch.zeros((4, arm.n), dtype=torch.float32)
    lo = np.array([[0.0, 0.0, 0.0], [0.2, 0.1, 0.0]])
    hi = np.array([[0.1, 0.1, 0.1], [0.1, 0.3, 0.2]])  # second box inverted along x
    with pytest.raises(ValueError, match="lo <= hi"):
        api.label_capsule_box(arm, q, arm.radius, lo, hi)
    with pytest.raises(ValueError, match="lo <= hi"):
        api.label_capsule_box(arm, q, arm.radius, lo[:1], hi)
    with pytest.raises(ValueError, match="lo <= hi"):
        api.label_capsule_box(arm, q, arm.radius, np.array([[np.nan, 0.0, 0.0]]), hi[:1])
    # well-formed boxes pass the check and reach the device-tensor check
    with pytest.raises(ValueError, match="device tensor"):
        api.label_capsule_box(arm, q, arm.radius, lo[:1], hi[:1])


def test_product_path_is_independent_of_the_oracle():
    """The package neither imports the oracle nor includes its sources; with the HIP library missing the binding
    raises, and the entry points refuse host tensors: nothing is computed on the host."""
    import ast
    import pathlib
    import subprocess
    import sys
    pkg = pathlib.Path(nat.__file__).resolve().parent
    for py in pkg.rglob("*.py"):
        for node in ast.walk(ast.parse(py.read_text())):
            names = [a.name for a in node.names] if isinstance(node, ast.Import) else \
                [node.module or ""] if isinstance(node, ast.ImportFrom) else []
            assert not any(n.split(".")[0] == "oracle" for n in names), py
    for src in list(pkg.rglob("*.hip")) + list(pkg.rglob("*.h")):
        for line in src.read_text().splitlines():
            assert not (line.lstrip().startswith("#include") and "oracle" in line), (src, line)
    code = (
        "import torch\n"
        "from paper_1910_06451_amd import _native as nat, api, workloads as wl\n"
        "nat.LIB_PATH = '/nonexistent/libfastron_fk.so'\n"
        "arm = wl.arm_3dof()\n"
        "q = torch.zeros(4, arm.n)\n"
        "calls = [lambda: api.fk_points(arm, q), lambda: api.fk_score(arm, q, torch.ones(4), 10.0, q),\n"
        "         lambda: api.label_capsule_box(arm, q, 0.04, [[0, 0, 0]], [[1, 1, 1]])]\n"
        "try:\n"
        "    nat.lib()\n"
        "    raise SystemExit('the binding loaded a library that is not there')\n"
        "except nat.FastronLibraryMissing:\n"
        "    pass\n"
        "for c in calls:\n"
        "    try:\n"
        "        c()\n"
        "    except nat.FastronLibraryMissing:\n"
        "        continue\n"
        "    except ValueError as e:\n"
        "        if 'device tensor' in str(e):  # host tensors are refused before the library is looked up\n"
        "            continue\n"
        "        raise SystemExit(f'unexpected ValueError: {e}')\n"
        "    raise SystemExit('an entry point ran without the HIP library')\n"
        "import sys\n"
        "assert 'oracle' not in sys.modules\n"
        "print('ok')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=pkg.parent, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
