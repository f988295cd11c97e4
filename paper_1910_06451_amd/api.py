"""Torch-facing wrappers with the same names as the C ABI entry points.

Each function checks dtype / device / contiguity, passes raw pointers and the
current HIP stream to the library, and returns torch tensors. No arithmetic
of the method happens here.
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import torch

from . import _native as nat
from ._native import HostChain, check

__all__ = [
    "control_point_frames", "fk_points", "model_bytes", "support_prep", "fk_score_prepared", "fk_score", "gram_update", "gram_update_points", "train", "train_points",
    "train_batch",
    "rbf_score", "rbf_train", "score_rational", "tune_get", "tune_set", "active_samples", "active_relabel", "active_update",
    "label_capsule_box", "PreparedModel", "Batch", "MLP", "SCORE_FP32", "SCORE_BF16", "SCORE_VALU", "BF16_PLAIN", "BF16_SPLIT2",
    "BF16_SPLIT3",
]

SCORE_FP32, SCORE_BF16, SCORE_VALU = nat.SCORE_FP32, nat.SCORE_BF16, nat.SCORE_VALU
BF16_PLAIN, BF16_SPLIT2, BF16_SPLIT3 = nat.BF16_PLAIN, nat.BF16_SPLIT2, nat.BF16_SPLIT3


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _chain(arm):
    return arm if isinstance(arm, HostChain) else HostChain(arm)


def tune_get(key: str) -> int:
    """Current value of a launch/tuning knob (-1 for an unknown key)."""
    return int(nat.lib().fastron_tune_get(key.encode()))


def tune_set(key: str, value: int) -> None:
    """Sets a launch/tuning knob; raises on an unknown key or a value out of range."""
    check(nat.lib().fastron_tune_set(key.encode(), int(value)))


def control_point_frames(arm, include_base: bool = False) -> np.ndarray:
    """Frame indices of the control points placed by the library's Section III-A rule (frame origins,
    none for a revolute joint with a_i = d_i = 0; frame 0 first when include_base)."""
    hc = nat.HostChain(arm)
    out = np.zeros(hc.n + 1, dtype=np.int32)
    M = ctypes.c_int32(0)
    nat.check(nat.lib().fastron_control_point_frames(ctypes.byref(hc.chain), int(bool(include_base)),
                                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                                     ctypes.byref(M)))
    return out[:M.value].copy()


def fk_points(arm, q: torch.Tensor) -> torch.Tensor:
    """Control points FK_m(q) for every configuration: (N, n) float32 -> (N, M, 3) float32."""
    hc = _chain(arm)
    _dev(q, torch.float32, "q")
    if q.dim() != 2 or q.shape[1] != hc.n:
        raise ValueError(f"q must be (N, {hc.n})")
    P = torch.empty((q.shape[0], hc.M, 3), dtype=torch.float32, device=q.device)
    check(nat.lib().fastron_fk_points(ctypes.byref(hc.chain), ctypes.byref(hc.cpoints), _ptr(q), q.shape[0],
                                      _ptr(P), _stream()))
    return P


def model_bytes(S: int, M: int) -> int:
    return int(nat.lib().fastron_model_bytes(int(S), int(M)))


class PreparedModel:
    """A support set prepared for scoring (device blob + descriptor)."""

    def __init__(self, S, M, gamma, device):
        self.nbytes = model_bytes(S, M)
        self.buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        aligned = (base + 255) & ~255
        self.desc = nat.Model(int(S), int(M), float(gamma), ctypes.c_void_p(aligned), self.nbytes)
        self.S, self.M, self.gamma = int(S), int(M), float(gamma)


def support_prep(arm, support_q: torch.Tensor, alpha: torch.Tensor, gamma: float) -> PreparedModel:
    hc = _chain(arm)
    _dev(support_q, torch.float32, "support_q")
    _dev(alpha, torch.float32, "alpha")
    S = support_q.shape[0]
    if support_q.dim() != 2 or support_q.shape[1] != hc.n or alpha.shape != (S,):
        raise ValueError("support_q must be (S, n) and alpha (S,)")
    model = PreparedModel(S, hc.M, gamma, support_q.device)
    check(nat.lib().fastron_support_prep(ctypes.byref(hc.chain), ctypes.byref(hc.cpoints), _ptr(support_q),
                                         _ptr(alpha), S, float(gamma), ctypes.byref(model.desc), _stream()))
    model._keep = (support_q, alpha)
    return model


def _score_outputs(N, device, want_f, want_label):
    f = torch.empty(N, dtype=torch.float32, device=device) if want_f else None
    lab = torch.empty(N, dtype=torch.int8, device=device) if want_label else None
    return f, lab


def fk_score_prepared(arm, model: PreparedModel, q: torch.Tensor, flags: int = SCORE_FP32, want_f=True,
                      want_label=True, out=None):
    """f(q) and sign labels against a prepared model. Returns (f, label); either may be None."""
    hc = _chain(arm)
    _dev(q, torch.float32, "q")
    if q.dim() != 2 or q.shape[1] != hc.n:
        raise ValueError(f"q must be (N, {hc.n})")
    f, lab = out if out is not None else _score_outputs(q.shape[0], q.device, want_f, want_label)
    check(nat.lib().fastron_fk_score_prepared(ctypes.byref(hc.chain), ctypes.byref(hc.cpoints),
                                              ctypes.byref(model.desc), _ptr(q), q.shape[0], _ptr(f), _ptr(lab),
                                              int(flags), _stream()))
    return f, lab


def score_rational(arm, gamma: float, flags: int = SCORE_FP32) -> bool:
    """True when scoring with this arm, gamma and flags sums each pair's 1/t^2 terms as one running fraction."""
    hc = _chain(arm)
    r = nat.lib().fastron_score_rational(ctypes.byref(hc.chain), ctypes.byref(hc.cpoints), float(gamma), int(flags))
    check(min(r, 0))
    return r == 1


def fk_score(arm, support_q: torch.Tensor, alpha: torch.Tensor, gamma: float, q: torch.Tensor,
             flags: int = SCORE_FP32, want_f=True, want_label=True, out=None):
    """One call: prepare the support set and score the queries. Returns (f, label)."""
    hc = _chain(arm)
    _dev(support_q, torch.float32, "support_q")
    _dev(alpha, torch.float32, "alpha")
    _dev(q, torch.float32, "q")
    S = support_q.shape[0]
    if support_q.dim() != 2 or support_q.shape[1] != hc.n or alpha.shape != (S,):
        raise ValueError("support_q must be (S, n) and alpha (S,)")
    if q.dim() != 2 or q.shape[1] != hc.n:
        raise ValueError(f"q must be (N, {hc.n})")
    f, lab = out if out is not None else _score_outputs(q.shape[0], q.device, want_f, want_label)
    check(nat.lib().fastron_fk_score(ctypes.byref(hc.chain), ctypes.byref(hc.cpoints), _ptr(support_q),
                                     _ptr(alpha), S, float(gamma), _ptr(q), q.shape[0], _ptr(f), _ptr(lab),
                                     int(flags), _stream()))
    return f, lab


def fk_score_noalloc(arm, support_q: torch.Tensor, alpha: torch.Tensor, gamma: float, q: torch.Tensor,
                     flags: int = SCORE_FP32, out=None):
    """fk_score with the prepared support set in the library's static device buffer (no device allocation by
    the library). `out` = (f, label) preallocated by the caller (either may be None); returns it."""
    hc = _chain(arm)
    _dev(support_q, torch.float32, "support_q")
    _dev(alpha, torch.float32, "alpha")
    _dev(q, torch.float32, "q")
    S = support_q.shape[0]
    if support_q.dim() != 2 or support_q.shape[1] != hc.n or alpha.shape != (S,):
        raise ValueError("support_q must be (S, n) and alpha (S,)")
    if q.dim() != 2 or q.shape[1] != hc.n:
        raise ValueError(f"q must be (N, {hc.n})")
    f, lab = out if out is not None else _score_outputs(q.shape[0], q.device, True, True)
    check(nat.lib().fastron_fk_score_noalloc(ctypes.byref(hc.chain), ctypes.byref(hc.cpoints), _ptr(support_q),
                                             _ptr(alpha), S, float(gamma), _ptr(q), q.shape[0], _ptr(f), _ptr(lab),
                                             int(flags), _stream()))
    return f, lab


def gram_update_points(P: torch.Tensor, gamma: float, i: int, delta_alpha: float, F: torch.Tensor | None = None,
                       want_kcol=True):
    """kcol = K_FK(X_j, X_i) over j on control points P (N, M, 3); F += delta_alpha * kcol (in place).
    Returns kcol (or None)."""
    _dev(P, torch.float32, "P")
    if P.dim() != 3 or P.shape[2] != 3:
        raise ValueError("P must be (N, M, 3)")
    N, M = P.shape[0], P.shape[1]
    F = _gram_F(F, N)
    kcol = torch.empty(N, dtype=torch.float32, device=P.device) if want_kcol else None
    check(nat.lib().fastron_gram_update_points(_ptr(P), N, M, float(gamma), int(i), float(delta_alpha), _ptr(F),
                                               _ptr(kcol), _stream()))
    return kcol


def gram_update(arm, X: torch.Tensor, gamma: float, i: int, delta_alpha: float, F: torch.Tensor | None = None,
                want_kcol=True):
    """The same update on configurations X (N, n): their control points are computed by the library."""
    hc = _chain(arm)
    _dev(X, torch.float32, "X")
    if X.dim() != 2 or X.shape[1] != hc.n:
        raise ValueError(f"X must be (N, {hc.n})")
    N = X.shape[0]
    F = _gram_F(F, N)
    kcol = torch.empty(N, dtype=torch.float32, device=X.device) if want_kcol else None
    check(nat.lib().fastron_gram_update(ctypes.byref(hc.chain), ctypes.byref(hc.cpoints), _ptr(X), N, float(gamma),
                                        int(i), float(delta_alpha), _ptr(F), _ptr(kcol), _stream()))
    return kcol


def _gram_F(F, N):
    if F is not None:
        _dev(F, torch.float32, "F")
        if F.shape != (N,):
            raise ValueError("F must be (N,)")
    return F


def _train_state(N, device, y, alpha, F, fp64, iter_max, s_max, trace_cap):
    _dev(y, torch.int8, "y")
    if y.shape != (N,):
        raise ValueError("y must hold one label per training row")
    dt = torch.float64 if fp64 else torch.float32
    alpha = torch.zeros(N, dtype=dt, device=device) if alpha is None else alpha.clone()
    F = torch.zeros(N, dtype=dt, device=device) if F is None else F.clone()
    _dev(alpha, dt, "alpha")
    _dev(F, dt, "F")
    iter_max = 20 * max(N, 1) if iter_max is None else int(iter_max)
    s_max = max(N, 1) if s_max is None else int(s_max)
    support = torch.empty(max(N, 1), dtype=torch.int32, device=device)
    tr_a = torch.zeros(max(trace_cap, 1), dtype=torch.int32, device=device) if trace_cap else None
    tr_i = torch.zeros(max(trace_cap, 1), dtype=torch.int32, device=device) if trace_cap else None
    return alpha, F, iter_max, s_max, support, tr_a, tr_i


def _train_result(st, alpha, F, support, ns, upd, tr_a, tr_i, trace_cap):
    check(st, allow=(nat.FASTRON_OK, nat.FASTRON_NOT_CONVERGED))
    out = dict(alpha=alpha, F=F, support=support[: ns.value], converged=(st == nat.FASTRON_OK), updates=upd.value)
    if trace_cap:
        k = min(upd.value, trace_cap)
        out["trace_action"] = tr_a[:k]
        out["trace_index"] = tr_i[:k]
    return out


def train_points(P: torch.Tensor, y: torch.Tensor, gamma: float, beta: float = 1.0, iter_max: int | None = None,
                 s_max: int | None = None, alpha: torch.Tensor | None = None, F: torch.Tensor | None = None,
                 fp64: bool = False, trace_cap: int = 0):
    """Algorithm 1 on the device over control points P (N, M, 3).
    Returns dict(alpha, F, support, converged, updates[, trace])."""
    _dev(P, torch.float32, "P")
    if P.dim() != 3 or P.shape[2] != 3:
        raise ValueError("P must be (N, M, 3)")
    N, M = P.shape[0], P.shape[1]
    alpha, F, iter_max, s_max, support, tr_a, tr_i = _train_state(N, P.device, y, alpha, F, fp64, iter_max, s_max,
                                                                  trace_cap)
    ns = ctypes.c_int64(0)
    upd = ctypes.c_int64(0)
    fn = nat.lib().fastron_train_points_f64 if fp64 else nat.lib().fastron_train_points
    st = fn(_ptr(P), _ptr(y), N, M, float(gamma), float(beta), iter_max, s_max, _ptr(alpha), _ptr(F),
            _ptr(support), ctypes.byref(ns), ctypes.byref(upd), _ptr(tr_a), _ptr(tr_i), int(trace_cap), _stream())
    return _train_result(st, alpha, F, support, ns, upd, tr_a, tr_i, trace_cap)


def train(arm, X: torch.Tensor, y: torch.Tensor, gamma: float, beta: float = 1.0, iter_max: int | None = None,
          s_max: int | None = None, alpha: torch.Tensor | None = None, F: torch.Tensor | None = None,
          fp64: bool = False, trace_cap: int = 0):
    """Algorithm 1 on the device over configurations X (N, n) of the arm (its control points computed by the
    library). Returns the same dict as train_points()."""
    hc = _chain(arm)
    _dev(X, torch.float32, "X")
    if X.dim() != 2 or X.shape[1] != hc.n:
        raise ValueError(f"X must be (N, {hc.n})")
    N = X.shape[0]
    alpha, F, iter_max, s_max, support, tr_a, tr_i = _train_state(N, X.device, y, alpha, F, fp64, iter_max, s_max,
                                                                  trace_cap)
    ns = ctypes.c_int64(0)
    upd = ctypes.c_int64(0)
    fn = nat.lib().fastron_train_f64 if fp64 else nat.lib().fastron_train
    st = fn(ctypes.byref(hc.chain), ctypes.byref(hc.cpoints), _ptr(X), _ptr(y), N, float(gamma), float(beta),
            iter_max, s_max, _ptr(alpha), _ptr(F), _ptr(support), ctypes.byref(ns), ctypes.byref(upd), _ptr(tr_a),
            _ptr(tr_i), int(trace_cap), _stream())
    return _train_result(st, alpha, F, support, ns, upd, tr_a, tr_i, trace_cap)


def rbf_score(support_x: torch.Tensor, alpha: torch.Tensor, gamma: float, q: torch.Tensor, want_f=True,
              want_label=True, out=None):
    """The model with the kernel on configurations (Eq. 3 on joint vectors): f(q) and its sign."""
    _dev(support_x, torch.float32, "support_x")
    _dev(alpha, torch.float32, "alpha")
    _dev(q, torch.float32, "q")
    S, n = support_x.shape
    if q.dim() != 2 or q.shape[1] != n or alpha.shape != (S,):
        raise ValueError("support_x (S, n), alpha (S,) and q (N, n) do not match")
    N = q.shape[0]
    f, lab = out if out is not None else _score_outputs(N, q.device, want_f, want_label)
    check(nat.lib().fastron_rbf_score(_ptr(support_x), _ptr(alpha), S, n, float(gamma), _ptr(q), N, _ptr(f),
                                      _ptr(lab), _stream()))
    return f, lab


def rbf_train(X: torch.Tensor, y: torch.Tensor, gamma: float, beta: float = 1.0, iter_max: int | None = None,
              s_max: int | None = None, alpha: torch.Tensor | None = None, F: torch.Tensor | None = None,
              fp64: bool = False, trace_cap: int = 0):
    """Algorithm 1 with the kernel on configurations on X (N, n). Returns the same dict as train()."""
    _dev(X, torch.float32, "X")
    _dev(y, torch.int8, "y")
    if trace_cap and not fp64:
        raise ValueError("the update trace is recorded by the FP64 mode only (fp64=True)")
    N, n = X.shape
    if y.shape != (N,):
        raise ValueError("X must be (N, n) and y (N,)")
    dt = torch.float64 if fp64 else torch.float32
    alpha = torch.zeros(N, dtype=dt, device=X.device) if alpha is None else alpha.clone()
    F = torch.zeros(N, dtype=dt, device=X.device) if F is None else F.clone()
    _dev(alpha, dt, "alpha")
    _dev(F, dt, "F")
    iter_max = 20 * max(N, 1) if iter_max is None else int(iter_max)
    s_max = max(N, 1) if s_max is None else int(s_max)
    support = torch.empty(max(N, 1), dtype=torch.int32, device=X.device)
    ns = ctypes.c_int64(0)
    upd = ctypes.c_int64(0)
    tr_a = tr_i = None
    if fp64:
        tr_a = torch.zeros(max(trace_cap, 1), dtype=torch.int32, device=X.device) if trace_cap else None
        tr_i = torch.zeros(max(trace_cap, 1), dtype=torch.int32, device=X.device) if trace_cap else None
        st = nat.lib().fastron_rbf_train_f64(_ptr(X), _ptr(y), N, n, float(gamma), float(beta), iter_max, s_max,
                                             _ptr(alpha), _ptr(F), _ptr(support), ctypes.byref(ns),
                                             ctypes.byref(upd), _ptr(tr_a), _ptr(tr_i), int(trace_cap), _stream())
    else:
        st = nat.lib().fastron_rbf_train(_ptr(X), _ptr(y), N, n, float(gamma), float(beta), iter_max, s_max,
                                         _ptr(alpha), _ptr(F), _ptr(support), ctypes.byref(ns), ctypes.byref(upd),
                                         _stream())
    check(st, allow=(nat.FASTRON_OK, nat.FASTRON_NOT_CONVERGED))
    out = dict(alpha=alpha, F=F, support=support[: ns.value], converged=(st == nat.FASTRON_OK), updates=upd.value)
    if fp64 and trace_cap:
        k = min(upd.value, trace_cap)
        out["trace_action"] = tr_a[:k]
        out["trace_index"] = tr_i[:k]
    return out


def train_batch(P: torch.Tensor, y: torch.Tensor, offsets, gamma: float, beta: float = 1.0,
                iter_max: int | None = None, s_max: int | None = None, alpha: torch.Tensor | None = None,
                F: torch.Tensor | None = None):
    """Algorithm 1 on several independent training sets at once (rows offsets[e] .. offsets[e+1] - 1 of P and y
    form set e). iter_max / s_max default to 20 N_e / N_e of the largest set. Returns dict(alpha, F,
    supports (list of index tensors relative to each set), converged (all sets), updates (list))."""
    _dev(P, torch.float32, "P")
    _dev(y, torch.int8, "y")
    N, M = P.shape[0], P.shape[1]
    if P.dim() != 3 or P.shape[2] != 3 or y.shape != (N,):
        raise ValueError("P must be (N, M, 3) and y (N,)")
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    E = off.shape[0] - 1
    if E < 1 or off[0] != 0 or off[-1] != N or np.any(np.diff(off) <= 0):
        raise ValueError("offsets must increase strictly from 0 to N")
    largest = int(np.max(np.diff(off)))
    alpha = torch.zeros(N, dtype=torch.float32, device=P.device) if alpha is None else alpha.clone()
    F = torch.zeros(N, dtype=torch.float32, device=P.device) if F is None else F.clone()
    _dev(alpha, torch.float32, "alpha")
    _dev(F, torch.float32, "F")
    if alpha.shape != (N,) or F.shape != (N,):
        raise ValueError("alpha and F must be (N,)")
    iter_max = 20 * largest if iter_max is None else int(iter_max)
    s_max = largest if s_max is None else int(s_max)
    support = torch.empty(N, dtype=torch.int32, device=P.device)
    ns = np.zeros(E, dtype=np.int64)
    upd = np.zeros(E, dtype=np.int64)
    p64 = ctypes.POINTER(ctypes.c_int64)
    st = nat.lib().fastron_train_batch(_ptr(P), _ptr(y), E, off.ctypes.data_as(p64), M, float(gamma), float(beta),
                                       iter_max, s_max, _ptr(alpha), _ptr(F), _ptr(support), ns.ctypes.data_as(p64),
                                       upd.ctypes.data_as(p64), _stream())
    check(st, allow=(nat.FASTRON_OK, nat.FASTRON_NOT_CONVERGED))
    supports = [support[off[e]:off[e] + ns[e]] for e in range(E)]
    return dict(alpha=alpha, F=F, supports=supports, converged=(st == nat.FASTRON_OK), updates=upd.tolist())


def label_capsule_box(arm, q: torch.Tensor, radius: float, boxes_lo, boxes_hi, want_clearance=True):
    """Geometric labels (+1 collision / -1 free, int8) and clearance (float32, min distance - radius)."""
    lo = np.asarray(boxes_lo, dtype=np.float64).reshape(-1, 3)
    hi = np.asarray(boxes_hi, dtype=np.float64).reshape(-1, 3)
    if lo.shape != hi.shape or np.any(~(lo <= hi)):
        raise ValueError("boxes need lo <= hi on every axis and as many lo as hi corners")
    hc = _chain(arm)
    _dev(q, torch.float32, "q")
    if q.dim() != 2 or q.shape[1] != hc.n:
        raise ValueError(f"q must be (N, {hc.n})")
    boxes = torch.from_numpy(np.ascontiguousarray(np.concatenate([lo, hi], axis=1))).to(q.device)
    N = q.shape[0]
    lab = torch.empty(N, dtype=torch.int8, device=q.device)
    clr = torch.empty(N, dtype=torch.float32, device=q.device) if want_clearance else None
    check(nat.lib().fastron_label_capsule_box(ctypes.byref(hc.chain), _ptr(q), N, float(radius), _ptr(boxes),
                                              boxes.shape[0], _ptr(lab), _ptr(clr), _stream()))
    return lab, clr


def active_samples(support_q: torch.Tensor, alpha: torch.Tensor, noise: torch.Tensor, k: int,
                   explore: torch.Tensor):
    """Training set of the next model update (two-stage active learning, Section III-B): the supports, k
    samples near each (support + noise row) and the exploration samples; weights kept on the supports."""
    for t, name in ((support_q, "support_q"), (alpha, "alpha"), (noise, "noise"), (explore, "explore")):
        _dev(t, torch.float32, name)
    S, n = support_q.shape
    E = explore.shape[0]
    if alpha.shape != (S,) or noise.shape != (S * k, n) or explore.dim() != 2 or explore.shape[1] != n:
        raise ValueError("support_q (S, n), alpha (S,), noise (S k, n) and explore (E, n) do not match")
    rows = S * (1 + k) + E
    X = torch.empty(rows, n, dtype=torch.float32, device=support_q.device)
    a0 = torch.empty(rows, dtype=torch.float32, device=support_q.device)
    check(nat.lib().fastron_active_samples(_ptr(support_q), _ptr(alpha), S, n, _ptr(noise), int(k), _ptr(explore),
                                           E, _ptr(X), _ptr(a0), _stream()))
    return X, a0


def active_relabel(y: torch.Tensor, alpha: torch.Tensor, S: int):
    """Zero (in place) the weights of the first S rows whose label y disagrees with the weight's sign."""
    _dev(y, torch.int8, "y")
    _dev(alpha, torch.float32, "alpha")
    if S < 0 or S > min(y.shape[0], alpha.shape[0]):
        raise ValueError("S must lie within both arrays")
    check(nat.lib().fastron_active_relabel(_ptr(y), int(S), _ptr(alpha), _stream()))
    return alpha


def active_update(arm, support_q: torch.Tensor, alpha: torch.Tensor, gamma: float, noise: torch.Tensor,
                  k: int, explore: torch.Tensor, boxes_lo, boxes_hi, beta: float = 1.0,
                  iter_max: int | None = None, s_max: int | None = None):
    """One model update after two-stage active learning (Section III-B), every step on the device: assemble
    the new training set, label every row geometrically, zero the weights of supports whose label changed,
    start from F = the current model's score of every row (F = K alpha) and run Algorithm 1. Returns
    train_points()'s dict plus X, y, F0 and the starting weights alpha0."""
    X, a0 = active_samples(support_q, alpha, noise, k, explore)
    y, _ = label_capsule_box(arm, X, arm.radius, boxes_lo, boxes_hi, want_clearance=False)
    S = support_q.shape[0]
    active_relabel(y, a0, S)
    F0, _ = fk_score(arm, support_q, a0[:S], gamma, X, want_label=False)
    alpha0 = a0.clone()
    out = train_points(fk_points(arm, X), y, gamma, beta=beta, iter_max=iter_max, s_max=s_max, alpha=a0, F=F0)
    out.update(X=X, y=y, F0=F0, alpha0=alpha0)
    return out


class Batch:
    """Many environments' models (one arm) scored in one persistent launch (the batched form).

    support_counts[e] / query_counts[e] give each environment's support-set and query-batch sizes; the support
    configurations, weights and queries are the concatenation over environments in that order.
    """

    def __init__(self, arm, support_counts, query_counts, gamma: float):
        self.hc = _chain(arm)
        sc = np.asarray(support_counts, dtype=np.int64)
        qc = np.asarray(query_counts, dtype=np.int64)
        if sc.shape != qc.shape or sc.ndim != 1:
            raise ValueError("support_counts and query_counts must be 1-D and of equal length")
        self.E = int(sc.shape[0])
        self.support_off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(sc)]).astype(np.int64))
        self.query_off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(qc)]).astype(np.int64))
        self.S_total = int(self.support_off[-1])
        self.N_total = int(self.query_off[-1])
        self.gamma = float(gamma)
        h = ctypes.c_void_p()
        lp = ctypes.POINTER(ctypes.c_int64)
        check(nat.lib().fastron_batch_create(ctypes.byref(self.hc.chain), ctypes.byref(self.hc.cpoints), self.E,
                                             self.support_off.ctypes.data_as(lp), self.query_off.ctypes.data_as(lp),
                                             self.gamma, ctypes.byref(h)))
        self._h = h
        self._keep = None

    def prepare(self, support_q: torch.Tensor, alpha: torch.Tensor):
        _dev(support_q, torch.float32, "support_q")
        _dev(alpha, torch.float32, "alpha")
        if support_q.shape != (self.S_total, self.hc.n) or alpha.shape != (self.S_total,):
            raise ValueError(f"support_q must be ({self.S_total}, {self.hc.n}) and alpha ({self.S_total},)")
        check(nat.lib().fastron_batch_prepare(self._h, _ptr(support_q), _ptr(alpha), _stream()))
        self._keep = (support_q, alpha)

    def _io(self, q, out):
        _dev(q, torch.float32, "q")
        if q.shape != (self.N_total, self.hc.n):
            raise ValueError(f"q must be ({self.N_total}, {self.hc.n})")
        if out is None:
            out = (torch.empty(self.N_total, dtype=torch.float32, device=q.device),
                   torch.empty(self.N_total, dtype=torch.int8, device=q.device))
        return out

    def score(self, q: torch.Tensor, out=None):
        f, lab = self._io(q, out)
        check(nat.lib().fastron_batch_score(self._h, _ptr(q), _ptr(f), _ptr(lab), _stream()))
        return f, lab

    def autotune(self, q: torch.Tensor, out=None) -> int:
        f, lab = self._io(q, out)
        check(nat.lib().fastron_batch_autotune(self._h, _ptr(q), _ptr(f), _ptr(lab), _stream()))
        return self.tile_queries

    @property
    def tile_queries(self) -> int:
        return int(nat.lib().fastron_batch_tile_queries(self._h))

    @property
    def shape(self) -> dict:
        """The launch shape in use: queries per work item, waves per workgroup, paired MFMAs, grid share (%) and
        whether the last autotune reused a cached shape."""
        v = [ctypes.c_int32(0) for _ in range(5)]
        check(nat.lib().fastron_batch_get_shape(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("queries_per_item", "waves_per_group", "paired", "grid_pct", "from_cache"),
                        (int(x.value) for x in v)))

    def set_shape(self, queries_per_item: int, waves_per_group: int, paired: int, grid_pct: int):
        check(nat.lib().fastron_batch_set_shape(self._h, int(queries_per_item), int(waves_per_group), int(paired),
                                                int(grid_pct), _stream()))

    def capture(self, q: torch.Tensor, out):
        """Record {counter reset, scoring launch} for these exact buffers on the current (non-default) stream."""
        f, lab = self._io(q, out)
        check(nat.lib().fastron_batch_capture(self._h, _ptr(q), _ptr(f), _ptr(lab), _stream()))
        self._graph_io = (q, f, lab)

    def replay(self):
        check(nat.lib().fastron_batch_replay(self._h, _stream()))

    def close(self):
        if getattr(self, "_h", None):
            nat.lib().fastron_batch_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # No library calls while the interpreter shuts down (the HIP runtime may be tearing down too); the
        # process releases the device memory anyway. The check is bound at definition time because module
        # globals such as `sys` may already be cleared when a late destructor runs.
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """Learned pre-screen on FK control points: 3M -> H -> H -> 1 (BF16 MFMA, FP32 masters, Adam)."""

    def __init__(self, d_in: int, hidden: int = 256, max_rows: int = 8192):
        h = ctypes.c_void_p()
        check(nat.lib().fastron_mlp_create(int(d_in), int(hidden), int(max_rows), ctypes.byref(h)))
        self._h = h
        self.d_in, self.hidden, self.max_rows = int(d_in), int(hidden), int(max_rows)
        self.n_params = int(nat.lib().fastron_mlp_param_count(h))

    def set_params(self, params: torch.Tensor, mu: torch.Tensor | None = None, sd: torch.Tensor | None = None):
        _dev(params, torch.float32, "params")
        if params.shape != (self.n_params,):
            raise ValueError(f"params must be ({self.n_params},)")
        for t, nm in ((mu, "mu"), (sd, "sd")):
            if t is not None:
                _dev(t, torch.float32, nm)
        check(nat.lib().fastron_mlp_set_params(self._h, _ptr(params), _ptr(mu), _ptr(sd), _stream()))

    def get_params(self, device):
        p = torch.empty(self.n_params, dtype=torch.float32, device=device)
        g = torch.empty(self.n_params, dtype=torch.float32, device=device)
        mu = torch.empty(self.d_in, dtype=torch.float32, device=device)
        sd = torch.empty(self.d_in, dtype=torch.float32, device=device)
        check(nat.lib().fastron_mlp_get_params(self._h, _ptr(p), _ptr(g), _ptr(mu), _ptr(sd), _stream()))
        return p, g, mu, sd

    def adam_state(self, device):
        """(m, v, step): the optimiser's moments and its step count."""
        m = torch.empty(self.n_params, dtype=torch.float32, device=device)
        v = torch.empty(self.n_params, dtype=torch.float32, device=device)
        step = ctypes.c_int64(0)
        check(nat.lib().fastron_mlp_get_adam_state(self._h, _ptr(m), _ptr(v), ctypes.byref(step), _stream()))
        return m, v, int(step.value)

    def _points(self, P):
        _dev(P, torch.float32, "P")
        if P.dim() != 3 or P.shape[1] * P.shape[2] != self.d_in:
            raise ValueError(f"P must be (N, M, 3) with 3M = {self.d_in}")
        return P

    def fit_standardisation(self, P: torch.Tensor):
        self._points(P)
        check(nat.lib().fastron_mlp_fit_standardisation(self._h, _ptr(P), P.shape[0], _stream()))

    def forward(self, P: torch.Tensor) -> torch.Tensor:
        self._points(P)
        z = torch.empty(P.shape[0], dtype=torch.float32, device=P.device)
        check(nat.lib().fastron_mlp_forward(self._h, _ptr(P), P.shape[0], _ptr(z), _stream()))
        return z

    def gradients(self, P: torch.Tensor, y: torch.Tensor) -> float:
        self._points(P)
        _dev(y, torch.int8, "y")
        if y.shape != (P.shape[0],):
            raise ValueError("y must hold one label per row of P")
        loss = ctypes.c_float(0.0)
        check(nat.lib().fastron_mlp_gradients(self._h, _ptr(P), _ptr(y), P.shape[0], ctypes.byref(loss), _stream()))
        return float(loss.value)

    def train_epoch(self, P: torch.Tensor, y: torch.Tensor, order: torch.Tensor | None = None, batch: int = 8192,
                    lr: float = 1e-3) -> float:
        self._points(P)
        _dev(y, torch.int8, "y")
        if y.shape != (P.shape[0],):
            raise ValueError("y must hold one label per row of P")
        if order is not None:
            _dev(order, torch.int32, "order")
            if order.shape != (P.shape[0],):
                raise ValueError("order must hold one row index per row of P")
        loss = ctypes.c_float(0.0)
        check(nat.lib().fastron_mlp_train_epoch(self._h, _ptr(P), _ptr(y), _ptr(order), P.shape[0], int(batch),
                                                float(lr), ctypes.byref(loss), _stream()))
        return float(loss.value)

    def screen(self, arm, model: "PreparedModel", q: torch.Tensor, tau: float):
        """Returns (label int8, logit float32, fell_back uint8, n_fallback)."""
        hc = _chain(arm)
        _dev(q, torch.float32, "q")
        N = q.shape[0]
        lab = torch.empty(N, dtype=torch.int8, device=q.device)
        logit = torch.empty(N, dtype=torch.float32, device=q.device)
        fb = torch.empty(N, dtype=torch.uint8, device=q.device)
        nb = int(nat.lib().fastron_mlp_screen_workspace_bytes(N, hc.n))
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=q.device)
        nfb = ctypes.c_int64(0)
        check(nat.lib().fastron_mlp_screen(self._h, ctypes.byref(hc.chain), ctypes.byref(hc.cpoints),
                                           ctypes.byref(model.desc), _ptr(q), N, float(tau), _ptr(logit), _ptr(lab),
                                           _ptr(fb), ctypes.byref(nfb), _ptr(ws), ws.numel(), _stream()))
        return lab, logit, fb, int(nfb.value)

    def close(self):
        if getattr(self, "_h", None):
            nat.lib().fastron_mlp_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # No library calls while the interpreter shuts down (the HIP runtime may be tearing down too); the
        # process releases the device memory anyway. The check is bound at definition time because module
        # globals such as `sys` may already be cleared when a late destructor runs.
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
