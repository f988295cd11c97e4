"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws random numbers and lays out arrays. It holds none of
the method's arithmetic (no kinematics, no kernel, no model) so that both the
GPU library's tests and the FP64 oracle can consume the very same inputs.

The paper's experiments use a Baxter arm and FCL-labelled random obstacles
(Section IV); neither is available here, so synthetic D-H arms with random
axis-aligned cubes stand in:

* ``arm_3dof``   -- planar 3-DOF revolute arm, link lengths 0.4/0.3/0.2 m,
  alpha = 0, d = 0, control points at frames 0..3 (M = 4).
* ``arm_7dof``   -- 7-DOF revolute arm, a_i ~ U[0.2, 0.4] m,
  alpha_i uniform over {0, +pi/2, -pi/2}, d_i = 0, control points at frames
  0..7 (M = 8).
* ``cubes``      -- axis-aligned cubes with centres uniform in [-0.8, 0.8]^3.
* ``configs``    -- joint vectors uniform in [-pi, pi]^n (float32).
* ``model``      -- support configurations and weights alpha ~ N(0, 1).
* ``batched_envs`` -- many environments with lognormal support-set sizes
  over [200, 8000] and uniform query counts over [1000, 100000].

Every stream draws from its own generator, derived from a master seed and
the stream's name, so adding a stream never shifts another one.
"""
from __future__ import annotations

import dataclasses
import zlib

import numpy as np

MASTER_SEED = 19100645


def rng(name: str, seed: int = MASTER_SEED) -> np.random.Generator:
    """Independent generator for the stream ``name`` under ``seed``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, zlib.crc32(name.encode())])))


@dataclasses.dataclass
class Arm:
    """Standard D-H chain plus control-point placement (frame index per point)."""

    a: np.ndarray
    alpha: np.ndarray
    d: np.ndarray
    theta: np.ndarray
    joint_type: np.ndarray  # 0 revolute, 1 prismatic
    frames: np.ndarray  # int32, frame index j_m in [0, n] per control point
    offsets: np.ndarray | None = None  # (M, 3) or None (T_m = identity)
    radius: float = 0.04  # capsule radius of every link for the geometric labeller

    @property
    def n(self) -> int:
        return int(self.a.shape[0])

    @property
    def M(self) -> int:
        return int(self.frames.shape[0])


def arm_3dof() -> Arm:
    n = 3
    return Arm(a=np.array([0.4, 0.3, 0.2]), alpha=np.zeros(n), d=np.zeros(n), theta=np.zeros(n),
               joint_type=np.zeros(n, dtype=np.int32), frames=np.arange(n + 1, dtype=np.int32))


def arm_7dof(seed: int = MASTER_SEED) -> Arm:
    g = rng("arm_7dof", seed)
    n = 7
    a = g.uniform(0.2, 0.4, size=n)
    alpha = g.choice(np.array([0.0, np.pi / 2, -np.pi / 2]), size=n)
    return Arm(a=a, alpha=alpha, d=np.zeros(n), theta=np.zeros(n), joint_type=np.zeros(n, dtype=np.int32),
               frames=np.arange(n + 1, dtype=np.int32))


def two_link(frames=(1, 2)) -> Arm:
    """Unit two-link planar arm used by the worked examples."""
    return Arm(a=np.array([1.0, 1.0]), alpha=np.zeros(2), d=np.zeros(2), theta=np.zeros(2),
               joint_type=np.zeros(2, dtype=np.int32), frames=np.asarray(frames, dtype=np.int32))


def cubes(name: str, count: int, side_lo: float, side_hi: float | None = None, seed: int = MASTER_SEED,
          centre_range: float = 0.8):
    """Axis-aligned cubes: returns (lo, hi), each (count, 3) float64."""
    g = rng(name, seed)
    c = g.uniform(-centre_range, centre_range, size=(count, 3))
    side = np.full(count, side_lo) if side_hi is None else g.uniform(side_lo, side_hi, size=count)
    h = 0.5 * side[:, None]
    return c - h, c + h


def configs(name: str, count: int, n: int, seed: int = MASTER_SEED, lo: float = -np.pi, hi: float = np.pi):
    """Joint vectors uniform in [lo, hi]^n as float32 (count, n)."""
    g = rng(name, seed)
    return g.uniform(lo, hi, size=(count, n)).astype(np.float32)


def weights(name: str, count: int, seed: int = MASTER_SEED):
    """Synthetic support weights alpha ~ N(0, 1) as float32."""
    return rng(name, seed).standard_normal(count).astype(np.float32)


def model(name: str, S: int, n: int, seed: int = MASTER_SEED):
    """Synthetic model: S support configurations and their weights."""
    return configs(name + "/support", S, n, seed), weights(name + "/alpha", S, seed)


@dataclasses.dataclass
class BatchedEnvs:
    support_counts: np.ndarray  # (E,) int64
    query_counts: np.ndarray  # (E,) int64
    cube_counts: np.ndarray  # (E,) int64

    @property
    def E(self) -> int:
        return int(self.support_counts.shape[0])

    def support_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.support_counts)]).astype(np.int64)

    def query_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.query_counts)]).astype(np.int64)


def batched_envs(E: int = 256, s_lo: int = 200, s_hi: int = 8000, q_lo: int = 1000, q_hi: int = 100000,
                 cubes_lo: int = 5, cubes_hi: int = 40, seed: int = MASTER_SEED) -> BatchedEnvs:
    """Environment sizes: ln S ~ N((ln s_lo + ln s_hi)/2, (ln s_hi - ln s_lo)/4) clipped to [s_lo, s_hi];
    query counts uniform over {q_lo..q_hi}; cube counts uniform over {cubes_lo..cubes_hi}."""
    g = rng("batched_envs", seed)
    mu = 0.5 * (np.log(s_lo) + np.log(s_hi))
    sd = (np.log(s_hi) - np.log(s_lo)) / 4.0
    S = np.clip(np.rint(np.exp(g.normal(mu, sd, size=E))), s_lo, s_hi).astype(np.int64)
    Q = g.integers(q_lo, q_hi + 1, size=E).astype(np.int64)
    C = g.integers(cubes_lo, cubes_hi + 1, size=E).astype(np.int64)
    return BatchedEnvs(S, Q, C)


def unit_directions(name: str, count: int, seed: int = MASTER_SEED) -> np.ndarray:
    """Uniformly random unit vectors in R^3 (count, 3)."""
    v = rng(name, seed).standard_normal(size=(count, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def mlp_init(d_in: int, hidden: int = 256, seed: int = MASTER_SEED, name: str = "mlp_init") -> np.ndarray:
    """He-normal initial weights (zero biases) for the screening network, flattened in the order
    W1 [d_in][H], b1 [H], W2 [H][H], b2 [H], w3 [H], b3 [1] as float32."""
    g = rng(name, seed)
    w1 = g.standard_normal((d_in, hidden)) * np.sqrt(2.0 / d_in)
    w2 = g.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden)
    w3 = g.standard_normal(hidden) * np.sqrt(2.0 / hidden)
    parts = [w1.ravel(), np.zeros(hidden), w2.ravel(), np.zeros(hidden), w3, np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def split_mlp_params(flat: np.ndarray, d_in: int, hidden: int = 256):
    """Views of a flat parameter vector as [W1, b1, W2, b2, w3, b3]."""
    sizes = [d_in * hidden, hidden, hidden * hidden, hidden, hidden, 1]
    shapes = [(d_in, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden,), ()]
    out, o = [], 0
    for sz, sh in zip(sizes, shapes):
        out.append(flat[o:o + sz].reshape(sh))
        o += sz
    return out
