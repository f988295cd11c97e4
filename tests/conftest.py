import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle

    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def dev():
    """The GPU under test; GPU tests fail (not skip) when it or the HIP library is missing."""
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1910_06451_amd import _native

    _native.lib()
    return torch.device("cuda:0")


def oracle_dh(oracle_mod, arm):
    return oracle_mod.dh_table(arm.a, arm.alpha, arm.d, arm.theta, arm.joint_type)


def announce(msg):
    """Name the case on stdout before a GPU step, so a fault still leaves a trace."""
    print(f"[case] {msg}", flush=True)


# Bound on |F_device - K alpha| after an FP32 run of Algorithm 1: each update adds delta_alpha K_ji to F_j with
# one float32 rounding, so F drifts from the exact K alpha by a random walk of roundings. Runs of up to a few
# thousand samples stay within 1e-3; the 50,000-sample run (about 1.6e5 updates) within 1e-2.
FP32_F_DRIFT = 1e-3


def assert_claim2(y, F_oracle, F_gpu, drift=FP32_F_DRIFT):
    """Claim 2 (Section III-B) for an FP32 device model judged in FP64: the device's own margins y F are all
    positive (Algorithm 1 stopped there), its F is within `drift` of the oracle's F = K alpha, and every FP64
    margin y K alpha is positive or, where not, no further below zero than that drift. Returns the number of
    non-positive FP64 margins (reported, expected 0)."""
    import numpy as np

    y = np.asarray(y, np.float64)
    F_gpu = np.asarray(F_gpu, np.float64)
    dF = float(np.abs(F_gpu - F_oracle).max())
    assert dF <= drift, dF
    assert np.all(y * F_gpu > 0), float((y * F_gpu).min())
    m = y * F_oracle
    bad = m <= 0
    assert np.all(m[bad] > -drift), float(m.min())
    return int(bad.sum())
