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
