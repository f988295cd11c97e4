"""bench.py's command line without a GPU: a multi-GPU request is refused with
a message before anything touches a device, and unknown legs are rejected."""
import os
import subprocess
import sys

from conftest import ROOT


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_unknown_leg_is_refused():
    r = _run("--legs", "kernels,nonsense")
    assert r.returncode == 2
    assert "nonsense" in r.stderr
