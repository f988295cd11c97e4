"""Fastron with the forward-kinematics kernel on MI355X (gfx950).

The computation lives in the HIP library ``libfastron_fk.so`` (C ABI in
``include/fastron_fk.h``); :mod:`paper_1910_06451_amd.api` is its torch-facing
binding and :mod:`paper_1910_06451_amd.workloads` draws the seeded synthetic
inputs. Importing this package does not load the library; the first call
into :mod:`api` does, and fails loudly if it has not been built.
"""
from . import workloads  # noqa: F401

__version__ = "1.0"
