"""MI355X-native CPR-FGMRES solver for fully implicit black-oil Jacobians.

The hot path runs in the HIP library libbo.so (C ABI in include/bo.h); the
module :mod:`paper_1606_00556_amd.bo` is its ctypes binding.
"""
from . import bo  # noqa: F401

__all__ = ["bo"]
