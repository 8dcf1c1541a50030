"""MI355X (gfx950) TPC sector tracker: CA + Kalman-filter track finding.

The compute path is the HIP library ``libtpcca.so`` behind the C ABI in
``include/tpcca.h``; ``paper_1709_00618_amd.tpcca`` is its ctypes binding.
"""
from . import tpcca  # noqa: F401

__all__ = ["tpcca"]
