"""MI355X-native batched tensor-product apply and fast-diagonalization inverse.

The computation lives in libtpfdm.so (HIP kernels for gfx950 behind the C-ABI
of include/tpfdm.h); ``tpfdm`` is its ctypes binding and ``workloads`` the
seeded synthetic inputs.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "tpfdm"]
