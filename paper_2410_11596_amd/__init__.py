"""Hermitian-symmetric (Z2) CTMRG for AMD Instinct MI355X.

The computation lives in libhctm.so (HIP kernels for gfx950 behind a C ABI,
include/hctm.h); `binding` is a thin ctypes layer over it and `inputs` draws
the seeded synthetic tensors used by the tests and the benchmark.
"""
from . import inputs  # noqa: F401
from .binding import CTMRG, HOTRG, HctmError, Server, lib, workspace_size  # noqa: F401
