"""MI355X-native Schwarz-preconditioned CG for finite cell systems.

The work runs in libfc.so (HIP kernels for gfx950 behind the C ABI of
include/fc.h); this package is its ctypes binding.
"""
from ._lib import (EXPORTS, Batch, FcError, HostSystem, Model, Precond, Problem, STORE_BF16,
                   STORE_F32, STORE_F64, load, pcg_solve, pcg_solve_noalloc)

__all__ = ["EXPORTS", "Batch", "FcError", "HostSystem", "Model", "Precond", "Problem", "STORE_BF16",
           "STORE_F32", "STORE_F64", "load", "pcg_solve", "pcg_solve_noalloc"]
