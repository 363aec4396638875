"""MI355X-native finite-volume compressible-Euler zone update.

The hot path (split MUSCL-Hancock/HLLC sweeps, gravity source, CFL
reduction, FP64 totals, batched persistent sweeps) lives in the HIP
library libhydro.so behind the C ABI of include/hydro.h; `hydro` is its
ctypes binding.  Importing this package does not load the library; the
first call into `hydro` does, and fails loudly if it was not built.
"""
from . import hydro  # noqa: F401

__all__ = ["hydro"]
