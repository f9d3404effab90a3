"""MI355X-native EOS-based multiphase lattice Boltzmann (arXiv 2103.08301).

The compute path is liblbm.so (HIP kernels for gfx950 behind the C ABI of
include/lbm.h); `lbm` is its ctypes binding.  Importing the package does not
load the library; the first call that needs it raises if it is not built.
"""
from . import lbm  # noqa: F401
from .lbm import Batch, Lattice, WallShearObjective  # noqa: F401

__all__ = ["lbm", "Batch", "Lattice", "WallShearObjective"]
