"""MI355X-native single-copy, two-step-merged D3Q19 lattice Boltzmann update.

The compute path is the HIP library ``liblbm.so`` (built from ``csrc/``) and
its C ABI (``include/lbm.h``); ``capi`` is a thin ctypes binding with the same
names, ``lattice`` a torch-facing wrapper and ``adjoint`` the autograd
function.  Importing the package loads nothing; the library is loaded on first
use and a missing library is an error, never a fallback.
"""
__all__ = ["capi", "lattice", "adjoint", "workloads"]
