"""MI355X-native vectorial lattice Boltzmann (shallow water) hot path.

The numerical work runs in hand-written HIP kernels for gfx950 behind the C-ABI
library ``liblbm.so`` (declared in ``include/lbm.h``).  This package is a thin
ctypes binding: importing it does not load the library; the first use does, and
fails loudly if the library is missing.
"""
__all__ = ["workloads"]
