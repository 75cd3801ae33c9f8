"""MI355X (gfx950) implementation of the MGM solve phase (arXiv 2204.06154).

The product is the native library libmgm.so (C ABI in include/mgm.h): host
setup in C++ and the V-cycle / Krylov hot path as HIP kernels. `mgm` is a thin
ctypes binding over it.
"""
from .mgm import Mgm, MgmError, load  # noqa: F401
