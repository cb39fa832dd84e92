"""CTR-IBIM linearised Poisson-Boltzmann solver for AMD MI355X.

The solver lives in ``libibim.so`` (hand-written HIP for gfx950 plus host C++
setup) behind the C ABI of ``include/ibim.h``; :mod:`.ibim` is its ctypes
binding.
"""
from .ibim import (CTR2, FP64, HYB, KREG, MIXED, PRECOND_DIAG, PRECOND_NONE, REQ_ACTIVE, REQ_DONE, REQ_FAILED, REQ_WAITING,  # noqa: F401
                   SUM_DIRECT, SUM_TREE, IbimError, Problem, Server, header_functions, load)
