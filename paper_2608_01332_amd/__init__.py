"""Rake-compress tree-LQR solver for AMD MI355X (gfx950).

The solver is the C-ABI library librcr.so (include/rcr.h); `rcr` is its thin
ctypes binding and `workloads` the seeded synthetic inputs.
"""
from . import workloads  # noqa: F401
