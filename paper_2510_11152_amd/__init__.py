"""MI355X-native matrix-free FAS multigrid (arXiv 2510.11152) on cell-centred grids.

The solver runs in hand-written HIP kernels behind the C ABI of include/fas.h
(libfas.so); this package only marshals torch tensors into those calls.
"""
from .api import Grid, heat, solve_mixed  # noqa: F401
