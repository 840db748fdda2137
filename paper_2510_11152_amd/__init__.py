"""MI355X-native matrix-free FAS multigrid (arXiv 2510.11152) on cell-centred and staggered grids.

The solver runs in hand-written HIP kernels behind the C ABI of include/fas.h
(libfas.so); this package only marshals torch tensors into those calls.
"""
from .api import (Grid, UnevenBatch, heat, solve_batched, solve_mixed, solve_stacked_mixed,  # noqa: F401
                  solve_uneven)
from .autograd import HeatSolveFn, heat_loss_and_grads  # noqa: F401
from .grain import GrainGrowth, count_grains, grain_map, grain_rhs  # noqa: F401
from .staggered import NavierStokes2D, StaggeredSolver  # noqa: F401
