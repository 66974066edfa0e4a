"""caskrylov for MI355X: SpMV-driven CG / GMRES with a cascaded kernel
predictor and asynchronous kernel switching (arXiv 2411.10143).

The compute path is libcaskrylov.so (HIP, gfx950); this package only binds
its C ABI.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import (Config, Features, SolveOpts, SolveResult, Matrix, CkError,  # noqa: F401
                       lib, spmv_create, spmv_destroy, spmv_features, spmv_select,
                       spmv_convert, spmv_apply, spmv_apply_f32, cg_solve, gmres_solve)
