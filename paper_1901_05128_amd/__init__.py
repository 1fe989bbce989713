"""MI355X-native convolution-quadrature solver for the two-state fractional
Fokker-Planck system (Sun, Nie & Deng): direct and fast (sum-of-geometric-
sequences) BE and BDF2 CQ, behind the C ABI of include/cqfp.h.

The Python side only marshals arguments to libcqfp.so (see _lib)."""
from ._lib import (CQError, Grid, Info, Params, Solver, cq_fast_rule, cq_history, cq_history_noalloc, cq_weights,
                   fp_solve,
                   lib, make_grid, make_params, params_of, prof_enable, prof_read, fp_solve_batched, fp_adjoint,
                   Adjoint,
                   BatchReport, SOLVER_NODAL, SOLVER_MODAL, BATCH_DEFAULT, BATCH_AUTOTUNE, BATCH_TIME_BLOCKED,
                   BATCH_MFMA_TILE, BATCH_PER_STEP)

__all__ = ["CQError", "Grid", "Info", "Params", "Solver", "cq_fast_rule", "cq_history", "cq_history_noalloc",
           "cq_weights",
           "fp_solve", "lib", "make_grid", "make_params", "params_of", "prof_enable", "prof_read", "fp_solve_batched", "fp_adjoint", "Adjoint", "BatchReport", "SOLVER_NODAL",
           "SOLVER_MODAL", "BATCH_DEFAULT", "BATCH_AUTOTUNE", "BATCH_TIME_BLOCKED", "BATCH_MFMA_TILE", "BATCH_PER_STEP"]
