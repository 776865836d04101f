"""MI355X (gfx950) implementation of the staggered-node PHS+poly RBF-FD
Navier-Stokes hot path: stencil generation, batched weight solves, ELL
operator application and the fractional-step solver, behind the C ABI in
include/rbffd.h.  Importing this package loads librbffd.so (built by
``python paper_2206_06495_amd/build.py``); there is no CPU fallback.
"""
from .api import (build_nodes, knn, assemble_weights, ell_apply, ell_autotune, ELL_SHAPES,
                  ell_transpose, Transpose, cast_f32, Solver, LidRollout, step_batch, OP_ID, OP_DX,
                  OP_DY, OP_LAP)
from ._lib import RbfError, EXPORTED, LIB_PATH

__all__ = ["build_nodes", "knn", "assemble_weights", "ell_apply", "ell_autotune", "ELL_SHAPES",
           "ell_transpose", "Transpose",
           "cast_f32", "Solver", "LidRollout", "step_batch",
           "OP_ID", "OP_DX", "OP_DY", "OP_LAP", "RbfError", "EXPORTED", "LIB_PATH"]
