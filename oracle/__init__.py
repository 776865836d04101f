"""CPU FP64 oracle for the staggered-node PHS+poly RBF-FD Navier-Stokes path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call, link or execute anything in this package;
only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the GPU path: it is written from the paper
(Chu & Schmidt, "RBF-FD discretization of the Navier-Stokes equations on
scattered but staggered nodes") in plain NumPy/SciPy, FP64 throughout, one
step of the method at a time, in the paper's order and notation.

Modules
  knn        n-nearest-neighbour stencils (Sec. 2.2 / Sec. 4)
  weights    local PHS+poly saddle-point solves (Sec. 2.1, eqs. (4)-(9))
  operators  global sparse differentiation matrices (Sec. 2.2, eq. (10))
  cavity     fractional-step solver (Sec. 3, eqs. (14)-(21)) with LU solves
  metrics    test-function error and modified wavenumber (Sec. 4, eqs. (22)-(24))
  adjoint    reverse-mode derivative of the cavity step (transposed stages)
  cylinder   the step on the cylinder channel (Sec. 5.2): open boundary rows,
             drag and lift by Simpson's rule
"""
from . import knn, weights, operators, cavity, metrics, adjoint, cylinder  # noqa: F401

OP_ID = 1
OP_DX = 2
OP_DY = 4
OP_LAP = 8
