"""CPU FP64 oracle of the one-step ADER-WENO finite-volume scheme.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct
definition of what the hot path computes, written from the paper (Dumbser,
Zanotti, Hidalgo, Balsara, "ADER-WENO finite volume schemes with space-time
adaptive mesh refinement"), Sections 2 and 3.  Only the tests, the package's smoke
check and the benchmark's CPU-baseline leg may import it; the HIP product path
never does, and it shares no code, headers, tables or constant generators with
it.  Seeded inputs come from paper_1212_3585_amd.workloads, which holds none of
the method's arithmetic.

Modules:
  basis      nodal Lagrange basis at Gauss-Legendre nodes, exact 1D integrals
  weno       dimension-by-dimension polynomial WENO (Section 2.2)
  physics    Euler (Section 4.1), GLM-MHD (Section 4.2) and linear-advection
             fluxes and wave speeds
  predictor  space-time DG predictor with Picard iteration (Section 2.3)
  scheme     CFL time step, Rusanov / Osher face fluxes, finite-volume update (2.1)
  amr        cell-by-cell AMR with local time stepping: Loehner indicator,
             projection, averaging, memory-variable flux sums (Section 3)
  brute      independent brute-force routes used to pin the above

Every function is fp64 numpy; batching over cells is the only vectorisation.
"""
from .basis import Basis1D, basis, gauss_legendre  # noqa: F401
from .physics import Euler, GLMMHD, LinearAdvection  # noqa: F401
from .predictor import predict, spacetime_matrices  # noqa: F401
from .scheme import (Problem, all_cells, cfl_dt, run, step,  # noqa: F401
                     step_cells)
from .weno import reconstruct, stencils, weno_1d  # noqa: F401
