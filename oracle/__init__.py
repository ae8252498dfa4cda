"""CPU oracle for the KNP-EMI time-step solve.  TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python binding)
never calls it and shares no code with it; the two meet only through the seeded
inputs of ``knp_inputs``.

What it computes is the plain definition of one step of the method: assemble the
IMEX-linearised KNP-EMI system A_{n-1} u_n = f_n (Sec. "Algebraic structure and
matrix assembly", eq. ``lin_sys``) exactly for P1 elements in float64, pin one
extracellular potential (Remark ``rem:nullspace``), and solve it with a sparse
direct LU (SciPy SuperLU, standing in for the paper's MUMPS).  Unpreconditioned
full GMRES and dense solves cross-check it on tiny meshes.

Modules
  mesh      region vertex sets, DOF numbering, membrane facets, structural pattern
  assemble  element/facet integrals, membrane models, block matrix, RHS, pin
  solve     sparse LU, dense solve, plain GMRES (optionally right-preconditioned)
  timeloop  the time loop with Rush-Larsen gating
  adjoint   discrete adjoint of the time loop

Parity pins live in ``tests/test_oracle_*.py``.  Functions without a pin say so in
their docstring ("parity unpinned").
"""
from . import mesh, assemble, solve, timeloop  # noqa: F401
