"""MI355X-native KNP-EMI time-step solve (assembly + AMG(P_0)-preconditioned GMRES).

The compute path is libknp.so (HIP kernels for gfx950 behind the C ABI in
include/knp.h); this package only marshals arguments (``knp``) and drives the time
loop (``simulate``).  Importing it loads the library and fails loudly if it has
not been built.
"""
from . import knp  # noqa: F401
from .knp import Context, KnpError, amg_opts, solve_opts  # noqa: F401

knp.lib()

from .simulate import KnpSolver  # noqa: E402,F401
