"""The oracle's time loop (Sec. "Time discretization").  Test infrastructure.

For n = 1..N_t: advance the gates with N_ode Rush-Larsen sub-steps at frozen
phi_M^{n-1} (Hodgkin-Huxley cells only), assemble A_{n-1}, f_n with u_{n-1} and
w_n, pin, and solve by sparse LU.  The state is never re-synchronised with
any other implementation.
"""
from __future__ import annotations

import numpy as np

from .assemble import Assembler, gamma_values, initial_gates, initial_state, rush_larsen
from .solve import lu_solve


def advance_gates(case, lay, gates, u_prev, dt):
    """w_n from w_{n-1} at the membrane vertices of Hodgkin-Huxley cells."""
    p = case.params
    _, _, phiM = gamma_values(lay, u_prev)
    hh = case.cell_model[lay.vert_cell[lay.gamma] - 1] == 1
    out = np.array(gates, dtype=np.float64, copy=True)
    if np.any(hh):
        out[hh] = rush_larsen(gates[hh], phiM[hh], p["phi_rest"], dt, p["n_ode"])
    return out


def step(asm: Assembler, u_prev, gates_prev, n, dt, theta=None):
    """One time step: returns (u_n, w_n, system)."""
    t_n = n * dt
    gates = advance_gates(asm.case, asm.lay, gates_prev, u_prev, dt)
    sys_ = asm.assemble(u_prev, gates, t_n, dt, theta)
    u = lu_solve(sys_.csr(), sys_.f)
    return u, gates, sys_


def run(case, n_steps=None, theta=None, asm=None, keep_systems=False):
    """Run the time loop from the case's initial state; returns dict of histories."""
    asm = asm or Assembler(case)
    lay = asm.lay
    u = initial_state(case, lay)
    w = initial_gates(case, lay)
    n_steps = case.n_steps if n_steps is None else n_steps
    us, ws, systems = [u], [w], []
    for n in range(1, n_steps + 1):
        u, w, s = step(asm, u, w, n, case.dt, theta)
        us.append(u)
        ws.append(w)
        if keep_systems:
            systems.append(s)
    return {"u": us, "gates": ws, "systems": systems, "asm": asm}
