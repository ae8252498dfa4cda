"""Writes tests/golden/lattice_pp8_oracle_steps.npz: the oracle's first two steps of the
config-3 lattice family at 8 grid intervals per cell pitch (4x4x4 jittered box cells on a
32^3 grid x 6 tets, 16 HH cells with the stimulus and 48 leak cells, dt = 0.05 ms,
N = 178,124 unknowns).  Calls only the oracle and the seeded inputs.

Stored per step n: the increment u_n - u_{n-1} and the gates w_n, both in float64; u_0
and w_0 follow from the seeded inputs.  One oracle step (assembly + SuperLU) takes
several minutes on one core.

    python tests/golden/make_lattice_golden.py [n_steps]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from knp_inputs import config_case  # noqa: E402
from oracle import timeloop  # noqa: E402
from oracle.assemble import Assembler, initial_gates, initial_state  # noqa: E402

PER_PITCH = 8


def main():
    n_steps = int(sys.argv[1]) if len(sys.argv) > 1 else 2
    case = config_case(3, per_pitch=PER_PITCH)
    asm = Assembler(case)
    lay = asm.lay
    u = initial_state(case, lay)
    w = initial_gates(case, lay)
    inc, gates = [], []
    for n in range(1, n_steps + 1):
        t0 = time.perf_counter()
        u_new, w, _ = timeloop.step(asm, u, w, n, case.dt)
        inc.append(u_new - u)
        gates.append(w.copy())
        u = u_new
        print(f"step {n}: {time.perf_counter() - t0:.1f} s (N = {lay.N})", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"lattice_pp{PER_PITCH}_oracle_steps.npz")
    np.savez_compressed(out, increments=np.stack(inc), gates=np.stack(gates), N=lay.N, per_pitch=PER_PITCH,
                        gamma=lay.gamma.astype(np.int32))
    print(f"wrote {out}")


if __name__ == "__main__":
    main()
