"""Writes tests/golden/cfg2_oracle_steps.npz: the oracle's first steps of the 3D Model A
workload at N_x = 32 (one cell, Hodgkin-Huxley membrane with the stimulus, dt = 0.05 ms,
N = 149,900 unknowns).  Calls only the oracle and the seeded inputs.

Stored per step n: the increment u_n - u_{n-1} in float64 and the gates w_n; u_0 and w_0
follow from the seeded inputs.  (Float32 increments are not enough: the potentials move
by a fifth of their range in one step near the stimulus, so float32 rounding of the
increment alone is 1.3e-8 of max |phi| per step, above the 1e-8 parity bar.)  One oracle step (assembly + SuperLU) takes several minutes here.

    python tests/golden/make_cfg2_golden.py [n_steps]
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


def main():
    n_steps = int(sys.argv[1]) if len(sys.argv) > 1 else 3
    case = config_case(2)
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
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg2_oracle_steps.npz")
    np.savez_compressed(out, increments=np.stack(inc), gates=np.stack(gates), N=lay.N,
                        gamma=lay.gamma.astype(np.int32))
    print(f"wrote {out}")


if __name__ == "__main__":
    main()
