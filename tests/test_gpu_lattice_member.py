"""The config-3 lattice family at 8 grid intervals per cell pitch (4x4x4 jittered box cells,
32^3 grid x 6 tets, N = 178,124; 16 HH cells with the stimulus, 48 leak cells) against the
oracle's first two steps, stored by tests/golden/make_lattice_golden.py.

Element by element: every block's max |u - u_ref| / max |u_ref| and its l2 error within
1e-8 with FP64 levels and within 1e-6 with FP32-stored levels, each solve at rtol 1e-13
(a solve that stops at the attainable accuracy must still have reached 1e-12).  The gates of
the HH cells equal the oracle's Rush-Larsen step from the GPU's own previous state within 1e-13.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from knp_inputs import config_case  # noqa: E402
from oracle.assemble import initial_state  # noqa: E402
from oracle.mesh import build_layout  # noqa: E402
from oracle.timeloop import advance_gates  # noqa: E402
from paper_2403_04491_amd import KnpSolver, amg_opts, solve_opts  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lattice_pp8_oracle_steps.npz")
PARITY = dict(rtol=1e-13, restart=200, max_it=8000, reorth=1)


def _blocks(Ni, Ne):
    return {"c_i": np.r_[0:3 * Ni], "c_e": np.r_[4 * Ni:4 * Ni + 3 * Ne],
            "phi": np.r_[3 * Ni:4 * Ni, 4 * Ni + 3 * Ne:4 * (Ni + Ne)]}


@pytest.fixture(scope="module")
def reference():
    if not os.path.exists(GOLDEN):
        pytest.skip("stored oracle steps missing (run tests/golden/make_lattice_golden.py)")
    g = np.load(GOLDEN, allow_pickle=False)
    case = config_case(3, per_pitch=int(g["per_pitch"]))
    lay = build_layout(case)
    u = [initial_state(case, lay)]
    for d in g["increments"]:
        u.append(u[-1] + d)
    return case, lay, u


@pytest.mark.parametrize("precision,tol", [(0, 1e-8), (1, 1e-6)])
def test_lattice_member_matches_stored_oracle_steps(reference, precision, tol):
    case, lay, u_ref = reference
    n_steps = len(u_ref) - 1
    print(f"[lattice pp8] N = {lay.N}, {n_steps} stored steps, precision {precision}", flush=True)
    s = KnpSolver(case, amg=amg_opts(precision=precision), solve=solve_opts(**PARITY))
    assert s.info.N == lay.N
    order = np.argsort(s.gamma)
    assert np.array_equal(s.gamma[order], lay.gamma)
    B = _blocks(s.info.N_i, s.info.N_e)
    prev = s.u.cpu().numpy()
    assert np.array_equal(prev, u_ref[0])
    for n in range(1, n_steps + 1):
        w_own = advance_gates(case, lay, s.gates.cpu().numpy()[order], prev, case.dt)
        info = s.step(allow_noconv=True)
        assert info.rel_res <= 1e-12, (n, info.its, info.rel_res)
        u = s.u.cpu().numpy()
        errs = {k: (float(np.linalg.norm(u[b] - u_ref[n][b]) / np.linalg.norm(u_ref[n][b])),
                    float(np.abs(u[b] - u_ref[n][b]).max() / np.abs(u_ref[n][b]).max())) for k, b in B.items()}
        hh = case.cell_model[lay.vert_cell[lay.gamma] - 1] == 1      # gates evolve on HH cells only
        gown = float(np.abs(s.gates.cpu().numpy()[order][hh] - w_own[hh]).max())
        print(f"  step {n}: {info.its} its, rel_res {info.rel_res:.2e}; (l2, element-wise) {errs}; "
              f"gates vs oracle gating of the same state {gown:.1e}", flush=True)
        for k, (l2, inf) in errs.items():
            assert l2 <= tol and inf <= tol, (n, k, l2, inf)
        assert gown <= 1e-13, (n, gown)
        prev = u
