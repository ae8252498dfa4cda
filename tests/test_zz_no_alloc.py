"""knp_assemble_step_noalloc (the assembly with its scratch in the library's static device
array) against knp_assemble_step, through the C ABI.

Both run the same kernels on the same inputs, so the stored matrix S A S, f and the
advanced gates must agree bit for bit.  Two meshes in a row, the second smaller (the
static array keeps the first call's contents), plus the state and NaN error paths
(the NaN counter is cleared at the start of every call).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from knp_inputs import config_case, model_a_case  # noqa: E402
from paper_2403_04491_amd import KnpSolver, knp  # noqa: E402


def _outputs(s, which, u_prev, gates_in, n):
    g = gates_in.clone()
    f = torch.empty(s.info.N, dtype=torch.float64, device=s.dev)
    fn = s.ctx.assemble_step if which == "plain" else s.ctx.assemble_step_noalloc
    fn(n * s.case.dt, s.case.dt, u_prev, g, s.theta, f)
    vals = torch.empty(s.info.nnz_A, dtype=torch.float64, device=s.dev)
    s.ctx.get_values(vals)
    torch.cuda.synchronize()
    return vals.cpu().numpy(), f.cpu().numpy(), g.cpu().numpy()


@pytest.mark.parametrize("name,make", [
    ("lattice_4x4x4_pp4", lambda: config_case(3, per_pitch=4)),
    ("modelA3d_nx8_hh", lambda: model_a_case(3, 8, "hh", 5e-5, 2, cfg_id=2)),
])
def test_noalloc_assembly_matches_the_allocating_one(name, make):
    case = make()
    print(f"[noalloc] {name}", flush=True)
    s = KnpSolver(case)
    assert s.info.n_gamma > 0
    fresh = s.u.clone()
    f = torch.empty_like(fresh)
    with pytest.raises(knp.KnpError) as ei:         # the first assembly fixes S and P_0
        s.ctx.assemble_step_noalloc(case.dt, case.dt, fresh, s.gates.clone(), s.theta, f)
    assert ei.value.status == 2
    s.assemble(1)                                    # first assembly through the allocating call
    # a state with varied potentials and concentrations for the compared step
    gen = torch.Generator(device=s.dev).manual_seed(7)
    u_prev = s.u * (1.0 + 1e-3 * (torch.rand(s.info.N, dtype=torch.float64, device=s.dev, generator=gen) - 0.5))
    for n in (2, 3):
        ref = _outputs(s, "plain", u_prev, s.gates, n)
        got = _outputs(s, "noalloc", u_prev, s.gates, n)
        for a, b, what in zip(ref, got, ("values", "f", "gates")):
            assert np.array_equal(a, b), (name, n, what, float(np.abs(a - b).max()))
    bad = u_prev.clone()
    bad[3] = float("nan")
    with pytest.raises(knp.KnpError) as ei:
        s.ctx.assemble_step_noalloc(4 * case.dt, case.dt, bad, s.gates.clone(), s.theta, f)
    assert ei.value.status == 6
    # the counter left set by the NaN call is cleared by the next call
    ref = _outputs(s, "plain", u_prev, s.gates, 4)
    got = _outputs(s, "noalloc", u_prev, s.gates, 4)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
