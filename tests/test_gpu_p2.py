"""The product-form assembly on the GPU against the oracle: quadratic (P2) elements, and
linear ones on a mesh whose vertex degree exceeds the element-walk kernels' limits.

The library gets the vertex mesh and adds the edge nodes itself (knp_mesh_upload_p2);
the oracle builds its P2 case from the same vertex mesh.  Checked: the layout bit for
bit, the assembled values per entry within 1e-12 of the row's largest (summation order
only), f and the gates, and the solutions of the first steps within 1e-8 (FP64 levels)
and 1e-6 (FP32 levels) per block, in l2 and element-wise, on 2D and 3D Model A meshes
with the Hodgkin-Huxley membrane and the stimulus.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from knp_inputs import model_a_case  # noqa: E402
from knp_inputs.fan import fan_case  # noqa: E402
from oracle import timeloop  # noqa: E402
from oracle.assemble import Assembler, initial_gates, initial_state  # noqa: E402
from oracle.p2 import p2_case  # noqa: E402
from oracle.timeloop import advance_gates  # noqa: E402
from paper_2403_04491_amd import KnpSolver, amg_opts, solve_opts  # noqa: E402

DEV = torch.device("cuda", 0)
PARITY = dict(rtol=1e-12, restart=400, max_it=4000, reorth=1)

CASES = {
    "modelA2d_nx8_hh": lambda: model_a_case(2, 8, "hh", 1e-4, 3, stim=True),
    "modelA3d_nx4_hh": lambda: model_a_case(3, 4, "hh", 5e-5, 2, cfg_id=2),
    "modelA2d_nx16_leak": lambda: model_a_case(2, 16, "leak", 1e-4, 3),
}


def _blocks(info):
    Ni, Ne = info.N_i, info.N_e
    return {"c_i": np.r_[0:3 * Ni], "c_e": np.r_[4 * Ni:4 * Ni + 3 * Ne],
            "phi": np.r_[3 * Ni:4 * Ni, 4 * Ni + 3 * Ne:4 * (Ni + Ne)]}


@pytest.mark.parametrize("name", list(CASES))
def test_p2_assembly_matches_oracle(name):
    base = CASES[name]()
    case = p2_case(base)
    print(f"[P2 assembly] {name}", flush=True)
    s = KnpSolver(base, order=2)
    asm = Assembler(case)
    lay = asm.lay
    assert np.array_equal(s.rowptr, asm.rowptr) and np.array_equal(s.colidx, asm.colidx)
    u0 = initial_state(case, lay)
    assert np.array_equal(s.u.cpu().numpy(), u0)
    w0 = initial_gates(case, lay)
    rng = np.random.default_rng(7)
    u1 = u0 * (1.0 + 1e-3 * rng.standard_normal(u0.shape))
    u1[lay.pin_dof] = 0.0
    for n, u_prev in ((1, u0), (2, u1)):
        w_ref = advance_gates(case, lay, w0, u_prev, case.dt)
        ref = asm.assemble(u_prev, w_ref, n * case.dt, case.dt)
        s.u = torch.as_tensor(u_prev, device=DEV)
        s.gates = torch.as_tensor(w0, device=DEV).contiguous()
        s.assemble(n)
        vals = torch.empty(s.info.nnz_A, dtype=torch.float64, device=DEV)
        s.ctx.get_values(vals)
        sc = torch.empty(s.info.N, dtype=torch.float64, device=DEV)
        s.ctx.get_scaling(sc)
        sc = sc.cpu().numpy()
        A = ref.csr()
        rows = np.repeat(np.arange(lay.N), np.diff(A.indptr))
        want = A.data * sc[rows] * sc[A.indices]
        got = vals.cpu().numpy()
        rowmax = np.maximum.reduceat(np.abs(want), asm.rowptr[:-1])
        err = np.abs(got - want) / rowmax[rows]
        print(f"  step {n}: worst entry error {err.max():.2e} of the row's largest", flush=True)
        assert err.max() <= 1e-12, (n, err.max(), int(rows[err.argmax()]))
        f = s.f.cpu().numpy()
        for b in _blocks(s.info).values():
            scale = np.abs(ref.f[b]).max()
            if scale > 0:
                assert np.abs(f[b] - ref.f[b]).max() <= 1e-12 * scale
        hh = case.cell_model[lay.vert_cell[lay.gamma] - 1] == 1
        if np.any(hh):
            assert np.allclose(s.gates.cpu().numpy()[hh], w_ref[hh], rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("name,precision,tol,gauge", [
    ("modelA2d_nx8_hh", 0, 1e-8, 0), ("modelA3d_nx4_hh", 0, 1e-8, 0), ("modelA2d_nx16_leak", 0, 1e-8, 0),
    ("modelA2d_nx8_hh", 1, 1e-6, 0),
    # the system without the point condition (knp_set_gauge 1) reaches the same steps
    ("modelA2d_nx8_hh", 0, 1e-8, 1), ("modelA3d_nx4_hh", 1, 1e-6, 1),
])
def test_p2_time_steps_match_oracle(name, precision, tol, gauge):
    base = CASES[name]()
    case = p2_case(base)
    steps = base.n_steps
    print(f"[P2 steps] {name} steps={steps} precision={precision} gauge={gauge}", flush=True)
    ref = timeloop.run(case, n_steps=steps)["u"]
    s = KnpSolver(base, order=2, gauge=gauge, amg=amg_opts(precision=precision), solve=solve_opts(**PARITY))
    its = []
    for n in range(1, steps + 1):
        info = s.step()
        its.append(info.its)
        u = s.u.cpu().numpy()
        for k, b in _blocks(s.info).items():
            l2 = np.linalg.norm(u[b] - ref[n][b]) / np.linalg.norm(ref[n][b])
            inf = np.abs(u[b] - ref[n][b]).max() / np.abs(ref[n][b]).max()
            assert l2 <= tol and inf <= tol, (n, k, l2, inf)
    print(f"  its per step {its}", flush=True)


@pytest.mark.parametrize("membrane", ["leak", "hh"])
def test_high_degree_p1_mesh_matches_oracle(membrane):
    """A 2D fan whose centre vertex has 41 region neighbours (more than the 32 the walk
    kernels hold) takes the product-form path with linear elements: assembled values per
    entry within 1e-12 of the row's largest, and two steps within 1e-8 per block."""
    case = fan_case(membrane=membrane, n_steps=2)
    print(f"[high degree] {case.name}", flush=True)
    asm = Assembler(case)
    lay = asm.lay
    s = KnpSolver(case, solve=solve_opts(**PARITY))
    assert np.array_equal(s.rowptr, asm.rowptr) and np.array_equal(s.colidx, asm.colidx)
    u0 = initial_state(case, lay)
    w0 = initial_gates(case, lay)
    w1 = advance_gates(case, lay, w0, u0, case.dt)
    ref_sys = asm.assemble(u0, w1, case.dt, case.dt)
    s.assemble(1)
    vals = torch.empty(s.info.nnz_A, dtype=torch.float64, device=DEV)
    s.ctx.get_values(vals)
    sc = torch.empty(s.info.N, dtype=torch.float64, device=DEV)
    s.ctx.get_scaling(sc)
    sc = sc.cpu().numpy()
    A = ref_sys.csr()
    rows = np.repeat(np.arange(lay.N), np.diff(A.indptr))
    want = A.data * sc[rows] * sc[A.indices]
    rowmax = np.maximum.reduceat(np.abs(want), asm.rowptr[:-1])
    err = np.abs(vals.cpu().numpy() - want) / rowmax[rows]
    assert err.max() <= 1e-12, err.max()
    ref = timeloop.run(case, n_steps=2)["u"]
    s2 = KnpSolver(case, solve=solve_opts(**PARITY))
    for n in (1, 2):
        s2.step()
        u = s2.u.cpu().numpy()
        for k, b in _blocks(s2.info).items():
            l2 = np.linalg.norm(u[b] - ref[n][b]) / np.linalg.norm(ref[n][b])
            inf = np.abs(u[b] - ref[n][b]).max() / np.abs(ref[n][b]).max()
            assert l2 <= 1e-8 and inf <= 1e-8, (n, k, l2, inf)


def test_p2_rejects_the_order1_vjp():
    base = model_a_case(2, 8, "leak", 1e-4, 1)
    s = KnpSolver(base, order=2)
    s.assemble(1)
    from paper_2403_04491_amd import knp
    z = torch.zeros(s.info.N, dtype=torch.float64, device=DEV)
    with pytest.raises(knp.KnpError) as ei:
        s.ctx.step_vjp(s.u, s.u, z, z.clone())
    assert ei.value.status == 1
