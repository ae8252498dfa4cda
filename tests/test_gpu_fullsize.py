"""GPU checks at the benchmark's full size (4x4x4 lattice, 132^3 grid, N = 1.0e7), in the
launch configuration bench.py times (FP32-stored AMG, FGMRES(30), rtol 1e-6).

The oracle cannot factor this system, so these checks use what holds at any size:
* the product with A against SciPy on the downloaded matrix, every row;
* the constant-potential nullspace of the operator (Remark on the constant-potential
  nullspace): A e = 0 and A^T e = 0 for e = (0, 1_i, 0, 1_e), away from the rows and
  columns that the pin of phi_e changes;
* the stopping criterion of a solved step, recomputed on the CPU from the downloaded
  matrix, scaling and right-hand side.
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from knp_inputs import config_case  # noqa: E402
from paper_2403_04491_amd import KnpSolver, amg_opts, solve_opts  # noqa: E402
from paper_2403_04491_amd.simulate import AMG_BY_GAUGE  # noqa: E402

DEV = torch.device("cuda", 0)
RTOL = 1e-6


def T(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


@pytest.fixture(scope="module")
def full():
    case = config_case(3, n_steps=2)
    s = KnpSolver(case, amg=amg_opts(precision=1), solve=solve_opts(rtol=RTOL, restart=30, max_it=2000))
    s.assemble()
    print(f"  full size: N = {s.info.N}, nnz(A) = {s.info.nnz_A}", flush=True)
    return s


def host_matrix(s):
    """The stored system matrix S A S (S = diag(P_0)^{-1/2}) on the ABI pattern."""
    vals = torch.empty(s.info.nnz_A, dtype=torch.float64, device=DEV)
    s.ctx.get_values(vals)
    N = s.info.N
    return sp.csr_matrix((vals.cpu().numpy(), s.colidx, s.rowptr), shape=(N, N))


def test_fullsize_product_matches_scipy(full):
    s = full
    A = host_matrix(s)
    N = s.info.N
    x = np.random.default_rng(21).standard_normal(N)
    y = torch.empty(N, dtype=torch.float64, device=DEV)
    s.ctx.apply(0, T(x), y)
    ref = A @ x
    bound = 1e-13 * (abs(A) @ np.abs(x))
    err = np.abs(y.cpu().numpy() - ref)
    assert np.all(err <= bound + 1e-300), (int(np.argmax(err - bound)), float(err.max()))


def test_fullsize_constant_potential_nullspace(full):
    s = full
    A = host_matrix(s)
    Ni, Ne, N = s.info.N_i, s.info.N_e, s.info.N
    sc = torch.empty(N, dtype=torch.float64, device=DEV)
    s.ctx.get_scaling(sc)
    e = np.zeros(N)
    e[3 * Ni:4 * Ni] = 1.0
    e[4 * Ni + 3 * Ne:] = 1.0
    e /= sc.cpu().numpy()            # (S A S)(S^{-1} e) = S (A e)
    pin = s.info.pin_dof
    near_pin_rows = np.zeros(N, bool)
    rows = np.repeat(np.arange(N), np.diff(A.indptr))
    near_pin_rows[rows[A.indices == pin]] = True      # rows that lost their pinned-column entry
    near_pin_rows[pin] = True
    absA = abs(A)
    r = A @ e
    scale = (absA @ e).max()
    assert np.abs(r[~near_pin_rows]).max() <= 1e-13 * scale
    # columns: the pinned row keeps only its diagonal, so the columns it touched differ
    near_pin_cols = np.zeros(N, bool)
    near_pin_cols[s.colidx[s.rowptr[pin]:s.rowptr[pin + 1]]] = True
    near_pin_cols[pin] = True
    rt = A.T @ e
    assert np.abs(rt[~near_pin_cols]).max() <= 1e-13 * (absA.T @ e).max()


def test_fullsize_steps_meet_the_stopping_rule(full):
    """Step 1 (the noisy first step, FGMRES(200) as in the benchmark's warm-up) and step 2
    (FGMRES(30), the benchmark's timed configuration); after each, the scaled residual
    recomputed on the CPU meets rtol."""
    s = full
    N = s.info.N
    for n, restart in ((1, 200), (2, 30)):
        if n > 1:
            s.assemble()
        opts = solve_opts(rtol=RTOL, restart=restart, max_it=4000)
        x, info, ok = s.solve(opts=opts)
        assert ok, (n, info.its, info.rel_res)
        A = host_matrix(s)
        sc = torch.empty(N, dtype=torch.float64, device=DEV)
        s.ctx.get_scaling(sc)
        S = sc.cpu().numpy()
        b = s.f.cpu().numpy()
        xs = x.cpu().numpy()
        # ||S (b - A x)|| = ||S b - (S A S)(S^{-1} x)||
        rel = np.linalg.norm(S * b - A @ (xs / S)) / np.linalg.norm(S * b)
        print(f"  step {n}: {info.its} iterations, library {info.rel_res:.3e}, recomputed {rel:.3e}", flush=True)
        assert rel <= RTOL * (1 + 1e-6), rel
        assert abs(rel - info.rel_res) <= 1e-3 * rel
        s.u = x
        s.n = n


def _blocks(info):
    Ni, Ne = info.N_i, info.N_e
    return {"c_i": np.r_[0:3 * Ni], "c_e": np.r_[4 * Ni:4 * Ni + 3 * Ne],
            "phi": np.r_[3 * Ni:4 * Ni, 4 * Ni + 3 * Ne:4 * (Ni + Ne)]}


def _errs(info, u, ref):
    return {k: (float(np.linalg.norm(u[b] - ref[b]) / np.linalg.norm(ref[b])),
                float(np.abs(u[b] - ref[b]).max() / np.abs(ref[b]).max())) for k, b in _blocks(info).items()}


def test_fullsize_fp32_levels_against_fp64_levels_at_tight_tolerance():
    """Step 2 of the full-size lattice from the same u_1, solved to rtol 1e-12 with the
    hierarchy stored and applied in FP64 and again in FP32 (FP64 Arnoldi, Hessenberg
    problem, update and residual in both): every block within 1e-6 of the FP64-level
    solution, element-wise and in l2.  The benchmark's rtol-1e-6 solution of the same
    system is reported against the same reference."""
    case = config_case(3, n_steps=2)
    s = KnpSolver(case, amg=amg_opts(precision=0), solve=solve_opts(rtol=RTOL, restart=30, max_it=4000))
    print(f"[fp32 vs fp64 levels] {case.name} N = {s.info.N}", flush=True)
    s.step(opts=solve_opts(rtol=RTOL, restart=200, max_it=4000))      # u_1
    s.assemble()                                                      # A_1, f_2 (fixed below)
    tight = solve_opts(rtol=1e-12, restart=60, max_it=6000)
    ref, info64, ok64 = s.solve(opts=tight)
    assert ok64, (info64.its, info64.rel_res)
    s.ctx.amg_setup(amg_opts(precision=1))
    x32, info32, ok32 = s.solve(opts=tight)
    assert ok32, (info32.its, info32.rel_res)
    loose, info_l, ok_l = s.solve(opts=solve_opts(rtol=RTOL, restart=30, max_it=4000))
    r = ref.cpu().numpy()
    e32 = _errs(s.info, x32.cpu().numpy(), r)
    el = _errs(s.info, loose.cpu().numpy(), r)
    print(f"  FP64 levels {info64.its} its, FP32 levels {info32.its} its at rtol 1e-12; "
          f"FP32 vs FP64 (l2, element-wise) {e32}", flush=True)
    print(f"  rtol 1e-6 FP32-level solve ({info_l.its} its) vs the reference: {el}", flush=True)
    for k, (l2, inf) in e32.items():
        assert l2 <= 1e-6 and inf <= 1e-6, (k, l2, inf)


def test_fullsize_gauge1_against_gauge0_at_tight_tolerance():
    """Step 2 of the full-size lattice from the same (u_1, w_1): the point-condition
    system (gauge 0) solved with FP64 levels to rtol 1e-12 is the reference; the system
    without the condition (gauge 1), in the benchmark's configuration (FP32 levels, its
    tuned cycle), solved to rtol 1e-12 must meet it within 1e-6 per block, element-wise
    and in l2 (the same solution, Remark on the nullspace).  The rtol-1e-6 solves of the
    two gauges are reported against it; the stopping rule bounds neither's error, and
    gauge 1's potentials must be at least 100 times closer in l2 than gauge 0's."""
    case = config_case(3, n_steps=2)
    s0 = KnpSolver(case, amg=amg_opts(precision=0), solve=solve_opts(rtol=RTOL, restart=30, max_it=4000))
    print(f"[gauge 1 vs gauge 0] {case.name} N = {s0.info.N}", flush=True)
    s0.step(opts=solve_opts(rtol=RTOL, restart=200, max_it=4000))      # u_1, w_1
    u1, w1 = s0.u.clone(), s0.gates.clone()
    s0.assemble()
    tight = solve_opts(rtol=1e-12, restart=60, max_it=6000)
    ref, info0, ok0 = s0.solve(opts=tight)
    assert ok0, (info0.its, info0.rel_res)
    r = ref.cpu().numpy()
    loose0, info_l0, ok_l0 = s0.solve(opts=solve_opts(rtol=RTOL, restart=30, max_it=4000))
    assert ok_l0
    el0 = _errs(s0.info, loose0.cpu().numpy(), r)
    print(f"  gauge 0 rtol 1e-6 ({info_l0.its} its) vs the reference: {el0}", flush=True)
    del s0, loose0
    s1 = KnpSolver(case, gauge=1, amg=amg_opts(precision=1, **AMG_BY_GAUGE[1]),
                   solve=solve_opts(rtol=RTOL, restart=30, max_it=4000))
    s1.u, s1.gates, s1.n = u1, w1, 1
    s1.assemble()
    x1, info1, ok1 = s1.solve(opts=tight)
    assert ok1, (info1.its, info1.rel_res)
    loose, info_l, ok_l = s1.solve(opts=solve_opts(rtol=RTOL, restart=30, max_it=4000))
    assert ok_l
    e1 = _errs(s1.info, x1.cpu().numpy(), r)
    el = _errs(s1.info, loose.cpu().numpy(), r)
    print(f"  gauge 0 FP64 levels {info0.its} its, gauge 1 FP32 levels {info1.its} its at rtol 1e-12: {e1}",
          flush=True)
    print(f"  gauge 1 rtol 1e-6 ({info_l.its} its) vs the reference: {el}", flush=True)
    assert x1.cpu().numpy()[s1.info.pin_dof] == 0.0
    for k, (l2, inf) in e1.items():
        assert l2 <= 1e-6 and inf <= 1e-6, (k, l2, inf)
    assert el["phi"][0] * 100 <= el0["phi"][0], (el["phi"], el0["phi"])
