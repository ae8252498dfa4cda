"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it pins.  None of them re-types the oracle's
formulas: they check exact counts printed in the paper, brute-force
enumerations, algebraic identities the discrete system must satisfy, closed-form
special cases, and paper-printed values.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from conftest import golden
from knp_inputs import config_case, model_a_case, model_a_evolution_case
from oracle import timeloop
from oracle.assemble import (Assembler, bulk_coo, gamma_coo, gamma_values, hh_rates,
                             initial_gates, initial_state, kir_factor, membrane_terms,
                             pump_flux, rush_larsen, p0_values, stimulus)
from oracle.mesh import build_layout, structural_pattern
from oracle.p2 import p2_case
from oracle.solve import dense_solve, gmres, lu_solve


def dof_formula(nx, d, p=1, K=3):
    """N = ((p N_x + 1)^d + (3 - d/2)(p N_x)^(d-1) + 2(d - 2)) (|K| + 1), Sec. "Model A"."""
    return int(round(((p * nx + 1) ** d + (3 - d / 2) * (p * nx) ** (d - 1) + 2 * (d - 2)) * (K + 1)))


# --------------------------------------------------------------------------- counts
@pytest.mark.parametrize("row", golden("table2_dofs.txt"))
def test_table2_dof_counts(row):
    nx, N = int(row[0]), int(row[1])
    assert dof_formula(nx, 2) == N
    lay = build_layout(model_a_case(2, nx))
    assert lay.N == N


@pytest.mark.parametrize("d,nx", [(2, 4), (2, 8), (3, 4), (3, 8), (3, 12)])
def test_dof_formula_small(d, nx):
    lay = build_layout(model_a_case(d, nx))
    assert lay.N == dof_formula(nx, d)
    # duplicated membrane vertices: N_i + N_e - n_vert = |Gamma vertices|
    assert sum(lay.N_r) - lay.n_vert == len(lay.gamma)


@pytest.mark.parametrize("d,nx", [(2, 4), (2, 8), (2, 16), (3, 4), (3, 8)])
def test_dof_formula_p2(d, nx):
    """The DOF-count formula of Sec. "Model A" for p = 2: vertex and edge nodes, the
    membrane ones duplicated."""
    lay = build_layout(p2_case(model_a_case(d, nx)))
    assert lay.N == dof_formula(nx, d, p=2)
    assert sum(lay.N_r) - lay.n_vert == len(lay.gamma)


def test_dof_count_p2_at_the_largest_robustness_case():
    """Sec. "Iterative solver robustness" prints N = 4.2e6 for (N_x, p) = (512, 2)."""
    lay = build_layout(p2_case(model_a_case(2, 512)))
    assert lay.N == dof_formula(512, 2, p=2) == 4210692
    assert round(lay.N / 1e5) == 42


def _brute_pattern(case):
    """Structural pattern by plain set enumeration over elements and facets."""
    lay = build_layout(case)
    Ni, Ne = lay.N_r
    off = (0, 4 * Ni)
    Nr = (Ni, Ne)
    pairs = [set(), set()]
    for e, t in zip(case.elem.tolist(), case.tag.tolist()):
        r = 0 if t >= 1 else 1
        for a in e:
            for b in e:
                pairs[r].add((a, b))
    gam = set()
    for f in lay.facets.tolist():
        for a in f:
            for b in f:
                gam.add((a, b))
    ent = set()
    loc = lay.loc
    for r in (0, 1):
        q = 1 - r
        for (a, b) in pairs[r]:
            ja, jb = loc[r, a], loc[r, b]
            for k in range(3):
                ent.add((off[r] + k * Nr[r] + ja, off[r] + k * Nr[r] + jb))
                ent.add((off[r] + k * Nr[r] + ja, off[r] + 3 * Nr[r] + jb))
                ent.add((off[r] + 3 * Nr[r] + ja, off[r] + k * Nr[r] + jb))
            ent.add((off[r] + 3 * Nr[r] + ja, off[r] + 3 * Nr[r] + jb))
        for (a, b) in gam:
            ja, jb = loc[r, a], loc[q, b]
            for f in range(4):
                ent.add((off[r] + f * Nr[r] + ja, off[q] + 3 * Nr[q] + jb))
    return lay, pairs, gam, ent


@pytest.mark.parametrize("d,nx,N,nnz", [(2, 4, 132, 1802), (3, 4, 604, 16390)])
def test_pattern_bruteforce_tiny(d, nx, N, nnz):
    case = model_a_case(d, nx)
    lay, pairs, gam, ent = _brute_pattern(case)
    rowptr, colidx = structural_pattern(case, lay)
    assert lay.N == N
    assert len(colidx) == nnz == len(ent)
    # closed form nnz = 10 sum_r P_r + 8 P_Gamma for three ions
    assert nnz == 10 * (len(pairs[0]) + len(pairs[1])) + 8 * len(gam)
    rows = np.repeat(np.arange(lay.N), np.diff(rowptr))
    got = set(zip(rows.tolist(), colidx.tolist()))
    assert got == ent
    # columns strictly ascending within each row
    for i in range(lay.N):
        seg = colidx[rowptr[i]:rowptr[i + 1]]
        assert np.all(np.diff(seg) > 0)


def test_pattern_config1_and_interior_row_lengths():
    case = config_case(1)
    asm = Assembler(case)
    assert asm.lay.N == 4612 and len(asm.colidx) == 77066
    lens = np.diff(asm.rowptr)
    # 2D right-diagonal split: 6 neighbours + self -> c-rows 14, phi-rows 28 in the interior
    assert np.bincount(lens).argmax() in (14,)
    assert 28 in set(lens.tolist())
    case3 = model_a_case(3, 8)
    asm3 = Assembler(case3)
    lens3 = np.diff(asm3.rowptr)
    # 3D Kuhn split: 14 neighbours + self -> c-rows 30, phi-rows 60 in the interior
    assert lens3.max() >= 60 and 30 in set(lens3.tolist()) and 60 in set(lens3.tolist())


# --------------------------------------------------------------------------- algebra
@pytest.fixture(scope="module")
def run2d():
    case = config_case(1)
    return case, timeloop.run(case, n_steps=2, keep_systems=True)


@pytest.fixture(scope="module")
def run3d():
    case = model_a_case(3, 8, "hh", 5e-5, 2, cfg_id=2)
    return case, timeloop.run(case, n_steps=2, keep_systems=True)


@pytest.fixture(scope="module")
def run2d_p2():
    case = p2_case(model_a_case(2, 8, "hh", 1e-4, 2, stim=True))
    return case, timeloop.run(case, n_steps=2, keep_systems=True)


@pytest.fixture(scope="module")
def run3d_p2():
    case = p2_case(model_a_case(3, 4, "hh", 5e-5, 2, cfg_id=2))
    return case, timeloop.run(case, n_steps=2, keep_systems=True)


@pytest.fixture(scope="module")
def run3d_kir():
    case = model_a_case(3, 8, "kir", 5e-5, 2, cfg_id=2)
    return case, timeloop.run(case, n_steps=2, keep_systems=True)


@pytest.mark.parametrize("which", ["run2d", "run3d", "run3d_kir", "run2d_p2", "run3d_p2"])
def test_nullspace_unpinned(which, request):
    """The unpinned operator annihilates e = (0, 1_i, 0, 1_e) from both sides and the
    potential rows of f sum to zero (Remark on the constant-potential nullspace)."""
    case, res = request.getfixturevalue(which)
    asm = res["asm"]
    lay = asm.lay
    Ni, Ne = lay.N_r
    s = asm.assemble(res["u"][1], res["gates"][1], 2 * case.dt, case.dt, pin=False)
    A = s.csr()
    e = np.zeros(lay.N)
    e[3 * Ni:4 * Ni] = 1.0
    e[4 * Ni + 3 * Ne:] = 1.0
    absA = abs(A)
    assert np.abs(A @ e).max() <= 1e-13 * (absA @ e).max()
    assert np.abs(A.T @ e).max() <= 1e-13 * (absA.T @ e).max()
    assert abs(e @ s.f) <= 1e-13 * np.abs(s.f * e).sum()


def test_cell_potential_near_null_vectors():
    """The constant intracellular potential of one cell, z_k, is a near-null vector of the
    operator from both sides: every bulk term of a row is a divergence form, so A z_k and
    z_k^T A keep only the membrane terms of cell k (the capacitive weight C_m/F times the
    membrane mass, eq. ``weak_disc``), and z_k^T A z_j is 0 for j != k and C_m/F times the
    membrane area of cell k for j = k.  The area is the closed form 2(ab + bc + ca) of the
    grid-aligned box cell, from the extent of its intracellular vertices."""
    case = config_case(3, per_pitch=4)
    asm = Assembler(case)
    lay = asm.lay
    Ni, Ne = lay.N_r
    u = initial_state(case, lay)
    s = asm.assemble(u, initial_gates(case, lay), case.dt, case.dt, pin=False)
    A = s.csr()
    absA = abs(A)
    Vi, Ve = np.asarray(lay.verts[0]), np.asarray(lay.verts[1])
    cell_i = lay.vert_cell[Vi]
    on_gamma = np.zeros(lay.n_vert, bool)
    on_gamma[lay.gamma] = True
    # cell of every DOF's vertex when that vertex is on the membrane, else 0
    dof_cell = np.zeros(lay.N, np.int64)
    for f in range(4):
        dof_cell[f * Ni:(f + 1) * Ni] = np.where(on_gamma[Vi], cell_i, 0)
        dof_cell[4 * Ni + f * Ne:4 * Ni + (f + 1) * Ne] = np.where(on_gamma[Ve], lay.vert_cell[Ve], 0)
    cells = np.unique(cell_i[cell_i > 0])
    assert len(cells) == 64
    Z = np.zeros((lay.N, len(cells)))
    for j, k in enumerate(cells):
        Z[3 * Ni + np.nonzero(cell_i == k)[0], j] = 1.0
    AZ, ZA = A @ Z, (A.T @ Z)
    scale_r, scale_c = (absA @ Z).max(), (absA.T @ Z).max()
    E = Z.T @ AZ
    Eabs = Z.T @ (absA @ Z)     # the scale of the rounding in E (the stiffness sums cancel)
    Cm_F = case.params["C_m"] / case.params["F"]
    for j, k in enumerate(cells):
        off = dof_cell != k
        assert np.abs(AZ[off, j]).max() <= 1e-13 * scale_r
        assert np.abs(ZA[off, j]).max() <= 1e-13 * scale_c
        assert np.abs(AZ[~off, j]).max() > 1e-6 * scale_r
        ext = np.ptp(case.xyz[Vi[cell_i == k]], axis=0)
        area = 2.0 * (ext[0] * ext[1] + ext[1] * ext[2] + ext[2] * ext[0])
        assert abs(E[j, j] - Cm_F * area) <= 1e-13 * Eabs[j, j]
    off_diag = E - np.diag(np.diag(E))
    assert np.abs(off_diag).max() <= 1e-13 * Eabs.max()


def _mass(case, lay, r):
    rr, cc, vv = bulk_coo(case, lay, r, kind="mass")
    return sp.coo_matrix((vv, (rr, cc)), shape=(lay.N_r[r],) * 2).tocsr()


def _gmass(case, lay, weight=None):
    gr, gc, gv = gamma_coo(case, lay, weight)
    return sp.coo_matrix((gv, (gr, gc)), shape=(lay.n_vert,) * 2).tocsr()


@pytest.mark.parametrize("which", ["run2d", "run3d", "run3d_kir", "run2d_p2", "run3d_p2"])
def test_invariants(which, request):
    """I1: sum_k z_k c_k is unchanged at every node (electroneutrality, eq. ``knp``).
    I2: per cell, C_m int (phi_M^n - phi_M^{n-1}) = -dt int I_ch (test w = 1 on the
        cell in eq. ``weak_disc2``).
    I3: per ion and region, int (c^n - c^{n-1}) = -sgn_r/(F z_k) [dt int I^k +
        C_m int alpha_r^k (phi_M^n - phi_M^{n-1})] (test v = 1 in eq. ``weak_disc``).
    """
    case, res = request.getfixturevalue(which)
    asm = res["asm"]
    lay = asm.lay
    p = case.params
    z = np.array(p["z"])
    F, Cm = p["F"], p["C_m"]
    u0, u1 = res["u"][0], res["u"][1]
    mem = res["systems"][0].mem
    for r in (0, 1):
        idx = np.arange(lay.N_r[r])
        q0 = sum(z[k] * u0[lay.dof(r, k, idx)] for k in range(3))
        q1 = sum(z[k] * u1[lay.dof(r, k, idx)] for k in range(3))
        # round-off floor: the pinned node's potential equation is only implied by
        # the others, so its charge balance carries their accumulated rounding
        assert np.abs(q1 - q0).max() <= 1e-9 * 137.0

    def on_gamma(x):
        y = np.zeros(lay.n_vert)
        y[lay.gamma] = x
        return y

    MG = _gmass(case, lay)
    _, _, ph0 = gamma_values(lay, u0)
    _, _, ph1 = gamma_values(lay, u1)
    dph = on_gamma(ph1 - ph0)
    ones_cell = on_gamma(np.ones(len(lay.gamma)))
    lhs = Cm * ones_cell @ (MG @ dph)
    rhs = -case.dt * ones_cell @ (MG @ on_gamma(mem.I.sum(axis=1)))
    assert abs(lhs - rhs) <= 1e-6 * abs(rhs)

    for r in (0, 1):
        sgn = 1.0 if r == 0 else -1.0
        M = _mass(case, lay, r)
        idx = np.arange(lay.N_r[r])
        for k in range(3):
            c0 = u0[lay.dof(r, k, idx)]
            dc = u1[lay.dof(r, k, idx)] - c0
            content = abs(M.sum(axis=0).A1 @ c0)
            lhs = M.sum(axis=0).A1 @ dc
            MGa = _gmass(case, lay, on_gamma(mem.alpha[r, :, k]))
            rhs = -sgn / (F * z[k]) * (case.dt * np.ones(lay.n_vert) @ (MG @ on_gamma(mem.I[:, k]))
                                        + Cm * np.ones(lay.n_vert) @ (MGa @ dph))
            assert abs(lhs - rhs) <= 1e-11 * content
            assert abs(rhs) > 1e-6 * abs(lhs - rhs) + 0.0


# --------------------------------------------------------------------------- membrane
def test_hh_steady_state_matches_table():
    p = config_case(1).params
    alpha, beta = hh_rates(np.array([p["phi_M0"]]), p["phi_rest"])
    w_inf = (alpha / (alpha + beta))[0]
    printed = {r[0]: float(r[1]) for r in golden("hh_initial_gates.txt")}
    for i, name in enumerate("nmh"):
        assert abs(w_inf[i] - printed[name]) < 1.5e-3, (name, w_inf[i], printed[name])


def test_hh_rates_removable_points():
    """alpha_n at V = 10 mV and alpha_m at V = 25 mV equal their limits 0.1 and 1 /ms."""
    rest = -0.065
    a, _ = hh_rates(np.array([rest + 0.010, rest + 0.025]), rest)
    assert abs(a[0, 0] - 100.0) < 1e-12 and abs(a[1, 1] - 1000.0) < 1e-12
    eps = 1e-9
    a2, _ = hh_rates(np.array([rest + 0.010 + eps, rest + 0.025 + eps]), rest)
    assert abs(a2[0, 0] - 100.0) < 1e-4 and abs(a2[1, 1] - 1000.0) < 1e-3


def test_rush_larsen_composes_exactly():
    """With phi_M frozen the gating ODE is linear with constant coefficients, so n
    Rush-Larsen sub-steps equal the exact solution over dt."""
    rng = np.random.default_rng(0)
    phi = rng.uniform(-0.09, 0.04, size=64)
    w0 = rng.uniform(0, 1, size=(64, 3))
    dt = 5e-5
    got = rush_larsen(w0, phi, -0.065, dt, 25)
    a, b = hh_rates(phi, -0.065)
    winf = a / (a + b)
    exact = winf + (w0 - winf) * np.exp(-(a + b) * dt)
    assert np.abs(got - exact).max() < 1e-14


def test_no_channels_uniform_state_is_stationary():
    """All conductances zero and uniform electroneutral data: u_n = u_0 exactly."""
    case = model_a_case(2, 16, "leak", 1e-4, 3)
    case.params["g_leak"] = [0.0, 0.0, 0.0]
    for r, base in enumerate((case.params["conc_i0"], case.params["conc_e0"])):
        for k in range(3):
            case.conc0[r, k] = base[k]
    res = timeloop.run(case)
    for u in res["u"][1:]:
        # sparse-LU rounding floor of this system (cond > 1e10) is ~1e-11 relative
        assert np.abs(u - res["u"][0]).max() <= 1e-10 * np.abs(res["u"][0]).max()


def test_sign_of_h_is_pinned():
    """Flipping the printed sign of h breaks the per-cell capacitive balance I2."""
    case = config_case(1)
    asm = Assembler(case)
    lay = asm.lay
    u0 = initial_state(case, lay)
    w0 = initial_gates(case, lay)
    s = asm.assemble(u0, w0, case.dt, case.dt)
    # h_r must equal sum_k z_k g_r^k (what eq. weak_disc2 needs to be the sum of weak_disc)
    z = np.array(case.params["z"])
    for r in (0, 1):
        assert np.allclose(s.mem.h[r], (s.mem.g[r] * z[None, :]).sum(axis=1), rtol=1e-13, atol=0)


# --------------------------------------------------------------------------- solvers
@pytest.mark.parametrize("d", [2, 3])
def test_tiny_bruteforce_solves_agree(d):
    case = model_a_case(d, 4, "hh" if d == 3 else "leak", 1e-4, 1)
    asm = Assembler(case)
    lay = asm.lay
    s = asm.assemble(initial_state(case, lay), initial_gates(case, lay), case.dt, case.dt)
    A = s.csr()
    x_lu = lu_solve(A, s.f)
    x_de = dense_solve(A, s.f)
    # full GMRES on the symmetrically diagonally scaled system (same solution)
    dsc = 1.0 / np.sqrt(A.diagonal())
    S = sp.diags(dsc)
    y, info = gmres(S @ A @ S, dsc * s.f, restart=None, rtol=1e-15, maxiter=lay.N)
    x_gm = dsc * y
    scale = np.abs(x_de).max()
    assert np.abs(x_lu - x_de).max() <= 1e-12 * scale
    assert np.abs(x_gm - x_de).max() <= 1e-12 * scale


@pytest.mark.parametrize("row", golden("lu_p0_iterations.txt"))
def test_lu_p0_gmres_iteration_count(row):
    """GMRES preconditioned by the exact block-diagonal P_0 converges in 3-4
    iterations on Model A 2D (Sec. "Iterative solver robustness").  The criterion
    is the preconditioned relative residual (left preconditioning), the default
    of the solver library the paper uses; initial guess u_0 as in Sec. "Solver
    configurations".  Model A has uniform initial concentrations."""
    dt, printed = float(row[0]), int(row[1])
    case = model_a_case(2, 32, "hh", dt, 1)
    for r, base in enumerate((case.params["conc_i0"], case.params["conc_e0"])):
        for k in range(3):
            case.conc0[r, k] = base[k]
    asm = Assembler(case)
    lay = asm.lay
    u0 = initial_state(case, lay)
    s = asm.assemble(u0, initial_gates(case, lay), dt, dt)
    A = s.csr()
    P0 = sp.csr_matrix((p0_values(s, lay), s.colidx, s.rowptr), shape=A.shape)
    lu = spla.splu(sp.csc_matrix(P0))
    _, info = gmres(lambda v: lu.solve(A @ v), lu.solve(s.f), x0=u0, restart=30,
                    rtol=1e-6, maxiter=100)
    assert 3 <= info["its"] <= 4 and (printed == 3 or info["its"] == printed), info["its"]
    _, info0 = gmres(A, s.f, x0=u0, restart=30, rtol=1e-6, maxiter=300)
    assert info0["its"] >= 100          # unpreconditioned GMRES stalls (same section)


@pytest.mark.parametrize("row", golden("lu_p0_iterations.txt"))
def test_lu_p0_gmres_iteration_count_p2(row):
    """The same 3-4 iterations with quadratic elements, which the same section states
    for p in {1, 2} (N_x = 16, N = 4,612)."""
    dt, printed = float(row[0]), int(row[1])
    case = p2_case(model_a_case(2, 16, "hh", dt, 1, noise=0.0))
    asm = Assembler(case)
    lay = asm.lay
    u0 = initial_state(case, lay)
    s = asm.assemble(u0, initial_gates(case, lay), dt, dt)
    A = s.csr()
    P0 = sp.csr_matrix((p0_values(s, lay), s.colidx, s.rowptr), shape=A.shape)
    lu = spla.splu(sp.csc_matrix(P0))
    _, info = gmres(lambda v: lu.solve(A @ v), lu.solve(s.f), x0=u0, restart=30,
                    rtol=1e-6, maxiter=100)
    assert 3 <= info["its"] <= 4 and (printed == 3 or info["its"] == printed), info["its"]


# --------------------------------------------------------------------------- Kir-Na/K
# Sec. "Passive dynamics: Kir--Na/K" and Table "Physical parameters".
def test_kir_factor_at_both_half_activation_points():
    """C and D are logistic factors with midpoints dphi_K = -18.5 mV and phi_M =
    -118.6 mV, where each equals 2; with E_K^0 = -118.6 mV also B = 2 and [K+]_e =
    [K+]_e^0 leaves f_Kir = A / 2."""
    got = kir_factor(4.0, -0.0185, -0.1186, -0.1186, 4.0)
    assert abs(got - (1.0 + np.exp(0.433)) / 2.0) < 1e-15


def test_kir_factor_normalisation_and_concentration_scaling():
    """At the initial state (phi_M = E_K = E_K^0, [K+]_e = [K+]_e^0) the factor is 1 up
    to the rounding of 18.5/42.5 = 0.4353 to the printed 0.433; it grows as the square
    root of [K+]_e at fixed potentials."""
    p = config_case(1).params
    psi = p["R"] * p["T"] / p["F"]
    E_K0 = psi * np.log(p["conc_e0"][1] / p["conc_i0"][1])
    f0 = kir_factor(4.0, 0.0, E_K0, E_K0, 4.0)
    assert abs(f0 - 1.0) < 2e-3
    for s in (0.25, 2.0, 9.0):
        assert abs(kir_factor(4.0 * s, 0.01, -0.07, E_K0, 4.0) / kir_factor(4.0, 0.01, -0.07, E_K0, 4.0)
                   - np.sqrt(s)) < 1e-14


def test_kir_factor_rectifies_inward():
    """Inward rectification: at fixed phi_M the conductance falls as the driving force
    phi_M - E_K grows (outward current limited) and tends to a finite limit for a
    large inward driving force; at fixed dphi_K it rises with phi_M."""
    d = np.linspace(-0.1, 0.1, 41)
    f = kir_factor(4.0, d, -0.07, -0.089, 4.0)
    assert np.all(np.diff(f) < 0)
    lim = kir_factor(4.0, -1.0, -0.07, -0.089, 4.0)
    assert abs(lim - kir_factor(4.0, -2.0, -0.07, -0.089, 4.0)) < 1e-8 * lim
    ph = np.linspace(-0.12, 0.0, 25)
    assert np.all(np.diff(kir_factor(4.0, 0.0, ph, -0.089, 4.0)) > 0)


def test_pump_flux_saturation():
    """Half-saturation at the thresholds, the 3/2-power in [Na+]_i (4 P_Na gives
    8/9), and the maximum rate rho_pump for large concentrations."""
    rho, PNa, PK = 1.115e-6, 10.0, 1.5
    assert abs(pump_flux(PNa, PK, rho, PNa, PK) - rho / 4) < 1e-15 * rho
    assert abs(pump_flux(4 * PNa, PK, rho, PNa, PK) - rho * (8 / 9) / 2) < 1e-15 * rho
    assert abs(pump_flux(1e12, 1e12, rho, PNa, PK) - rho) < 1e-15
    assert pump_flux(0.0, 4.0, rho, PNa, PK) == 0.0 and pump_flux(12.0, 0.0, rho, PNa, PK) == 0.0


def _kir_terms(g_leak=None, rho=None, model=2, at_thresholds=False):
    case = model_a_case(2, 8, "kir", 1e-4, 1)
    case.cell_model[:] = model
    if g_leak is not None:
        case.params["g_leak"] = g_leak
    if rho is not None:
        case.params["rho_pump"] = rho
    lay = Assembler(case).lay
    u0 = initial_state(case, lay)
    if at_thresholds:      # ICS Na+ = P_Na and ECS K+ = P_K on the membrane
        u0[lay.dof(0, 0, lay.loc[0, lay.gamma])] = case.params["P_Na"]
        u0[lay.dof(1, 1, lay.loc[1, lay.gamma])] = case.params["P_K"]
    return case, lay, membrane_terms(case, lay, u0, None, case.dt, case.dt)


def test_pump_moves_three_na_out_per_two_k_in():
    """With every channel closed only the pump acts: the Na+ and K+ membrane fluxes
    I_k / (F z_k) are 3 j and -2 j (outward positive), Cl- carries nothing, and the
    net current is F j_pump > 0."""
    case, lay, mem = _kir_terms(g_leak=[0.0, 0.0, 0.0])
    p = case.params
    z = np.array(p["z"])
    flux = mem.I / (p["F"] * z[None, :])
    j = flux[:, 0] / 3.0
    assert np.all(j > 0)
    assert np.allclose(flux[:, 1], -2.0 * j, rtol=1e-14, atol=0)
    assert np.all(flux[:, 2] == 0)
    assert np.allclose(mem.I.sum(axis=1), p["F"] * j, rtol=1e-13, atol=0)
    # the pump reads the ICS Na+ and the ECS K+: at their thresholds j = rho / 4
    case, lay, mem = _kir_terms(g_leak=[0.0, 0.0, 0.0], at_thresholds=True)
    j = mem.I[:, 0] / (3.0 * p["F"] * z[0])
    assert np.allclose(j, p["rho_pump"] / 4, rtol=1e-14, atol=0)


def test_kir_reduces_to_leak_without_pump():
    """rho_pump = 0: Na+ and Cl- currents equal the leak model's; the K+ current is the
    leak current times f_Kir, which is below 1 here since phi_M^0 lies above E_K."""
    _, _, leak = _kir_terms(rho=0.0, model=0)
    _, _, kir = _kir_terms(rho=0.0, model=2)
    assert np.array_equal(kir.I[:, 0], leak.I[:, 0]) and np.array_equal(kir.I[:, 2], leak.I[:, 2])
    ratio = kir.I[:, 1] / leak.I[:, 1]
    assert np.all((ratio > 0.7) & (ratio < 0.95))
    _, _, kirp = _kir_terms(model=2)
    assert np.array_equal(kirp.I[:, 2], leak.I[:, 2])
    assert np.all(kirp.I[:, 0] > leak.I[:, 0]) and np.all(kirp.I[:, 1] < kir.I[:, 1])


# --------------------------------------------------------------------------- Model A evolution
# Sec. "Model A": HH membrane, periodic Na stimulus on all of Gamma, uniform initial values.
@pytest.fixture(scope="module")
def model_a_run():
    case = model_a_evolution_case(nx=16, n_steps=300)
    res = timeloop.run(case)
    phi = np.array([gamma_values(res["asm"].lay, u)[2] for u in res["u"]])
    return case, res, phi


def test_model_a_membrane_potential_is_homogeneous(model_a_run):
    """The membrane potential of Model A is the same all over Gamma (the Model A figure's
    caption): over 300 steps, three action potentials included, the spread over the
    membrane vertices stays below 1 uV."""
    _, _, phi = model_a_run
    assert np.abs(phi - phi.mean(axis=1, keepdims=True)).max() < 1e-6


def test_model_a_first_step_is_forward_euler_of_the_point_model(model_a_run):
    """From uniform data phi_M is uniform on Gamma, and the per-cell capacitive balance
    (I2) makes the first step one forward-Euler step of the point (0-D) HH membrane,
    C_m (phi^1 - phi^0) = -dt I(phi^0, w_1, t_1), with w_1 after the Rush-Larsen
    sub-steps (Sec. "Time discretization") and the stimulus at t_1."""
    case, _, phi = model_a_run
    p = case.params
    psi = p["R"] * p["T"] / p["F"]
    E = psi / np.array(p["z"]) * np.log(np.array(p["conc_e0"]) / np.array(p["conc_i0"]))
    w1 = rush_larsen(np.array([p["gates0"]]), np.array([p["phi_M0"]]), p["phi_rest"], case.dt, p["n_ode"])[0]
    g = np.array(p["g_leak"], dtype=float)
    g[0] += stimulus(p, case.dt) + p["gbar_Na"] * w1[1] ** 3 * w1[2]
    g[1] += p["gbar_K"] * w1[0] ** 4
    expect = p["phi_M0"] - case.dt / p["C_m"] * float(g @ (p["phi_M0"] - E))
    assert abs(phi[1].mean() - expect) < 1e-9, (phi[1].mean(), expect)
    assert abs(phi[1].mean() - phi[0].mean()) > 0.02       # a 23 mV jump: the stimulus acts


def test_model_a_fires_once_per_stimulus(model_a_run):
    """Each stimulus (every tau = 10 ms = 100 steps) triggers one action potential:
    phi_M crosses 0 mV within 1 ms of the onset, is back below -50 mV within 5 ms,
    and stays there until the next onset."""
    case, _, phi = model_a_run
    m = phi.mean(axis=1)
    per = int(round(case.params["stim_tau"] / case.dt))
    for k in range(3):
        on = k * per
        assert m[on + 1:on + 11].max() > 0.0, k
        assert m[on + 50:on + per].max() < -0.050, k


def test_model_a_lu_p0_iterations_stay_low_over_time(model_a_run):
    """Over the 300 steps, action potentials included, GMRES preconditioned by the exact
    LU of P_0 needs 1-6 iterations per step (Sec. "Iterative solver robustness", the
    figure of iterations over 300 steps) under the paper's stopping rule: the
    left-preconditioned residual relative to the preconditioned right-hand side, from
    the initial guess u_{n-1}.  P_0 is that of the first step, as in the paper."""
    case, res, _ = model_a_run
    asm = res["asm"]
    lay = asm.lay
    lu = None
    its = []
    for n in range(1, case.n_steps + 1):
        s = asm.assemble(res["u"][n - 1], res["gates"][n], n * case.dt, case.dt)
        A = s.csr()
        if lu is None:
            P0 = sp.csr_matrix((p0_values(s, lay), s.colidx, s.rowptr), shape=A.shape)
            lu = spla.splu(sp.csc_matrix(P0))
        _, info = gmres(lambda v: lu.solve(A @ v), lu.solve(s.f), x0=res["u"][n - 1], restart=30,
                        rtol=1e-6, maxiter=100)
        its.append(info["its"])
    assert 1 <= min(its) and max(its) <= 6, (min(its), max(its))


def test_model_a_p_n_and_p_0_need_the_same_iterations(model_a_run):
    """Using P_0 for every step instead of the time-dependent P_n has little or no
    impact on GMRES convergence (Sec. "Solution and preconditioning strategy", after
    eq. ``P_prec``): over Model A's 300 steps, LU(P_n) and LU(P_0) differ by at most one
    iteration per step under the paper's stopping rule."""
    case, res, _ = model_a_run
    asm = res["asm"]
    lay = asm.lay
    lu0 = None
    for n in range(1, case.n_steps + 1):
        s = asm.assemble(res["u"][n - 1], res["gates"][n], n * case.dt, case.dt)
        A = s.csr()
        lun = spla.splu(sp.csc_matrix(sp.csr_matrix((p0_values(s, lay), s.colidx, s.rowptr), shape=A.shape)))
        lu0 = lun if lu0 is None else lu0
        its = [gmres(lambda v, lu=lu: lu.solve(A @ v), lu.solve(s.f), x0=res["u"][n - 1], restart=30,
                     rtol=1e-6, maxiter=100)[1]["its"] for lu in (lu0, lun)]
        assert abs(its[0] - its[1]) <= 1, (n, its)


def _duffy_rule(d, n=8):
    """Points (barycentric) and weights (per unit measure) of a collapsed Gauss-Legendre
    rule on the d-simplex, exact for polynomials of degree < 2n - d."""
    g, w = np.polynomial.legendre.leggauss(n)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    pts, wts = [], []
    for idx in itertools.product(range(n), repeat=d):
        u = [g[i] for i in idx]
        wt = np.prod([w[i] for i in idx])
        # x_1 = u_1, x_2 = (1 - u_1) u_2, ...; Jacobian prod (1 - u_k)^(d - k)
        x, rest = [], 1.0
        for k in range(d):
            x.append(rest * u[k])
            wt *= (1.0 - u[k]) ** (d - 1 - k)
            rest *= 1.0 - u[k]
        lam = [1.0 - sum(x)] + x
        pts.append(lam)
        wts.append(wt * math.factorial(d))        # the reference simplex has measure 1/d!
    return np.array(pts), np.array(wts)


def _p2_values_and_lambda_derivs(lam):
    """P2 basis by its closed forms (vertex lambda_a(2 lambda_a - 1), edge 4 lambda_a
    lambda_b) and its derivatives in each lambda_i, at one barycentric point."""
    n = len(lam)
    pairs = list(itertools.combinations(range(n), 2))
    val = [lam[a] * (2 * lam[a] - 1) for a in range(n)] + [4 * lam[a] * lam[b] for a, b in pairs]
    der = np.zeros((n + len(pairs), n))
    for a in range(n):
        der[a, a] = 4 * lam[a] - 1
    for q, (a, b) in enumerate(pairs):
        der[n + q, a] = 4 * lam[b]
        der[n + q, b] = 4 * lam[a]
    return np.array(val), der


@pytest.mark.parametrize("d", [2, 3])
def test_p2_element_integrals_against_quadrature(d):
    """The exact barycentric moments of the P2 mass, stiffness and weighted stiffness
    on one random simplex equal a collapsed Gauss-Legendre quadrature of the basis
    written out in closed form (Sec. "Spatial discretization", p = 2)."""
    from oracle.assemble import simplex_geometry
    from oracle.p2 import reference_tensors
    rng = np.random.default_rng(d)
    x = rng.standard_normal((d + 1, d))
    vol, g = simplex_geometry(x, np.arange(d + 1)[None, :])
    vol, g = vol[0], g[0]
    M, S, W = reference_tensors(d)
    G = g @ g.T
    w = rng.uniform(0.5, 2.0, M.shape[0])
    pts, wts = _duffy_rule(d)
    assert abs(wts.sum() - 1.0) < 1e-13
    Mq = np.zeros_like(M)
    Kq = np.zeros_like(M)
    Wq = np.zeros_like(M)
    for lam, wt in zip(pts, wts):
        val, der = _p2_values_and_lambda_derivs(lam)
        grad = der @ g                                # physical gradients
        Mq += wt * np.outer(val, val)
        Kq += wt * grad @ grad.T
        Wq += wt * (w @ val) * grad @ grad.T
    assert np.abs(M - Mq).max() < 1e-13
    assert np.abs(np.einsum("ij,abij->ab", G, S) - Kq).max() < 1e-11 * np.abs(Kq).max()
    assert np.abs(np.einsum("m,ij,mabij->ab", w, G, W) - Wq).max() < 1e-11 * np.abs(Wq).max()
    assert vol > 0


def test_p2_initial_data_interpolates_linear_fields():
    """Initial data at the edge nodes is the mean of the two vertices' values: exact
    for data linear in the coordinates (the P1 interpolant of the per-vertex data)."""
    case = model_a_case(3, 4)
    lin = 10.0 + 1e6 * case.xyz @ np.array([1.0, 2.0, -3.0])
    case.conc0[:] = lin[None, None, :]
    c2 = p2_case(case)
    expect = 10.0 + 1e6 * c2.xyz @ np.array([1.0, 2.0, -3.0])
    assert np.allclose(c2.conc0[0, 1], expect, rtol=1e-14, atol=1e-12)
    assert c2.xyz.shape[0] == case.n_vert + len(c2.edges)
