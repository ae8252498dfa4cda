"""Pins of the oracle's membrane integrals and of the weighting of alpha_r^k.

The invariants I2/I3 and the manufactured solutions use the oracle's own membrane
mass matrix on both sides, so a wrong scale of the membrane measure cancels in them;
the same holds for a wrong weighting of the capacitive split alpha_r^k.  These tests
tie both to values the geometry and the paper's definitions fix on their own:

* the membrane mass matrices M_{r,Gamma}, M_{rq,Gamma} and the coefficient-weighted ones
  (Sec. "Algebraic structure and matrix assembly") are integrals over Gamma, so
  1^T M_Gamma 1 is the membrane's measure and u^T M_Gamma[w] v the integral of w u v,
  which for box cells is a sum over their faces, integrated here by tensor
  Gauss-Legendre rules (exact for the polynomial degrees involved);
* alpha_r^k = D_k z_k^2 c_k / sum_l D_l z_l^2 c_l (Sec. "Interface conditions", next to
  the capacitive current): with this weighting the capacitive current splits among the
  ions exactly as the bulk drift does (tilde-tau_k z_k c_k), so with uniform
  concentrations and no channel currents one step moves the potentials and leaves
  every concentration where it was.  Any other weighting makes the ion rows disagree
  with the potential rows and moves the concentrations.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from knp_inputs import lattice_case, model_a_case
from oracle.assemble import Assembler, gamma_coo, initial_gates, initial_state
from oracle.mesh import PHI, build_layout
from oracle.solve import lu_solve


def _gamma_matrix(case, lay, weight=None):
    gr, gc, gv = gamma_coo(case, lay, weight)
    return sp.coo_matrix((gv, (gr, gc)), shape=(lay.n_vert,) * 2).tocsr()


def _box_faces(case):
    """Faces of every cell box in metres: (fixed axis, its coordinate, lo, hi) with lo/hi
    the box's extent along the other axes."""
    h = np.array(case.length_um, dtype=np.float64) / np.array(case.shape) * 1e-6
    faces = []
    for lo_i, hi_i in case.cell_box:
        lo = lo_i * h
        hi = hi_i * h
        for a in range(case.dim):
            others = [b for b in range(case.dim) if b != a]
            for xa in (lo[a], hi[a]):
                faces.append((a, xa, lo[others], hi[others], others))
    return faces


def _gauss_face_integral(case, fn, npts=3):
    """Integral over all membrane faces of fn(points [n, dim]) by tensor Gauss-Legendre."""
    t, w = np.polynomial.legendre.leggauss(npts)
    total = 0.0
    for a, xa, lo, hi, others in _box_faces(case):
        m = len(others)
        pts, wts = [], []
        for idx in itertools.product(range(npts), repeat=m):
            p = np.zeros(case.dim)
            p[a] = xa
            wt = 1.0
            for j, b in enumerate(others):
                half = 0.5 * (hi[j] - lo[j])
                p[b] = lo[j] + half * (1.0 + t[idx[j]])
                wt *= half * w[idx[j]]
            pts.append(p)
            wts.append(wt)
        total += np.dot(np.array(wts), fn(np.array(pts)))
    return total


def _cases():
    return {
        "modelA_2d": model_a_case(2, 8),
        "modelA_3d": model_a_case(3, 8),
        "lattice_2d": lattice_case(cells=(3, 2), pitch_um=(1.0, 1.0), per_pitch=10, n_hh=0, cfg_id=7),
        "lattice_3d": lattice_case(cells=(2, 2, 2), pitch_um=(1.0, 1.0, 1.0), per_pitch=8, n_hh=0, cfg_id=4),
    }


@pytest.fixture(scope="module")
def cases():
    return {k: (c, build_layout(c)) for k, c in _cases().items()}


def test_model_a_membrane_measure_closed_form(cases):
    """Model A's cell is [0.25, 0.75]^d um: its boundary has length 4 x 0.5 um = 2.0e-6 m
    in 2D and area 6 x 0.25 um^2 = 1.5e-12 m^2 in 3D (Sec. "Model A")."""
    for key, exact in (("modelA_2d", 2.0e-6), ("modelA_3d", 1.5e-12)):
        case, lay = cases[key]
        MG = _gamma_matrix(case, lay)
        assert abs(MG.sum() - exact) <= 1e-14 * exact, key


@pytest.mark.parametrize("key", ["lattice_2d", "lattice_3d"])
def test_lattice_membrane_measure_from_the_cell_boxes(cases, key):
    """Sum over the cells of each box's perimeter (2D) or surface (3D), from its grid
    extent times the grid spacing."""
    case, lay = cases[key]
    h = np.array(case.length_um) / np.array(case.shape) * 1e-6
    side = (case.cell_box[:, 1] - case.cell_box[:, 0]) * h[None, :]
    if case.dim == 2:
        exact = np.sum(2.0 * (side[:, 0] + side[:, 1]))
    else:
        exact = np.sum(2.0 * (side[:, 0] * side[:, 1] + side[:, 1] * side[:, 2] + side[:, 0] * side[:, 2]))
    MG = _gamma_matrix(case, lay)
    assert abs(MG.sum() - exact) <= 1e-13 * exact


@pytest.mark.parametrize("key", ["modelA_2d", "modelA_3d", "lattice_2d", "lattice_3d"])
def test_membrane_mass_integrates_products_of_linear_fields(cases, key):
    """For linear w, u, v: 1^T M_Gamma[w] 1 = int_Gamma w, u^T M_Gamma v = int_Gamma u v
    and u^T M_Gamma[w] v = int_Gamma w u v (the P1 interpolants are exact)."""
    case, lay = cases[key]
    rng = np.random.Generator(np.random.PCG64(11))
    L = np.array(case.length_um) * 1e-6
    coef = [rng.uniform(0.5, 2.0, size=case.dim + 1) for _ in range(3)]

    def lin(c):
        return lambda x: c[0] + (x / L[None, :]) @ c[1:]

    fw, fu, fv = (lin(c) for c in coef)
    w, u, v = fw(case.xyz), fu(case.xyz), fv(case.xyz)
    MG = _gamma_matrix(case, lay)
    MGw = _gamma_matrix(case, lay, w)
    one = np.ones(lay.n_vert)
    checks = [
        (one @ (MGw @ one), _gauss_face_integral(case, fw)),
        (u @ (MG @ v), _gauss_face_integral(case, lambda x: fu(x) * fv(x))),
        (u @ (MGw @ v), _gauss_face_integral(case, lambda x: fw(x) * fu(x) * fv(x))),
    ]
    for got, exact in checks:
        assert abs(got - exact) <= 1e-13 * abs(exact)


def _capacitive_step(case):
    """One oracle step from uniform table concentrations, no channel currents and a
    membrane potential that varies along Gamma."""
    p = dict(case.params)
    p["g_leak"] = [0.0, 0.0, 0.0]
    case.params = p
    case.cell_model[:] = 0
    case.cell_stim[:] = 0
    for r, base in enumerate((p["conc_i0"], p["conc_e0"])):
        for k in range(3):
            case.conc0[r, k, :] = base[k]
    asm = Assembler(case)
    lay = asm.lay
    u0 = initial_state(case, lay)
    # phi_i^{n-1} varies by +-10 mV over the domain; phi_e^{n-1} by +-2 mV
    L = np.array(case.length_um) * 1e-6
    for r, amp in ((0, 0.010), (1, 0.002)):
        x = case.xyz[lay.verts[r]] / L[None, :]
        wave = np.sin(2.0 * np.pi * x[:, 0]) * np.cos(np.pi * x[:, -1])
        u0[lay.dof(r, PHI, np.arange(lay.N_r[r]))] += amp * wave
    s = asm.assemble(u0, initial_gates(case, lay), case.dt, case.dt)
    u1 = lu_solve(s.csr(), s.f)
    return lay, u0, u1


@pytest.mark.parametrize("make", [
    lambda: model_a_case(2, 16, noise=0.0),
    lambda: model_a_case(3, 8, noise=0.0, dt=5e-5),
    lambda: lattice_case(cells=(2, 2, 2), pitch_um=(1.0, 1.0, 1.0), per_pitch=8, n_hh=0, cfg_id=4),
], ids=["modelA_2d", "modelA_3d", "lattice_3d"])
def test_capacitive_split_follows_the_drift_split(make):
    """alpha_r^k weights D_k z_k^2 c_k: at uniform concentrations without channel currents
    the concentrations stay put (to rounding) while the potentials move by millivolts.

    Rounding leaves ~1e-12 relative away from the pinned vertex and up to ~1e-10 at it
    (its potential equation is only implied by the others); dropping D_k from the
    weights moves every ion by 2e-8 to 6e-6 relative on these meshes."""
    lay, u0, u1 = _capacitive_step(make())
    dphi = 0.0
    for r in (0, 1):
        idx = np.arange(lay.N_r[r])
        for k in range(3):
            c0 = u0[lay.dof(r, k, idx)]
            c1 = u1[lay.dof(r, k, idx)]
            assert np.abs(c1 - c0).max() <= 1e-9 * np.abs(c0).max(), (r, k)
        dphi = max(dphi, np.abs(u1[lay.dof(r, PHI, idx)] - u0[lay.dof(r, PHI, idx)]).max())
    assert dphi > 1e-4      # the potentials do move (by ~mV)
