"""Method of manufactured solutions for the single-step linearised problem.

The paper verifies its solver with manufactured solutions and states only that the
expected rates were obtained (Sec. "Implementation and numerical verification").
For P1 elements the expected rate of the nodal error in L2 is 2.

Construction.  Smooth exact fields whose normal derivatives vanish on the outer
boundary and on the faces of the Model A cell (X = x / L in {0, 1/4, 3/4, 1}):
products of a quintic with zero slope at those four points.  With zero
normal fluxes, the strong form of eq. ``weak_disc``/``weak_disc2`` for one step is

  c* + dt div J*_k - a_k = dt s_k                    in each region,
  dt sum_k z_k div J*_k  = s_phi                     in each region,
  sgn_r C_r^k phi*_M     = -(g_r^k + sGamma_k)       on Gamma,
  sgn_r (C_m/F) phi*_M   = -(h_r + sGamma_phi)       on Gamma,

with J*_k = -D_k (grad c*_k + z_k/psi a_k grad phi*), a = c^{n-1}.  Sources enter the
oracle as nodal P1 fields (volume: + M s, membrane: - M_Gamma s).  The potential
equations are singular up to the common constant (the pinned mode), so the
interpolated data must be discretely compatible: the extracellular potential source
is shifted by a constant (an O(h^2) change) so that the potential rows of f sum to 0.
"""
import numpy as np
import pytest

from knp_inputs import model_a_case
from oracle.assemble import Assembler, initial_gates
from oracle.p2 import p2_case
from oracle.mesh import PHI
from oracle.solve import lu_solve


class FlatPoly:
    """f(x) = amp * prod_d p(x_d / L) over the axes with k_d != 0, where p is the
    quintic with p(0) = 0, max |p| = 1 on [0, 1] and p'(X) proportional to
    X (X - 1/4)(X - 3/4)(X - 1): zero slope on the outer boundary and on the faces of
    the Model A cell.  Value, gradient and Laplacian in closed form."""

    def __init__(self, amp, ks, L):
        P = np.polynomial.polynomial
        dp = P.polyfromroots([0.0, 0.25, 0.75, 1.0])
        p = P.polyint(dp)
        s = np.abs(P.polyval(np.linspace(0.0, 1.0, 1001), p)).max()
        self.c = (p / s, dp / s, P.polyder(dp) / s)
        self.amp, self.ks, self.L = amp, ks, L

    def _f(self, d, x, der):
        if self.ks[d] == 0:
            return np.ones_like(x) if der == 0 else np.zeros_like(x)
        return np.polynomial.polynomial.polyval(x / self.L, self.c[der]) / self.L ** der

    def _prod(self, x, ders):
        t = self.amp * np.ones(len(x))
        for d in range(x.shape[1]):
            t = t * self._f(d, x[:, d], ders[d])
        return t

    def val(self, x):
        return self._prod(x, [0] * x.shape[1])

    def grad(self, x):
        n = x.shape[1]
        return np.stack([self._prod(x, [1 if e == d else 0 for e in range(n)])
                         for d in range(n)], axis=1)

    def lap(self, x):
        n = x.shape[1]
        return sum(self._prod(x, [2 if e == d else 0 for e in range(n)]) for d in range(n))


def _solve_mms(dim, nx, dt=1e-4, degree=1):
    case = model_a_case(dim, nx, "leak", dt, 1)
    if degree == 2:
        case = p2_case(case)
    p = case.params
    L = 1e-6
    z = np.array(p["z"])
    D = np.array(p["D"])
    F, Cm = p["F"], p["C_m"]
    psi = p["R"] * p["T"] / F
    ks = lambda *k: tuple(k[:dim])
    base = (p["conc_i0"], p["conc_e0"])
    prev = [[FlatPoly(0.1 * base[r][k], ks(4, 4, 4), L) for k in range(2)] for r in (0, 1)]
    dcon = [[FlatPoly(0.05 * base[r][k], ks(4, 4, 0), L) for k in range(2)] for r in (0, 1)]
    phi = [FlatPoly(0.01, ks(4, 0, 4), L), FlatPoly(0.005, ks(0, 4, 4), L)]
    phi_const = [p["phi_M0"], 0.0]             # p(0) = 0: phi*_e vanishes at the pinned corner

    asm = Assembler(case)
    lay = asm.lay
    N = lay.N
    u_prev = np.zeros(N)
    u_star = np.zeros(N)
    vol = np.zeros(N)
    for r in (0, 1):
        V = lay.verts[r]
        x = case.xyz[V]
        idx = np.arange(len(V))
        a_val, a_grad, c_val, c_lap = [], [], [], []
        for k in range(3):
            if k < 2:
                av = base[r][k] + prev[r][k].val(x)
                ag = prev[r][k].grad(x)
                cv = av + dcon[r][k].val(x)
                cl = prev[r][k].lap(x) + dcon[r][k].lap(x)
            else:                               # Cl = Na + K keeps both states neutral
                av = a_val[0] + a_val[1]
                ag = a_grad[0] + a_grad[1]
                cv = c_val[0] + c_val[1]
                cl = c_lap[0] + c_lap[1]
            a_val.append(av), a_grad.append(ag), c_val.append(cv), c_lap.append(cl)
        ph_val = phi_const[r] + phi[r].val(x)
        ph_grad = phi[r].grad(x)
        ph_lap = phi[r].lap(x)
        divJ_sum = 0.0
        for k in range(3):
            drift = (a_grad[k] * ph_grad).sum(axis=1) + a_val[k] * ph_lap
            divJ = -D[k] * (c_lap[k] + z[k] / psi * drift)
            u_prev[lay.dof(r, k, idx)] = a_val[k]
            u_star[lay.dof(r, k, idx)] = c_val[k]
            vol[lay.dof(r, k, idx)] = c_val[k] - a_val[k] + dt * divJ
            divJ_sum = divJ_sum + z[k] * divJ
        u_prev[lay.dof(r, PHI, idx)] = ph_val
        u_star[lay.dof(r, PHI, idx)] = ph_val
        vol[lay.dof(r, PHI, idx)] = dt * divJ_sum

    # membrane sources from the step's own membrane terms (data of the scheme)
    s0 = asm.assemble(u_prev, initial_gates(case, lay), dt, dt)
    mem = s0.mem
    gam_src = np.zeros((2, 4, lay.n_vert))
    phiM_star = (u_star[lay.dof(0, PHI, lay.loc[0, lay.gamma])]
                 - u_star[lay.dof(1, PHI, lay.loc[1, lay.gamma])])
    for r, sgn in ((0, 1.0), (1, -1.0)):
        for k in range(3):
            gam_src[r, k, lay.gamma] = -sgn * mem.C[r, :, k] * phiM_star - mem.g[r, :, k]
        gam_src[r, PHI, lay.gamma] = -sgn * (Cm / F) * phiM_star - mem.h[r]
    s = asm.assemble(u_prev, initial_gates(case, lay), dt, dt, vol_source=vol,
                     gamma_source=gam_src, pin=False)
    phi_rows = np.r_[lay.dof(0, PHI, np.arange(lay.N_r[0])), lay.dof(1, PHI, np.arange(lay.N_r[1]))]
    e_idx = lay.dof(1, PHI, np.arange(lay.N_r[1]))
    ones_e = np.zeros(N)
    ones_e[e_idx] = 1.0
    unit = (asm.assemble(u_prev, initial_gates(case, lay), dt, dt, vol_source=ones_e,
                         pin=False).f[phi_rows].sum()
            - asm.assemble(u_prev, initial_gates(case, lay), dt, dt, pin=False).f[phi_rows].sum())
    vol[e_idx] -= s.f[phi_rows].sum() / unit
    s = asm.assemble(u_prev, initial_gates(case, lay), dt, dt, vol_source=vol,
                     gamma_source=gam_src)
    u = lu_solve(s.csr(), s.f)
    return case, lay, u, u_star


def _l2(case, lay, r, e):
    from oracle.assemble import bulk_coo
    import scipy.sparse as sp
    rr, cc, vv = bulk_coo(case, lay, r, kind="mass")
    M = sp.coo_matrix((vv, (rr, cc)), shape=(lay.N_r[r],) * 2).tocsr()
    return np.sqrt(e @ (M @ e))


@pytest.mark.parametrize("dim,sizes", [(2, (16, 32, 64)), (3, (8, 12, 16))])
def test_mms_second_order(dim, sizes):
    errs = []
    for nx in sizes:
        case, lay, u, us = _solve_mms(dim, nx)
        row = []
        for r in (0, 1):
            idx = np.arange(lay.N_r[r])
            for f in range(4):
                d = lay.dof(r, f, idx)
                row.append(_l2(case, lay, r, u[d] - us[d]))
        errs.append(np.array(row))
    rates = np.log2(errs[-2] / errs[-1]) / np.log2(sizes[-1] / sizes[-2])
    assert np.all(rates > 1.8), rates
    assert np.all(rates < 2.6), rates


def test_mms_p2_third_order_2d():
    """Quadratic elements (p = 2, Sec. "Spatial discretization"): the nodal error of
    every field converges at least at third order in L2 (2D, N_x = 16 -> 32)."""
    errs = []
    for nx in (16, 32):
        case, lay, u, us = _solve_mms(2, nx, degree=2)
        row = []
        for r in (0, 1):
            idx = np.arange(lay.N_r[r])
            for f in range(4):
                d = lay.dof(r, f, idx)
                row.append(_l2(case, lay, r, u[d] - us[d]))
        errs.append(np.array(row))
    rates = np.log2(errs[0] / errs[1])
    assert np.all(rates > 2.7), rates
