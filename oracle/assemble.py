"""Exact P1 assembly of the IMEX-linearised KNP-EMI system.  Test infrastructure.

Sources followed (paper sections / equations):
  * bulk matrices M_r, A_r, A_r^{k,n}        Sec. "Algebraic structure ...", first display
  * membrane matrices M_{r,Gamma}, M_{rq,Gamma}  same section, second display
  * region block operator and coupling blocks  displays for \\mathcal{A}_r^n, \\mathcal{B}_{rq}^n
  * global system and right-hand side         eq. ``lin_sys`` and the f_r^{k,n}, f_r^{phi,n} display
  * tau, tilde-tau                            definition before the \\mathcal{A}_r^n display
  * alpha, C, g, h                            eq. ``weak_disc``/``weak_disc2`` and their short-hands
  * membrane currents                         eq. ``HH_ionic_model`` and the passive-leak reading
  * Kir-Na/K currents, f_Kir, j_pump          Sec. "Passive dynamics: Kir--Na/K"
  * pinned potential                          Remark ``rem:nullspace``

Readings where the text is silent or garbled (each is listed in the design notes):
  * h_r = sgn_r (dt I_ch - C_m phi_M^{n-1}) / F.  The printed "+" contradicts the
    weak form the short-hand is derived from; with "-" it equals sum_k z_k g_r^k.
  * Nonlinear membrane coefficients (alpha, C, I, g, h) are evaluated at the
    membrane vertices and treated as P1 fields on Gamma; every integral is exact.
  * alpha_r uses r-side concentrations; E_k uses both copies of the vertex;
    phi_M = phi_i - phi_e of the vertex pair.
  * Passive leak membrane: I_k = theta * g_leak^k (phi_M - E_k) for every ion.
  * Kir-Na/K: [K+]_e^0 and E_K^0 are the table's initial values ([K+]_e^0 = 4 mM,
    E_K^0 = psi/z_K ln([K+]_e^0/[K+]_i^0)), constants of the model; theta scales the
    leak conductances (the Kir K current included) and not the pump.  A = 1 + e^0.433
    as printed.
  * The pinned DOF is phi_e at one vertex: its row and column are zeroed except
    the diagonal, and its right-hand side is 0.

Exact P1 integrals on a simplex of dimension m with measure |T| and barycentric
coordinates lambda:  int prod lambda_a^{p_a} = m! |T| prod p_a! / (m + sum p_a)!.
"""
from __future__ import annotations

from collections import Counter
from dataclasses import dataclass
from math import factorial

import numpy as np
import scipy.sparse as sp

from .mesh import Layout, PHI, embed, structural_pattern


# --------------------------------------------------------------------------- geometry
def simplex_geometry(xyz, elem):
    """Volumes |T| and barycentric gradients grad(lambda_a) [n, d+1, d]."""
    x = xyz[elem]                               # [n, d+1, d]
    J = np.transpose(x[:, 1:, :] - x[:, :1, :], (0, 2, 1))   # columns x_a - x_0
    d = J.shape[1]
    vol = np.abs(np.linalg.det(J)) / factorial(d)
    Jinv = np.linalg.inv(J)                     # rows = grad(lambda_1..d)
    g = np.empty((len(elem), d + 1, d))
    g[:, 1:, :] = Jinv
    g[:, 0, :] = -Jinv.sum(axis=1)
    return vol, g


def facet_measure(xyz, facets):
    x = xyz[facets]
    if facets.shape[1] == 2:
        return np.linalg.norm(x[:, 1] - x[:, 0], axis=1)
    return 0.5 * np.linalg.norm(np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), axis=1)


def _moment(m, idx):
    """int over an m-simplex of prod lambda_idx, divided by |F|."""
    mult = Counter(idx)
    num = factorial(m)
    for c in mult.values():
        num *= factorial(c)
    return num / factorial(m + len(idx))


# --------------------------------------------------------------------------- bulk
def bulk_coo(case, lay: Layout, r: int, weight=None, kind="stiff"):
    """COO triplets (rows, cols, vals) of M_r ("mass"), A_r ("stiff") or the
    weighted stiffness int weight grad(phi_j).grad(phi_l) with a weight in the same
    space given by region-local nodal values (P1: exact as the mean over the element
    times A_T; P2: exact barycentric moments)."""
    sel = (case.tag >= 1) if r == 0 else (case.tag == 0)
    el_glob = case.elem[sel].astype(np.int64)
    el = lay.loc[r][el_glob]
    if getattr(case, "degree", 1) == 2:
        return _bulk_coo_p2(case, el_glob, el, weight, kind)
    vol, g = simplex_geometry(case.xyz, el_glob)
    d1 = el.shape[1]
    rows, cols, vals = [], [], []
    for a in range(d1):
        for b in range(d1):
            if kind == "mass":
                v = vol * _moment(d1 - 1, (a, b))
            else:
                v = vol * np.einsum("ij,ij->i", g[:, a, :], g[:, b, :])
                if weight is not None:
                    v = v * weight[el].mean(axis=1)
            rows.append(el[:, a])
            cols.append(el[:, b])
            vals.append(v)
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def _bulk_coo_p2(case, el_glob, el, weight, kind):
    from .p2 import reference_tensors
    d = case.dim
    M, S, W = reference_tensors(d)
    vol, g = simplex_geometry(case.xyz, el_glob[:, :d + 1])
    G = np.einsum("eid,ejd->eij", g, g)              # grad(lambda_i) . grad(lambda_j)
    if kind == "mass":
        local = vol[:, None, None] * M[None]
    elif weight is None:
        local = vol[:, None, None] * np.einsum("eij,abij->eab", G, S)
    else:
        local = vol[:, None, None] * np.einsum("em,eij,mabij->eab", weight[el], G, W)
    n = el.shape[1]
    rows = np.repeat(el, n, axis=1).ravel()
    cols = np.tile(el, (1, n)).ravel()
    return rows, cols, local.reshape(len(el), n * n).ravel()


def gamma_coo(case, lay: Layout, weight=None):
    """COO over global node ids of int_Gamma w phi_a phi_b (w = 1 if None; else a
    membrane field in the same space given by nodal values indexed by global id)."""
    f = lay.facets
    if getattr(case, "degree", 1) == 2:
        from .p2 import facet_tensors
        m = case.dim - 1
        meas = facet_measure(case.xyz, f[:, :m + 1])
        F2, F3 = facet_tensors(m)
        n = f.shape[1]
        if weight is None:
            local = meas[:, None, None] * F2[None]
        else:
            local = meas[:, None, None] * np.einsum("ec,abc->eab", weight[f], F3)
        return np.repeat(f, n, axis=1).ravel(), np.tile(f, (1, n)).ravel(), local.reshape(len(f), n * n).ravel()
    meas = facet_measure(case.xyz, f)
    m = f.shape[1] - 1
    rows, cols, vals = [], [], []
    for a in range(m + 1):
        for b in range(m + 1):
            if weight is None:
                v = meas * _moment(m, (a, b))
            else:
                v = np.zeros(len(f))
                for c in range(m + 1):
                    v = v + weight[f[:, c]] * meas * _moment(m, (a, b, c))
            rows.append(f[:, a])
            cols.append(f[:, b])
            vals.append(v)
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


# --------------------------------------------------------------------------- membrane
def hh_rates(phi_M, phi_rest):
    """Hodgkin-Huxley 1952 rates (alpha, beta) in 1/s for gates (n, m, h).

    V = 1000 (phi_M - phi_rest) in mV, classical formulas in 1/ms, times 1000.
    The 0/0 points of alpha_n (V = 10) and alpha_m (V = 25) use their limits.
    """
    V = 1000.0 * (np.asarray(phi_M, dtype=np.float64) - phi_rest)

    def ratio(x):       # x / (exp(x/10) - 1), limit 10 at x = 0
        x = np.asarray(x, dtype=np.float64)
        out = np.full_like(x, 10.0)
        nz = x != 0.0
        out[nz] = x[nz] / np.expm1(x[nz] / 10.0)
        return out

    a_n = 0.01 * ratio(10.0 - V)
    b_n = 0.125 * np.exp(-V / 80.0)
    a_m = 0.1 * ratio(25.0 - V)
    b_m = 4.0 * np.exp(-V / 18.0)
    a_h = 0.07 * np.exp(-V / 20.0)
    b_h = 1.0 / (np.exp((30.0 - V) / 10.0) + 1.0)
    alpha = np.stack([a_n, a_m, a_h], axis=-1) * 1000.0
    beta = np.stack([b_n, b_m, b_h], axis=-1) * 1000.0
    return alpha, beta


def rush_larsen(w, phi_M, phi_rest, dt, n_sub):
    """n_sub Rush-Larsen steps of size dt/n_sub of eq. ``gating`` with phi_M frozen."""
    alpha, beta = hh_rates(phi_M, phi_rest)
    tau_inv = alpha + beta
    w_inf = alpha / tau_inv
    decay = np.exp(-tau_inv * (dt / n_sub))
    w = np.array(w, dtype=np.float64, copy=True)
    for _ in range(n_sub):
        w = w_inf + (w - w_inf) * decay
    return w


def kir_factor(K_e, dphi_K, phi_M, E_K0, K_e0):
    """Inward-rectifier factor f_Kir (Sec. "Passive dynamics: Kir--Na/K"): two
    Boltzmann factors, in dphi_K = phi_M - E_K and in phi_M, normalised by their
    values at the initial K reversal potential, times sqrt([K+]_e/[K+]_e^0)."""
    A = 1.0 + np.exp(0.433)
    B = 1.0 + np.exp(-(0.1186 + E_K0) / 0.0441)
    C = 1.0 + np.exp((dphi_K + 0.0185) / 0.0425)
    D = 1.0 + np.exp(-(0.1186 + phi_M) / 0.0441)
    return A * B / (C * D) * np.sqrt(K_e / K_e0)


def pump_flux(Na_i, K_e, rho, P_Na, P_K):
    """Na/K pump flux density j_pump (same section, eq. ``pump``): saturating in the
    ICS Na+ (exponent 1.5) and in the ECS K+ concentration."""
    na = Na_i ** 1.5
    return rho * na / (na + P_Na ** 1.5) * K_e / (K_e + P_K)


def stimulus(p, t):
    """Model A periodic Na stimulus g_stim(t) = gbar exp(-(t mod tau)/a)."""
    return p["g_stim_bar"] * np.exp(-np.fmod(t, p["stim_tau"]) / p["stim_a"])


@dataclass
class MembraneTerms:
    """Nodal membrane quantities at the Gamma vertices (lay.gamma order)."""
    E: np.ndarray        # [n_g, 3]
    I: np.ndarray        # [n_g, 3]  channel currents I_ch^k
    alpha: np.ndarray    # [2, n_g, 3]
    C: np.ndarray        # [2, n_g, 3]
    g: np.ndarray        # [2, n_g, 3]
    h: np.ndarray        # [2, n_g]
    phi_M: np.ndarray    # [n_g]


def gamma_values(lay: Layout, u: np.ndarray):
    """(c_i [n_g,3], c_e [n_g,3], phi_M [n_g]) at the membrane vertices."""
    gi = lay.loc[0, lay.gamma]
    ge = lay.loc[1, lay.gamma]
    ci = np.stack([u[lay.dof(0, k, gi)] for k in range(3)], axis=1)
    ce = np.stack([u[lay.dof(1, k, ge)] for k in range(3)], axis=1)
    phiM = u[lay.dof(0, PHI, gi)] - u[lay.dof(1, PHI, ge)]
    return ci, ce, phiM


def membrane_terms(case, lay: Layout, u_prev, gates, t, dt, theta=None) -> MembraneTerms:
    """alpha, C, I_ch, g, h at every Gamma vertex from u_{n-1} and w_n."""
    p = case.params
    z = np.array(p["z"])
    D = np.array(p["D"])
    F, Cm = p["F"], p["C_m"]
    psi = p["R"] * p["T"] / F
    theta = case.theta if theta is None else np.asarray(theta)
    ci, ce, phiM = gamma_values(lay, u_prev)
    cell = lay.vert_cell[lay.gamma] - 1
    model = case.cell_model[cell]
    stim = case.cell_stim[cell]
    th = theta[cell]

    E = psi / z[None, :] * np.log(ce / ci)
    gcond = th[:, None] * np.array(p["g_leak"])[None, :]
    gcond[:, 0] += np.where(stim == 1, stimulus(p, t), 0.0)
    hh = model == 1
    if np.any(hh):
        w = np.asarray(gates)[hh]
        n_, m_, h_ = w[:, 0], w[:, 1], w[:, 2]
        gcond[hh, 0] += p["gbar_Na"] * m_ ** 3 * h_
        gcond[hh, 1] += p["gbar_K"] * n_ ** 4
    I = gcond * (phiM[:, None] - E)
    kir = model == 2
    if np.any(kir):
        K_e0, K_i0 = p["conc_e0"][1], p["conc_i0"][1]
        E_K0 = psi / z[1] * np.log(K_e0 / K_i0)
        fk = kir_factor(ce[kir, 1], phiM[kir] - E[kir, 1], phiM[kir], E_K0, K_e0)
        jp = pump_flux(ci[kir, 0], ce[kir, 1], p["rho_pump"], p["P_Na"], p["P_K"])
        I = I.astype(np.result_type(I, fk, jp))
        I[kir, 0] += 3.0 * F * z[0] * jp
        I[kir, 1] = I[kir, 1] * fk - 2.0 * F * z[1] * jp

    dtype = np.result_type(ci, ce, phiM, I)          # complex under complex-step perturbation
    alpha = np.empty((2,) + ci.shape, dtype=dtype)
    C = np.empty_like(alpha)
    g = np.empty_like(alpha)
    h = np.empty((2, len(phiM)), dtype=dtype)
    for r, (c, sgn) in enumerate(((ci, 1.0), (ce, -1.0))):
        wgt = D[None, :] * z[None, :] ** 2 * c
        alpha[r] = wgt / wgt.sum(axis=1, keepdims=True)
        C[r] = alpha[r] * Cm / (F * z[None, :])
        g[r] = sgn * (dt * I - alpha[r] * Cm * phiM[:, None]) / (F * z[None, :])
        h[r] = sgn * (dt * I.sum(axis=1) - Cm * phiM) / F
    return MembraneTerms(E, I, alpha, C, g, h, phiM)


# --------------------------------------------------------------------------- system
@dataclass
class System:
    rowptr: np.ndarray
    colidx: np.ndarray
    vals: np.ndarray
    f: np.ndarray
    mem: MembraneTerms

    def csr(self):
        N = len(self.rowptr) - 1
        return sp.csr_matrix((self.vals, self.colidx, self.rowptr), shape=(N, N))


class Assembler:
    """Holds the mesh layout and pattern; assembles A_{n-1}, f_n for one step."""

    def __init__(self, case):
        from .mesh import build_layout
        self.case = case
        self.lay = build_layout(case)
        self.rowptr, self.colidx = structural_pattern(case, self.lay)

    def _sp(self, coo, shape):
        r, c, v = coo
        A = sp.coo_matrix((v, (r, c)), shape=shape).tocsr()
        A.sum_duplicates()
        return A

    def assemble(self, u_prev, gates, t, dt, theta=None, pin=True,
                 vol_source=None, gamma_source=None) -> System:
        """A_{n-1} and f_n of eq. ``lin_sys``.

        vol_source: optional nodal P1 sources s_r^f (array [N]) added as M_r s to
        each field row; gamma_source: optional nodal membrane sources [2, 4, n_vert]
        added as -M_{r,Gamma} s.  Both are zero for the paper's workloads and exist
        for manufactured-solution checks.
        """
        case, lay = self.case, self.lay
        p = case.params
        z = np.array(p["z"])
        D = np.array(p["D"])
        F, Cm = p["F"], p["C_m"]
        psi = p["R"] * p["T"] / F
        tau = dt * D
        ttau = tau * z / psi
        N = lay.N
        Nr = lay.N_r
        mem = membrane_terms(case, lay, u_prev, gates, t, dt, theta)

        blocks = {}            # (row block, col block) -> csr, block = (region, field)

        def put(rb, cb, M):
            key = (rb, cb)
            blocks[key] = blocks[key] + M if key in blocks else M

        dtype = np.result_type(u_prev, mem.C)
        nodal = np.zeros(lay.n_vert, dtype=dtype)
        f = np.zeros(N, dtype=dtype)

        def put_f(r, fld, val):
            s0 = lay.dof(r, fld, 0)
            f[s0:s0 + Nr[r]] = val

        for r in (0, 1):
            q = 1 - r
            shp = (Nr[r], Nr[r])
            M = self._sp(bulk_coo(case, lay, r, kind="mass"), shp)
            A = self._sp(bulk_coo(case, lay, r, kind="stiff"), shp)
            Ak = []
            for k in range(3):
                ck = u_prev[lay.dof(r, k, np.arange(Nr[r]))]
                Ak.append(self._sp(bulk_coo(case, lay, r, weight=ck, kind="stiff"), shp))

            def gam(weight, cols_region):
                gr, gc, gv = gamma_coo(case, lay, weight)
                return self._sp((lay.loc[r][gr], lay.loc[cols_region][gc], gv),
                                (Nr[r], Nr[cols_region]))

            MG_rr = gam(None, r)
            MG_rq = gam(None, q)
            for k in range(3):
                nodal[:] = 0.0
                nodal[lay.gamma] = mem.C[r, :, k]
                CMG_rr = gam(nodal, r)
                CMG_rq = gam(nodal, q)
                put((r, k), (r, k), M + tau[k] * A)
                put((r, k), (r, PHI), CMG_rr + ttau[k] * Ak[k])
                put((r, k), (q, PHI), -CMG_rq)
                put((r, PHI), (r, k), z[k] * tau[k] * A)
            put((r, PHI), (r, PHI), (Cm / F) * MG_rr + sum(z[k] * ttau[k] * Ak[k] for k in range(3)))
            put((r, PHI), (q, PHI), -(Cm / F) * MG_rq)

            # right-hand side
            for k in range(3):
                ck = u_prev[lay.dof(r, k, np.arange(Nr[r]))]
                gk = np.zeros(Nr[r], dtype=dtype)
                gk[lay.loc[r, lay.gamma]] = mem.g[r, :, k]
                fk = M @ ck - MG_rr @ gk
                if vol_source is not None:
                    fk = fk + M @ vol_source[lay.dof(r, k, np.arange(Nr[r]))]
                if gamma_source is not None:
                    fk = fk - MG_rr @ gamma_source[r, k, lay.verts[r]]
                put_f(r, k, fk)
            hr = np.zeros(Nr[r], dtype=dtype)
            hr[lay.loc[r, lay.gamma]] = mem.h[r]
            fphi = -(MG_rr @ hr)
            if vol_source is not None:
                fphi = fphi + M @ vol_source[lay.dof(r, PHI, np.arange(Nr[r]))]
            if gamma_source is not None:
                fphi = fphi - MG_rr @ gamma_source[r, PHI, lay.verts[r]]
            put_f(r, PHI, fphi)

        order = [(r, f) for r in (0, 1) for f in range(4)]
        grid = [[blocks.get((rb, cb)) for cb in order] for rb in order]
        for i, rb in enumerate(order):          # bmat needs a shape per block row/col
            if all(x is None for x in grid[i]):
                raise AssertionError("empty block row")
        Aglob = sp.bmat(grid, format="csr")
        vals = embed(Aglob, self.rowptr, self.colidx)
        if pin:
            vals, f = pin_system(self.rowptr, self.colidx, vals, f, lay.pin_dof)
        return System(self.rowptr, self.colidx, vals, f, mem)



def pin_system(rowptr, colidx, vals, f, pin):
    """Point Dirichlet phi_e(x_e) = 0: zero row and column, keep the diagonal."""
    vals = vals.copy()
    f = f.copy()
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    in_row = rows == pin
    in_col = colidx == pin
    diag = in_row & in_col
    vals[(in_row | in_col) & ~diag] = 0.0
    f[pin] = 0.0
    return vals, f


def initial_state(case, lay: Layout):
    """u_0 from the per-vertex initial concentrations and (phi_i^0, phi_e^0)."""
    u = np.zeros(lay.N)
    for r in (0, 1):
        V = lay.verts[r]
        for k in range(3):
            u[lay.dof(r, k, np.arange(len(V)))] = case.conc0[r, k, V]
        u[lay.dof(r, PHI, np.arange(len(V)))] = case.phi0[r]
    return u


def initial_gates(case, lay: Layout):
    return np.tile(np.array(case.params["gates0"], dtype=np.float64), (len(lay.gamma), 1))


def p0_values(sys_: System, lay: Layout):
    """Values of P_0: the entries of A whose row and column lie in the same
    (region, field) block; other entries set to zero (eq. ``P_prec``)."""
    N = lay.N
    Ni, Ne = lay.N_r
    bounds = np.array([0, Ni, 2 * Ni, 3 * Ni, 4 * Ni, 4 * Ni + Ne, 4 * Ni + 2 * Ne,
                       4 * Ni + 3 * Ne, N])
    blk = np.searchsorted(bounds, np.arange(N), side="right") - 1
    rows = np.repeat(np.arange(N), np.diff(sys_.rowptr))
    keep = blk[rows] == blk[sys_.colidx]
    return np.where(keep, sys_.vals, 0.0)
