"""Time loop on the device: for n = 1..N_t assemble A_{n-1}, f_n and solve with
GMRES + AMG(P_0) (Sec. "Time discretization", Sec. "Solver configurations").
P_0 and its hierarchy are built once, after the first assembly."""
from __future__ import annotations

import numpy as np
import torch

from .knp import Context, amg_opts, solve_opts


def initial_vector(case, dof_vertex, info, edges=None):
    """u_0 in the library's DOF layout from per-vertex initial data.  With the edge list of
    an order-2 mesh, the data at the edge node n_vert + e is the mean of its two vertices'
    (the linear interpolant of the per-vertex data)."""
    conc = case.conc0
    if edges is not None and len(edges):
        conc = np.concatenate([conc, 0.5 * (conc[:, :, edges[:, 0]] + conc[:, :, edges[:, 1]])], axis=2)
    u0 = np.empty(info.N)
    Nr = (info.N_i, info.N_e)
    off = (0, 4 * info.N_i)
    for r in (0, 1):
        for f in range(4):
            sl = slice(off[r] + f * Nr[r], off[r] + (f + 1) * Nr[r])
            u0[sl] = conc[r, f, dof_vertex[sl]] if f < 3 else case.phi0[r]
    return u0


# AMG settings swept on the 132^3 lattice (steps 6-25, FP32 levels) in each gauge (the
# other options keep the library's defaults).  With the point condition (gauge 0) the
# per-cell potential modes keep the iteration count up and a cheap cycle wins; with the
# nullspace handled by the solve (gauge 1) more smoothing on the coarser levels pays.
AMG_BY_GAUGE = {
    0: dict(cheb_degree=5, cheb_ratio=2.5, coarse_drop=0.01, coarse_post_degree=1),
    1: dict(cheb_degree=3, cheb_ratio=3.5, coarse_drop=0.02, coarse_post_degree=4),
}


class KnpSolver:
    """Holds one context and the state (u, gates) of a run on one GPU."""

    def __init__(self, case, device=0, amg=None, solve=None, theta=None, order=1, gauge=0, extrapolate=False):
        """case: a vertex mesh with per-vertex data; order 2 adds the edge nodes (P2);
        gauge: 0 = point condition on phi_e in the system, 1 = nullspace handled by the
        solve (knp_set_gauge); extrapolate: start each solve from 2 u_{n-1} - u_{n-2}
        (knp_extrapolate) once two steps are known, instead of from u_{n-1}."""
        self.case = case
        self.order = order
        self.gauge = gauge
        self.extrapolate = extrapolate
        self._u_prev = None
        self.dev = torch.device("cuda", device)
        self.ctx = Context(device)
        self.info = self.ctx.mesh_upload(case.dim, case.xyz, case.elem, case.tag, case.pin_vertex, order=order)
        if gauge:
            self.ctx.set_gauge(gauge)
        self.ctx.set_params(case.params, case.cell_model, case.cell_stim)
        self.rowptr, self.colidx, self.dof_vertex = self.ctx.get_layout()
        self.gamma = self.ctx.get_gamma()
        self.edges = self.ctx.get_edges() if order == 2 else None
        u0 = initial_vector(case, self.dof_vertex, self.info, self.edges)
        self.u = torch.tensor(u0, dtype=torch.float64, device=self.dev)
        g0 = np.tile(np.asarray(case.params["gates0"], dtype=np.float64), (self.info.n_gamma, 1))
        self.gates = torch.tensor(g0, dtype=torch.float64, device=self.dev).contiguous()
        th = case.theta if theta is None else theta
        self.theta = torch.as_tensor(np.asarray(th, dtype=np.float64), device=self.dev).contiguous()
        self.f = torch.empty(self.info.N, dtype=torch.float64, device=self.dev)
        self.amg_opts = amg if amg is not None else amg_opts()
        self.solve_opts = solve if solve is not None else solve_opts()
        self.amg_ready = False
        self.n = 0
        self.history = []

    @property
    def u(self):
        return self._u

    @u.setter
    def u(self, v):
        # a state set from outside starts a new history (no extrapolation from it)
        self._u = v
        self._u_prev = None

    def membrane_rows(self):
        """Device indices (phi_i rows, phi_e rows) of the membrane nodes (vertices, and
        edge nodes n_vert + e at order 2), in the order of knp_get_gamma, so that
        phi_M = u[rows_i] - u[rows_e]."""
        Ni, Ne = self.info.N_i, self.info.N_e
        n_nodes = self.case.n_vert + (len(self.edges) if self.edges is not None else 0)
        pos_i = np.full(n_nodes, -1, np.int64)
        pos_e = np.full(n_nodes, -1, np.int64)
        pos_i[self.dof_vertex[3 * Ni:4 * Ni]] = np.arange(3 * Ni, 4 * Ni)
        pos_e[self.dof_vertex[4 * Ni + 3 * Ne:]] = np.arange(4 * Ni + 3 * Ne, 4 * Ni + 4 * Ne)
        ri, re = pos_i[self.gamma], pos_e[self.gamma]
        if np.any(ri < 0) or np.any(re < 0):
            raise RuntimeError("membrane vertex without a DOF in both regions")
        return (torch.as_tensor(ri, device=self.dev), torch.as_tensor(re, device=self.dev))

    def assemble(self, n=None):
        """Assemble step n; the hierarchy is built after the first assembly, and rebuilt
        after every one when the AMG options ask for the time-dependent P_n."""
        n = self.n + 1 if n is None else n
        self.ctx.assemble_step(n * self.case.dt, self.case.dt, self.u, self.gates, self.theta, self.f)
        if not self.amg_ready or self.amg_opts.operator_step == 1:
            self.ctx.amg_setup(self.amg_opts)
            self.amg_ready = True

    def solve(self, allow_noconv=False, opts=None):
        if self.extrapolate and self._u_prev is not None:
            x = torch.empty_like(self._u)
            self.ctx.extrapolate(self._u, self._u_prev, x)
        else:
            x = self._u.clone()
        info, ok = self.ctx.gmres_solve(self.f, x, opts if opts is not None else self.solve_opts,
                                        allow_noconv=allow_noconv)
        return x, info, ok

    def step(self, allow_noconv=False, opts=None):
        self.assemble()
        x, info, ok = self.solve(allow_noconv, opts)
        self._u_prev, self._u = self._u, x
        self.n += 1
        self.history.append({"n": self.n, "its": info.its, "rel_res": info.rel_res, "converged": ok})
        return info

    def run(self, n_steps=None):
        n_steps = self.case.n_steps if n_steps is None else n_steps
        out = [self.u.clone()]
        for _ in range(n_steps):
            self.step()
            out.append(self.u.clone())
        return out
