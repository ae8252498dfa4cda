"""Discrete adjoint of the time loop with checkpointing, behind torch.autograd.

Objective: J(theta) = sum_{n=1}^{N_t} dt sum_p phi_e^n(x_p)^2 at probe vertices;
theta_c multiplies every leak conductance of cell c.  With R_n = A(u_{n-1},
theta) u_n - f(u_{n-1}, theta) (eq. ``lin_sys``) and the Lagrangian
J - sum_n lambda_n^T R_n, the adjoint recursion runs backwards from n = N_t:

  A_{n-1}^T lambda_n = dj_n/du_n - (dR_{n+1}/du_n)^T lambda_{n+1},
  dJ/dtheta = - sum_n (dR_n/dtheta)^T lambda_n.

Every piece runs in libknp: the transposed solve with the same AMG(P_0)
preconditioner (knp_adjoint_solve) and the vector-Jacobian products
(knp_step_vjp).  The forward trajectory is kept only at checkpoints every
`every` steps; each segment is recomputed (bitwise identically) before its
reverse sweep.  Passive-leak membranes only.

Accuracy: the probe potentials are ~1e-5 of the potential block and ~1e-8 of
the concentrations, so the forward tolerance `rtol` (relative to the whole
scaled right-hand side) bounds the relative accuracy of J and its gradient;
rtol 1e-14 gives phi_e at the probes to ~1e-9.  The adjoint right-hand side sits
on the probe DOFs alone and lambda is ~1e19 times larger than it, which puts
the attainable adjoint residual near 1e-12 at 4e3 unknowns and near 1e-9 at
2e6.  A solve that stops on its floor (KNP_E_NOCONV) is accepted when its
recomputed residual is within 10 x its rtol (`fwd_accept`, `adj_accept`); the
residuals reached are kept in stats["forward_rel_res"] and ["adjoint_rel_res"].
"""
from __future__ import annotations

import numpy as np
import torch

from .knp import solve_opts
from .simulate import KnpSolver


class AdjointProblem:
    def __init__(self, case, device=0, every=8, rtol=1e-12, adj_rtol=1e-10, restart=400, amg=None,
                 progress=None, adj_accept=None, fwd_accept=None, max_it=4000):
        if np.any(case.cell_model != 0):
            raise ValueError("the adjoint supports passive-leak membranes only")
        if every < 1:
            raise ValueError("checkpoint interval must be >= 1")
        self.case = case
        self.every = every
        self.opts = solve_opts(rtol=rtol, restart=restart, max_it=max_it, reorth=1)
        self.adj_opts = solve_opts(rtol=adj_rtol, restart=restart, max_it=max_it, reorth=1)
        self.adj_accept = 10.0 * adj_rtol if adj_accept is None else adj_accept
        self.fwd_accept = 10.0 * rtol if fwd_accept is None else fwd_accept
        self.solver = KnpSolver(case, device=device, amg=amg, solve=self.opts)
        s = self.solver
        self.u0 = s.u.clone()
        info = s.info
        # phi_e DOF of each probe vertex
        phe = slice(4 * info.N_i + 3 * info.N_e, 4 * (info.N_i + info.N_e))
        vert_of = s.dof_vertex[phe]
        local = {int(v): i for i, v in enumerate(vert_of)}
        idx = [4 * info.N_i + 3 * info.N_e + local[int(p)] for p in case.probes]
        self.pd = torch.tensor(idx, dtype=torch.int64, device=s.dev)
        self.stats = {"forward_its": [], "forward_rel_res": [], "adjoint_its": [], "adjoint_rel_res": []}
        self.progress = progress          # optional callable(str), one line per solve

    # ------------------------------------------------------------------ forward
    def _step(self, u_prev, n, theta):
        s = self.solver
        s.u = u_prev
        s.theta = theta
        s.assemble(n)
        x, info, ok = s.solve(allow_noconv=True)
        if not ok and not info.rel_res <= self.fwd_accept:
            raise RuntimeError(f"forward solve of step {n} stalled at relative residual {info.rel_res:.3e} "
                               f"(rtol {self.opts.rtol:g}, accepted up to {self.fwd_accept:g}) after "
                               f"{info.its} iterations")
        self.stats["forward_its"].append(info.its)
        self.stats["forward_rel_res"].append(info.rel_res)
        if self.progress:
            self.progress(f"forward step {n}: {info.its} its, rel_res {info.rel_res:.2e}")
        return x

    def forward(self, theta):
        """J and the checkpoints {n: u_n} for n = 0, every, 2 every, ..."""
        case = self.case
        theta = theta.detach().to(self.solver.dev, torch.float64).contiguous()
        u = self.u0.clone()
        ckpt = {0: u.clone()}
        J = torch.zeros((), dtype=torch.float64, device=self.solver.dev)
        for n in range(1, case.n_steps + 1):
            u = self._step(u, n, theta)
            J = J + case.dt * torch.sum(u[self.pd] ** 2)
            if n % self.every == 0:
                ckpt[n] = u.clone()
        return J, ckpt

    # ------------------------------------------------------------------ reverse
    def gradient(self, theta, ckpt=None):
        case = self.case
        s = self.solver
        theta = theta.detach().to(s.dev, torch.float64).contiguous()
        if ckpt is None:
            _, ckpt = self.forward(theta)
        N = s.info.N
        carry = torch.zeros(N, dtype=torch.float64, device=s.dev)
        tbar = torch.zeros(s.info.n_cells, dtype=torch.float64, device=s.dev)
        starts = sorted(ckpt)
        lam_next = lam_next2 = None   # lambda_{n+1}, lambda_{n+2}: the initial guess of step n
        for k in range(len(starts) - 1, -1, -1):
            a = starts[k]
            b = starts[k + 1] if k + 1 < len(starts) else case.n_steps
            if b <= a:
                continue
            seg = [ckpt[a]]
            for n in range(a + 1, b + 1):          # recompute the segment
                seg.append(self._step(seg[-1], n, theta))
            for n in range(b, a, -1):
                u_n, u_prev = seg[n - a], seg[n - a - 1]
                rhs = -carry
                rhs[self.pd] += 2.0 * case.dt * u_n[self.pd]
                s.u = u_prev
                s.theta = theta
                s.assemble(n)                      # A_{n-1} for this step
                # the adjoint state changes little from one step to the next, as the forward
                # state does, so the solve starts from the later steps' solutions, linearly
                # extrapolated once two are known
                if lam_next is None:
                    lam = torch.zeros(N, dtype=torch.float64, device=s.dev)
                elif lam_next2 is None:
                    lam = lam_next.clone()
                else:
                    lam = 2.0 * lam_next - lam_next2
                info, ok = s.ctx.adjoint_solve(rhs, lam, self.adj_opts, allow_noconv=True)
                lam_next2, lam_next = lam_next, lam
                if not ok and not info.rel_res <= self.adj_accept:
                    raise RuntimeError(f"adjoint solve of step {n} stalled at relative residual "
                                       f"{info.rel_res:.3e} (rtol {self.adj_opts.rtol:g}, accepted up to "
                                       f"{self.adj_accept:g}) after {info.its} iterations")
                self.stats["adjoint_its"].append(info.its)
                self.stats["adjoint_rel_res"].append(info.rel_res)
                if self.progress:
                    self.progress(f"adjoint step {n}: {info.its} its, rel_res {info.rel_res:.2e}")
                carry = torch.zeros(N, dtype=torch.float64, device=s.dev)
                s.ctx.step_vjp(u_prev, u_n, lam, carry, tbar)
        return -tbar


class ProbeObjective(torch.autograd.Function):
    """J(theta) with a hand-written discrete-adjoint backward."""

    @staticmethod
    def forward(ctx, theta, problem):
        J, ckpt = problem.forward(theta)
        ctx.problem = problem
        ctx.ckpt = ckpt
        ctx.save_for_backward(theta)
        return J

    @staticmethod
    def backward(ctx, gJ):
        (theta,) = ctx.saved_tensors
        grad = ctx.problem.gradient(theta, ctx.ckpt)
        return (gJ * grad).to(theta.device, theta.dtype), None
