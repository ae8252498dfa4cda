"""Gradient of a time-integrated probe objective with respect to per-cell leak
factors, by the tangent-linear (forward-sensitivity) method.  Test infrastructure.

Objective:  J(theta) = sum_{n=1}^{N_t} dt sum_p phi_e^n(x_p)^2 over probe vertices
x_p, where u_n solves R_n(u_n, u_{n-1}, theta) = A(u_{n-1}, theta) u_n - f(u_{n-1}, theta)
= 0 (eq. ``lin_sys``) and theta_c multiplies every leak conductance of cell c.

Gradient (plain definition): for each cell c propagate the sensitivity
  du_n/dtheta_c = -A_{n-1}^{-1} [ (dR_n/du_{n-1}) du_{n-1}/dtheta_c + dR_n/dtheta_c ],
with du_0/dtheta_c = 0, and sum dJ/dtheta_c = sum_n dt sum_p 2 phi_e^n(x_p) dphi_e^n(x_p).
The bracket is one directional derivative of R_n in (u_{n-1}, theta), taken by the
complex-step method on the oracle's own assembly (exact to rounding, no
cancellation).  Passive-leak membranes only (no gates to differentiate).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import Assembler, initial_gates, initial_state
from .mesh import PHI


def probe_dofs(asm: Assembler, probes):
    lay = asm.lay
    return np.asarray(lay.dof(1, PHI, lay.loc[1, np.asarray(probes)]), dtype=np.int64)


def objective(case, theta, n_steps=None, asm=None, keep=False):
    """J(theta) and (optionally) the trajectory, by the oracle time loop.  A complex
    theta propagates through every assembly and LU solve (complex-step use)."""
    asm = asm or Assembler(case)
    n_steps = case.n_steps if n_steps is None else n_steps
    pd = probe_dofs(asm, case.probes)
    u = initial_state(case, asm.lay)
    w = initial_gates(case, asm.lay)
    J = 0.0
    traj = [u]
    for n in range(1, n_steps + 1):
        s = asm.assemble(u, w, n * case.dt, case.dt, theta)
        u = spla.splu(sp.csc_matrix(s.csr())).solve(s.f)
        J = J + case.dt * np.sum(u[pd] ** 2)
        traj.append(u)
    return (J, traj) if keep else J


def gradient_complex_step(case, theta, n_steps=None, h=1e-30):
    """dJ/dtheta_c = Im J(theta + i h e_c) / h through the whole time loop."""
    asm = Assembler(case)
    theta = np.asarray(theta, dtype=np.float64)
    grad = np.zeros(len(theta))
    for c in range(len(theta)):
        th = theta.astype(np.complex128)
        th[c] += 1j * h
        grad[c] = np.imag(objective(case, th, n_steps, asm)) / h
    return grad


def gradient_tangent(case, theta, n_steps=None, h=1e-30):
    """dJ/dtheta for every cell by forward sensitivities with complex-step JVPs."""
    asm = Assembler(case)
    n_steps = case.n_steps if n_steps is None else n_steps
    theta = np.asarray(theta, dtype=np.float64)
    J, traj = objective(case, theta, n_steps, asm, keep=True)
    J = float(np.real(J))
    pd = probe_dofs(asm, case.probes)
    w = initial_gates(case, asm.lay)
    lus = []
    for n in range(1, n_steps + 1):
        s = asm.assemble(traj[n - 1], w, n * case.dt, case.dt, theta)
        lus.append(spla.splu(sp.csc_matrix(s.csr())))
    grad = np.zeros(len(theta))
    for c in range(len(theta)):
        du = np.zeros(asm.lay.N)
        e = np.zeros(len(theta))
        e[c] = 1.0
        for n in range(1, n_steps + 1):
            u_prev = traj[n - 1] + 1j * h * du
            th = theta + 1j * h * e
            s = asm.assemble(u_prev, w, n * case.dt, case.dt, th)
            R = s.csr() @ traj[n] - s.f
            jvp = np.imag(R) / h
            du = -lus[n - 1].solve(jvp)
            grad[c] += case.dt * float(np.sum(2.0 * traj[n][pd] * du[pd]))
    return J, grad
