"""CPU test of the identity behind the solver's stopping test on converged cycles.

When a flexible GMRES cycle ends with its recurrence estimate within rtol, the library
tests the updated iterate's residual formed from the Arnoldi relation,
r_0 - (S A S) Z y = V (beta e_1 - H y), instead of a product with the operator, and only
while 1e-12 G <= rtol ||S b|| / 100 with G = sqrt(j + 1) sum_k |y_k| ||H e_k||.

Here the same recurrence (classical Gram-Schmidt, preconditioned vectors rounded to FP32,
products and updates in FP64) runs in NumPy on the oracle's scaled system of a 3D
Hodgkin-Huxley cell. At every cycle end whose estimate meets rtol:
- the residual from the relation equals b - A x of the updated iterate to 1e-13 of ||b||,
  and to 1e-14 (G + ||b||): a hundredth of the bound the library assumes;
- it sees what the estimate misses. Unpreconditioned FGMRES(200) loses orthogonality: its
  estimate reaches rtol while the true residual stays above it. The residual from the
  relation is then above rtol too, so such a cycle is never taken for converged.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from knp_inputs import model_a_case
from oracle.assemble import Assembler, initial_gates, initial_state, p0_values


@pytest.fixture(scope="module")
def system():
    case = model_a_case(3, 8, "hh", 5e-5, 2, cfg_id=2)
    asm = Assembler(case)
    lay = asm.lay
    sysm = asm.assemble(initial_state(case, lay), initial_gates(case, lay), case.dt, case.dt, pin=True)
    A = sysm.csr().tocsr()
    S = 1.0 / np.sqrt(np.abs(A.diagonal()))
    As = (sp.diags(S) @ A @ sp.diags(S)).tocsr()
    P0 = sp.csr_matrix((p0_values(sysm, lay), sysm.colidx, sysm.rowptr), shape=A.shape)
    lu = spl.splu((sp.diags(S) @ P0 @ sp.diags(S)).tocsc())
    return As, S * sysm.f, lu


def fgmres_cycle_ends(As, b, precond, m, rtol, max_it=4000):
    """Flexible GMRES(m) from zero; returns, for every cycle end whose estimate meets rtol,
    (estimate, residual from the relation, true residual, their distance, G), relative to ||b||."""
    N = As.shape[0]
    x = np.zeros(N)
    bn = np.linalg.norm(b)
    its = 0
    out = []
    while its < max_it:
        r = b - As @ x
        beta = np.linalg.norm(r)
        if beta / bn <= rtol:
            break
        V = np.zeros((m + 1, N))
        Z = np.zeros((m, N), np.float32)
        H = np.zeros((m + 1, m))
        R = np.zeros((m + 1, m))
        cs, sn, g = np.zeros(m), np.zeros(m), np.zeros(m + 1)
        V[0], g[0] = r / beta, beta
        for j in range(m):
            Z[j] = precond(V[j])
            w = As @ Z[j].astype(np.float64)
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            hn = np.linalg.norm(w)
            H[:j + 1, j], H[j + 1, j] = h, hn
            V[j + 1] = w / hn
            R[:, j] = H[:, j]
            for i in range(j):
                t = cs[i] * R[i, j] + sn[i] * R[i + 1, j]
                R[i + 1, j] = -sn[i] * R[i, j] + cs[i] * R[i + 1, j]
                R[i, j] = t
            den = np.hypot(R[j, j], R[j + 1, j])
            cs[j], sn[j] = R[j, j] / den, R[j + 1, j] / den
            R[j, j], R[j + 1, j] = den, 0.0
            g[j + 1], g[j] = -sn[j] * g[j], cs[j] * g[j]
            its += 1
            if abs(g[j + 1]) / bn <= rtol:
                break
        k = j + 1
        y = np.linalg.solve(np.triu(R[:k, :k]), g[:k])
        x = x + Z[:k].astype(np.float64).T @ y
        if abs(g[k]) / bn <= rtol:
            c = -H[:k + 1, :k] @ y
            c[0] += beta
            r_rel = V[:k + 1].T @ c
            r_true = b - As @ x
            G = np.sqrt(k + 1) * np.sum(np.abs(y) * np.linalg.norm(H[:k + 1, :k], axis=0))
            out.append((abs(g[k]) / bn, np.linalg.norm(r_rel) / bn, np.linalg.norm(r_true) / bn,
                        np.linalg.norm(r_rel - r_true) / bn, G / bn))
    return out


@pytest.mark.parametrize("precond,m", [("lu", 30), ("lu", 200), ("none", 200), ("none", 30)])
def test_residual_from_the_arnoldi_relation(system, precond, m):
    As, b, lu = system
    M = (lambda v: lu.solve(v).astype(np.float32)) if precond == "lu" else (lambda v: v.astype(np.float32))
    rtol = 1e-6
    ends = fgmres_cycle_ends(As, b, M, m, rtol)
    assert ends
    for est, rel, true, gap, G in ends:
        print(f"  est {est:.3e} relation {rel:.3e} true {true:.3e} gap {gap:.1e} G {G:.1e}")
        # the rounding of the relation grows with G; the product b - A x carries its own
        # (of order the unit roundoff times ||b|| here), hence G + 1
        assert gap <= 1e-13 and gap <= 1e-14 * (G + 1.0)
        assert (rel <= rtol) == (true <= rtol)
    if (precond, m) == ("none", 200):
        # the estimate met rtol while the true residual did not; the relation saw it
        assert any(true > rtol and rel > rtol for est, rel, true, gap, G in ends)
