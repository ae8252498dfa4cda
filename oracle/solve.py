"""Linear solvers of the oracle.  Test infrastructure.

* ``lu_solve``: sparse direct LU (SciPy SuperLU), in place of the paper's MUMPS
  direct solver (Sec. "Solver configurations").
* ``dense_solve``: LAPACK dense solve, for brute-force checks on tiny meshes.
* ``gmres``: textbook GMRES (Arnoldi with modified Gram-Schmidt, Givens
  rotations), optionally restarted and right-preconditioned.  The k-th iterate
  is the unique minimiser of ||b - A x||_2 over x0 + Z K_k, so it can be compared
  iterate by iterate with any other implementation of the same recurrence.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def lu_solve(A: sp.spmatrix, f: np.ndarray) -> np.ndarray:
    return spla.splu(sp.csc_matrix(A)).solve(f)


def dense_solve(A: sp.spmatrix, f: np.ndarray) -> np.ndarray:
    return np.linalg.solve(A.toarray(), f)


def gmres(A, b, x0=None, M=None, restart=None, rtol=1e-10, maxiter=1000,
          record_iterates=False):
    """Right-preconditioned GMRES(restart) (restart=None: no restart).

    Stops when ||b - A x_k||_2 <= rtol ||b||_2 (the recurrence's estimate, which
    equals the true residual norm in exact arithmetic).  Returns (x, info) with
    info = {"its", "res" (relative residual estimates), "iterates"}.
    """
    n = len(b)
    Aop = (lambda v: A @ v) if not callable(A) else A
    Mop = (lambda v: v) if M is None else M
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), {"its": 0, "res": [0.0], "iterates": []}
    m = maxiter if restart is None else restart
    its = 0
    res_hist = []
    iterates = []
    while True:
        r = b - Aop(x)
        beta = np.linalg.norm(r)
        res_hist.append(beta / bnorm)
        if beta <= rtol * bnorm or its >= maxiter:
            break
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            Z[j] = Mop(V[j])
            w = Aop(Z[j])
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            res_hist.append(abs(g[j + 1]) / bnorm)
            if record_iterates:
                y = np.linalg.solve(np.triu(H[:j + 1, :j + 1]), g[:j + 1])
                iterates.append(x + Z[:j + 1].T @ y)
            if abs(g[j + 1]) <= rtol * bnorm or its >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + Z[:j_done].T @ y
        if abs(g[j_done]) <= rtol * bnorm or its >= maxiter:
            r = b - Aop(x)
            res_hist.append(np.linalg.norm(r) / bnorm)
            break
    return x, {"its": its, "res": res_hist, "iterates": iterates}
