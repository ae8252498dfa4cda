"""Quadratic (P2) Lagrange elements for the oracle.  Test infrastructure.

Sec. "Spatial discretization" admits Lagrange elements of any order p on the
conforming simplicial mesh, one space for all fields of a region; the robustness
study and Model D use p = 2.  A P2 space has one node per vertex and one per edge;
nodes on Gamma (its vertices and the edges of its facets) are duplicated, one copy
per region, which is what the Model A DOF-count formula states for general p.

Everything the P1 oracle does carries over node by node:
  * nodes: vertex v keeps id v; edge e (sorted vertex pair, lexicographic order)
    gets id n_vert + e;
  * element nodes: the d+1 vertices, then the edges (a, b), a < b, in
    lexicographic order of the local pair; facet nodes likewise;
  * nonlinear membrane coefficients are evaluated at the membrane nodes and
    treated as P2 fields on Gamma (the P1 reading, node by node);
  * the initial data at an edge node is the mean of its two vertices' values
    (the P1 interpolant of the per-vertex data);
  * every integral is exact: products of basis functions are polynomials in the
    barycentric coordinates, integrated with
    int_T prod lambda_a^{p_a} = m! |T| prod p_a! / (m + sum p_a)!.
"""
from __future__ import annotations

import copy
from functools import lru_cache
from itertools import combinations
from math import factorial

import numpy as np


# --------------------------------------------------------------------------- polynomials
def _basis(m):
    """P2 basis on the m-simplex: lambda_a (2 lambda_a - 1) at the vertices, then
    4 lambda_a lambda_b at the edges; each a dict exponent-tuple -> coefficient."""
    n = m + 1
    out = []
    for a in range(n):
        e2 = [0] * n
        e2[a] = 2
        e1 = [0] * n
        e1[a] = 1
        out.append({tuple(e2): 2.0, tuple(e1): -1.0})
    for a, b in combinations(range(n), 2):
        e = [0] * n
        e[a] = e[b] = 1
        out.append({tuple(e): 4.0})
    return out


def _mul(p, q):
    r = {}
    for ep, cp in p.items():
        for eq, cq in q.items():
            e = tuple(x + y for x, y in zip(ep, eq))
            r[e] = r.get(e, 0.0) + cp * cq
    return r


def _diff(p, i):
    r = {}
    for e, c in p.items():
        if e[i] > 0:
            f = list(e)
            f[i] -= 1
            r[tuple(f)] = r.get(tuple(f), 0.0) + c * e[i]
    return r


def _integral(p, m):
    """int over an m-simplex of p, divided by its measure."""
    s = 0.0
    for e, c in p.items():
        num = factorial(m)
        for x in e:
            num *= factorial(x)
        s += c * num / factorial(m + sum(e))
    return s


@lru_cache(maxsize=None)
def reference_tensors(d):
    """Per unit measure: M[a,b] = int phi_a phi_b; S[a,b,i,j] = int d_i phi_a d_j phi_b;
    W[m,a,b,i,j] = int phi_m d_i phi_a d_j phi_b (d_i: derivative in lambda_i)."""
    B = _basis(d)
    n = len(B)
    dB = [[_diff(b, i) for i in range(d + 1)] for b in B]
    M = np.array([[_integral(_mul(B[a], B[b]), d) for b in range(n)] for a in range(n)])
    S = np.zeros((n, n, d + 1, d + 1))
    W = np.zeros((n, n, n, d + 1, d + 1))
    for a in range(n):
        for b in range(n):
            for i in range(d + 1):
                for j in range(d + 1):
                    pij = _mul(dB[a][i], dB[b][j])
                    S[a, b, i, j] = _integral(pij, d)
                    for k in range(n):
                        W[k, a, b, i, j] = _integral(_mul(B[k], pij), d)
    return M, S, W


@lru_cache(maxsize=None)
def facet_tensors(m):
    """Per unit measure on an m-simplex: F2[a,b] = int phi_a phi_b and
    F3[a,b,c] = int phi_a phi_b phi_c."""
    B = _basis(m)
    n = len(B)
    F2 = np.array([[_integral(_mul(B[a], B[b]), m) for b in range(n)] for a in range(n)])
    F3 = np.array([[[_integral(_mul(_mul(B[a], B[b]), B[c]), m) for c in range(n)]
                    for b in range(n)] for a in range(n)])
    return F2, F3


# --------------------------------------------------------------------------- the P2 case
def _edges(elem_v):
    """Sorted unique vertex pairs of all element edges, and each element's edge ids
    in local lexicographic pair order."""
    d1 = elem_v.shape[1]
    pairs = list(combinations(range(d1), 2))
    a = np.stack([np.minimum(elem_v[:, i], elem_v[:, j]) for i, j in pairs], axis=1)
    b = np.stack([np.maximum(elem_v[:, i], elem_v[:, j]) for i, j in pairs], axis=1)
    nv = int(elem_v.max()) + 1
    keys = a * nv + b
    uniq, inv = np.unique(keys.ravel(), return_inverse=True)
    edges = np.stack([uniq // nv, uniq % nv], axis=1)
    return edges, inv.reshape(keys.shape)


def p2_case(case):
    """The same workload with P2 nodes standing in for the vertices: node
    coordinates, element and facet node lists, and per-node initial data."""
    c = copy.copy(case)
    elem_v = case.elem.astype(np.int64)
    nv = case.n_vert
    edges, eid = _edges(elem_v)
    c.degree = 2
    c.elem_vertices = elem_v
    c.n_vert_p1 = nv
    c.edges = edges
    c.elem = np.concatenate([elem_v, nv + eid], axis=1)
    c.xyz = np.concatenate([case.xyz, 0.5 * (case.xyz[edges[:, 0]] + case.xyz[edges[:, 1]])], axis=0)
    c.conc0 = np.concatenate([case.conc0, 0.5 * (case.conc0[:, :, edges[:, 0]] + case.conc0[:, :, edges[:, 1]])],
                             axis=2)
    return c


def facet_nodes(case, facets_v):
    """P2 node lists of facets given by their sorted vertex ids."""
    nv = case.n_vert_p1
    keys_all = case.edges[:, 0] * nv + case.edges[:, 1]
    cols = [facets_v]
    for i, j in combinations(range(facets_v.shape[1]), 2):
        a = np.minimum(facets_v[:, i], facets_v[:, j])
        b = np.maximum(facets_v[:, i], facets_v[:, j])
        pos = np.searchsorted(keys_all, a * nv + b)
        if np.any(keys_all[np.minimum(pos, len(keys_all) - 1)] != a * nv + b):
            raise AssertionError("facet edge not among the element edges")
        cols.append((nv + pos)[:, None])
    return np.concatenate(cols, axis=1)
