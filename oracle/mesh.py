"""Degrees of freedom, membrane facets and the structural sparsity pattern.

Follows Sec. "Spatial discretization" and "Algebraic structure and matrix
assembly": one P1 space per region, Gamma vertices duplicated (one copy per
region, as the Model A DOF-count formula implies), unknowns ordered
[c_i^1..c_i^K, phi_i, c_e^1..c_e^K, phi_e] block by block (eq. ``lin_sys``),
region DOFs in ascending global vertex id.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

NF = 4          # fields per region: Na, K, Cl, phi
PHI = 3


@dataclass
class Layout:
    dim: int
    n_vert: int
    verts: tuple            # (V_i, V_e): sorted global vertex ids per region
    loc: np.ndarray         # int64 [2, n_vert]; region-local index or -1
    gamma: np.ndarray       # sorted global ids of membrane vertices
    facets: np.ndarray      # int64 [n_f, dim]; membrane facets (sorted vertex ids; for P2
                            # then the facet's edge nodes)
    facet_cell: np.ndarray  # int64 [n_f]; cell id (>= 1) of the ICS side
    vert_cell: np.ndarray   # int64 [n_vert]; cell id of ICS vertices, 0 otherwise
    pin_vertex: int

    @property
    def N_r(self):
        return (len(self.verts[0]), len(self.verts[1]))

    @property
    def N(self):
        return NF * (self.N_r[0] + self.N_r[1])

    def off(self, r):
        return 0 if r == 0 else NF * self.N_r[0]

    def dof(self, r, f, local):
        """Global DOF of field f in region r at region-local index ``local``."""
        return self.off(r) + f * self.N_r[r] + np.asarray(local)

    @property
    def pin_dof(self):
        return int(self.dof(1, PHI, self.loc[1, self.pin_vertex]))


def element_faces(elem):
    """All faces (d vertices, sorted) of all simplices, with their element index."""
    d1 = elem.shape[1]
    faces = []
    for drop in range(d1):
        keep = [a for a in range(d1) if a != drop]
        faces.append(elem[:, keep])
    faces = np.sort(np.concatenate(faces, axis=0), axis=1)
    owner = np.tile(np.arange(elem.shape[0]), d1)
    return faces, owner


def build_layout(case) -> Layout:
    elem = case.elem.astype(np.int64)
    tag = case.tag.astype(np.int64)
    n_vert = case.n_vert
    ics = tag >= 1
    Vi = np.unique(elem[ics])
    Ve = np.unique(elem[~ics])
    loc = -np.ones((2, n_vert), dtype=np.int64)
    loc[0, Vi] = np.arange(len(Vi))
    loc[1, Ve] = np.arange(len(Ve))

    vert_cell = np.zeros(n_vert, dtype=np.int64)
    lo = np.full(n_vert, np.iinfo(np.int64).max)
    ev = elem[ics]
    et = np.repeat(tag[ics], ev.shape[1])
    np.maximum.at(vert_cell, ev.ravel(), et)
    np.minimum.at(lo, ev.ravel(), et)
    if np.any((vert_cell > 0) & (lo != vert_cell)):
        raise ValueError("two cells share a vertex")

    elem_v = getattr(case, "elem_vertices", elem)      # P2: the vertex columns
    faces, owner = element_faces(elem_v)
    key_order = np.lexsort(faces.T[::-1])
    faces = faces[key_order]
    owner = owner[key_order]
    same = np.all(faces[1:] == faces[:-1], axis=1)
    first = np.nonzero(same)[0]
    t1 = tag[owner[first]]
    t2 = tag[owner[first + 1]]
    is_gamma = (t1 == 0) != (t2 == 0)
    if np.any((t1 != t2) & (t1 > 0) & (t2 > 0)):
        raise ValueError("two cells share a facet")
    facets = faces[first[is_gamma]]
    if getattr(case, "degree", 1) == 2:
        from .p2 import facet_nodes
        facets = facet_nodes(case, facets)
    facet_cell = np.maximum(t1[is_gamma], t2[is_gamma])
    # boundary faces (appearing once) must be extracellular
    count_two = np.zeros(len(faces), dtype=bool)
    count_two[first] = True
    count_two[first + 1] = True
    if np.any(tag[owner[~count_two]] != 0):
        raise ValueError("a cell touches the outer boundary")
    gamma = np.intersect1d(Vi, Ve)
    if case.pin_vertex in set(gamma.tolist()) or loc[1, case.pin_vertex] < 0:
        raise ValueError("pinned vertex must be an extracellular vertex off the membrane")
    return Layout(case.dim, n_vert, (Vi, Ve), loc, gamma, facets, facet_cell, vert_cell,
                  int(case.pin_vertex))


def region_pairs(case, lay: Layout, r: int) -> np.ndarray:
    """Ordered pairs (a, b) of region-local indices sharing an element of region r."""
    elem = case.elem.astype(np.int64)
    sel = (case.tag >= 1) if r == 0 else (case.tag == 0)
    el = lay.loc[r][elem[sel]]
    d1 = el.shape[1]
    a = np.repeat(el, d1, axis=1).ravel()
    b = np.tile(el, (1, d1)).ravel()
    Nr = lay.N_r[r]
    keys = np.unique(a * Nr + b)
    return np.stack([keys // Nr, keys % Nr], axis=1)


def gamma_pairs(lay: Layout) -> np.ndarray:
    """Ordered pairs (a, b) of global vertex ids sharing a membrane facet."""
    f = lay.facets
    d = f.shape[1]
    a = np.repeat(f, d, axis=1).ravel()
    b = np.tile(f, (1, d)).ravel()
    keys = np.unique(a * lay.n_vert + b)
    return np.stack([keys // lay.n_vert, keys % lay.n_vert], axis=1)


def structural_pattern(case, lay: Layout):
    """CSR pattern (rowptr int64, colidx int32) of the global matrix.

    Every (row, column) that any element or membrane facet couples in the block
    rows of eq. ``lin_sys``: per region r and partner q,
      c_r^k rows: columns c_r^k (P_r), phi_r (P_r), phi_q (Gamma pairs),
      phi_r rows: columns c_r^1..c_r^K (P_r), phi_r (P_r), phi_q (Gamma pairs).
    Zeros are kept; the pinned row and column keep their pattern.
    """
    rows, cols = [], []
    gp = gamma_pairs(lay)
    for r in (0, 1):
        q = 1 - r
        P = region_pairs(case, lay, r)
        ga = lay.loc[r][gp[:, 0]]
        gb = lay.loc[q][gp[:, 1]]
        for k in range(3):
            rows += [lay.dof(r, k, P[:, 0]), lay.dof(r, k, P[:, 0]), lay.dof(r, k, ga)]
            cols += [lay.dof(r, k, P[:, 1]), lay.dof(r, PHI, P[:, 1]), lay.dof(q, PHI, gb)]
        for k in range(3):
            rows.append(lay.dof(r, PHI, P[:, 0]))
            cols.append(lay.dof(r, k, P[:, 1]))
        rows += [lay.dof(r, PHI, P[:, 0]), lay.dof(r, PHI, ga)]
        cols += [lay.dof(r, PHI, P[:, 1]), lay.dof(q, PHI, gb)]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    N = lay.N
    keys = np.unique(rows * N + cols)
    r_ = keys // N
    c_ = keys % N
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(rowptr, r_ + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, c_.astype(np.int32)


def embed(A: sp.spmatrix, rowptr, colidx) -> np.ndarray:
    """Values of A laid out on the structural pattern; fails if A has a nonzero
    outside the pattern."""
    N = len(rowptr) - 1
    A = A.tocoo()
    keys_pat = np.repeat(np.arange(N, dtype=np.int64), np.diff(rowptr)) * N + colidx
    vals = np.zeros(len(colidx), dtype=A.dtype)
    keys = A.row.astype(np.int64) * N + A.col
    pos = np.searchsorted(keys_pat, keys)
    pos_c = np.minimum(pos, len(keys_pat) - 1)
    hit = keys_pat[pos_c] == keys
    if np.any(A.data[~hit] != 0.0):
        raise AssertionError("matrix has a nonzero outside the structural pattern")
    np.add.at(vals, pos_c[hit], A.data[hit])
    return vals
