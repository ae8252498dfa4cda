"""Host check of the static operators behind the order-1 per-step assembly, built with
g++ alone: the row terms of the bulk values (csrc/rows.cpp) and the membrane operators
(csrc/p2.cpp, build_p2_membrane).

For the P1 field c_h of nodal values c, the weighted stiffness int c_h grad phi_i .
grad phi_j of every entry of a region's pattern is rebuilt from the terms as the
kernel forms it (ring sum plus (c_i + c_j)/(d - 1) times the weight sum off the
diagonal, minus the row's off-diagonal sum on it) and compared with the oracle's
weighted stiffness, which integrates element by element; the mass row likewise with the
oracle's mass matrix.  Meshes: a uniform 2D and 3D grid (right-angled elements, where
the dropped weights are those of vanishing integrals), the same grids with every interior
vertex moved at random (no integral vanishes), and a 2D fan whose centre has 41
neighbours.  Also checked: the row groups (consecutive rows, at most 64 entries, the
row-start mask, the largest term count and row length) and the term offsets; and the
membrane integrals int_Gamma C phi_a phi_b (C a P1 membrane field) and int_Gamma phi_a
phi_b of every membrane entry against the oracle's facet integrals.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from knp_inputs import config_case, model_a_case
from knp_inputs.fan import fan_case
from oracle.assemble import bulk_coo, gamma_coo
from oracle.mesh import build_layout

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2403_04491_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "knp_internal.h"
template <typename T> static void rd(FILE *f, std::vector<T> &v, size_t n) {
    v.resize(n);
    if (n && std::fread(v.data(), sizeof(T), n, f) != n) throw 1;
}
template <typename T> static void wr(FILE *f, const std::vector<T> &v, size_t n) {
    if (n) std::fwrite(v.data(), sizeof(T), n, f);
}
int main(int argc, char **argv) {
    FILE *in = std::fopen(argv[1], "rb");
    int64_t hdr[4];
    if (std::fread(hdr, sizeof(int64_t), 4, in) != 4) return 2;
    const int dim = int(hdr[0]);
    std::vector<double> xyz;
    std::vector<int32_t> elem, tag;
    rd(in, xyz, size_t(hdr[1]) * dim);
    rd(in, elem, size_t(hdr[2]) * (dim + 1));
    rd(in, tag, size_t(hdr[2]));
    std::fclose(in);
    knp::HostMesh m;
    knp::build_host_mesh(m, dim, 1, hdr[1], xyz.data(), hdr[2], elem.data(), tag.data(), hdr[3]);
    knp::RowTerms rt[2];
    if (!knp::build_row_terms(m, rt)) return 3;
    FILE *out = std::fopen(argv[2], "wb");
    for (int r = 0; r < 2; ++r) {
        const int64_t nent = m.prow[r][m.Nr[r]];
        const int64_t h[4] = {m.Nr[r], nent, int64_t(rt[r].groups.size()), rt[r].groups.back().term0};
        std::fwrite(h, sizeof(int64_t), 4, out);
        wr(out, m.prow[r], size_t(m.Nr[r] + 1));
        wr(out, m.pcol[r], size_t(nent));
        wr(out, rt[r].groups, rt[r].groups.size());
        wr(out, rt[r].tcount, size_t(nent));
        wr(out, rt[r].tslot, size_t(h[3]));
        wr(out, rt[r].tval, size_t(h[3]));
        wr(out, rt[r].mval, size_t(nent));
    }
    knp::P2Host o;
    knp::build_p2_membrane(m, o);
    const int64_t ng = int64_t(m.gamma.size()), nmem = m.grow[ng];
    const int64_t h2[2] = {ng, o.cptr[nmem]};
    std::fwrite(h2, sizeof(int64_t), 2, out);
    wr(out, m.gamma, size_t(ng));
    wr(out, m.grow, size_t(ng + 1));
    wr(out, m.gcol, size_t(nmem));
    wr(out, o.mg, size_t(nmem));
    wr(out, o.cptr, size_t(nmem + 1));
    wr(out, o.cnode, size_t(h2[1]));
    wr(out, o.cval, size_t(h2[1]));
    wr(out, o.rpos[0], size_t(nmem));
    wr(out, o.rpos[1], size_t(nmem));
    std::fclose(out);
    return 0;
}
"""

GROUP = np.dtype([("term0", "<i8"), ("starts", "<u8"), ("row0", "<i4"), ("tmax", "<i2"), ("nmax", "<i2")])


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("rows")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([gxx, "-O2", "-std=c++17", "-fopenmp", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{CSRC}",
                    str(src), os.path.join(CSRC, "mesh.cpp"), os.path.join(CSRC, "rows.cpp"),
                    os.path.join(CSRC, "p2.cpp"), "-o", str(exe)], check=True)
    return str(exe), d


def _run(driver, case):
    exe, d = driver
    fin, fout = d / "mesh.bin", d / "rows.bin"
    with open(fin, "wb") as f:
        np.array([case.dim, case.xyz.shape[0], case.elem.shape[0], case.pin_vertex], "<i8").tofile(f)
        np.ascontiguousarray(case.xyz, "<f8").tofile(f)
        np.ascontiguousarray(case.elem, "<i4").tofile(f)
        np.ascontiguousarray(case.tag, "<i4").tofile(f)
    subprocess.run([exe, str(fin), str(fout)], check=True)
    buf = open(fout, "rb").read()
    pos, out = 0, []

    def take(dt, n):
        nonlocal pos
        a = np.frombuffer(buf, dtype=dt, count=n, offset=pos)
        pos += a.nbytes
        return a

    for _ in range(2):
        Nr, nent, ng, nt = (int(x) for x in take("<i8", 4))
        out.append(dict(prow=take("<i8", Nr + 1), pcol=take("<i4", nent), groups=take(GROUP, ng),
                        tcount=take("u1", nent), tslot=take("u1", nt), tval=take("<f8", nt), mval=take("<f8", nent)))
    ng, nt = (int(x) for x in take("<i8", 2))
    mem = dict(gamma=take("<i4", ng), grow=take("<i8", ng + 1))
    nmem = int(mem["grow"][-1])
    mem.update(gcol=take("<i4", nmem), mg=take("<f8", nmem), cptr=take("<i8", nmem + 1), cnode=take("<i4", nt),
               cval=take("<f8", nt), rpos=(take("<i4", nmem), take("<i4", nmem)))
    out.append(mem)
    return out


def _jitter(case, amount, seed):
    """Move every vertex off the outer boundary by up to amount of the local spacing."""
    xyz = case.xyz.copy()
    lo, hi = xyz.min(axis=0), xyz.max(axis=0)
    h = (hi - lo) / np.array(case.shape)
    inner = np.all((xyz > lo + 0.5 * h) & (xyz < hi - 0.5 * h), axis=1)
    rng = np.random.default_rng(seed)
    xyz[inner] += amount * h * rng.uniform(-1.0, 1.0, size=(int(inner.sum()), case.dim))
    case.xyz = xyz
    return case


CASES = {
    "grid2d": lambda: model_a_case(2, 8, "leak", 1e-4, 1),
    "grid3d": lambda: model_a_case(3, 4, "leak", 5e-5, 1),
    "lattice3d": lambda: config_case(3, per_pitch=5),
    "grid2d_moved": lambda: _jitter(model_a_case(2, 8, "leak", 1e-4, 1), 0.2, 1),
    "grid3d_moved": lambda: _jitter(model_a_case(3, 4, "leak", 5e-5, 1), 0.2, 2),
    "fan40": lambda: fan_case(),
}


def _products(rt, d, c):
    """Per entry of the region's pattern: the weighted stiffness from the terms."""
    prow, pcol, tcount = rt["prow"], rt["pcol"], rt["tcount"].astype(np.int64)
    nent = len(pcol)
    rows = np.repeat(np.arange(len(prow) - 1), np.diff(prow))
    toff = np.concatenate([[0], np.cumsum(tcount)])
    ent_of_term = np.repeat(np.arange(nent), tcount)
    wcol = pcol[prow[rows[ent_of_term]] + rt["tslot"]]       # weight vertex of each term
    ring = np.bincount(ent_of_term, weights=rt["tval"] * c[wcol], minlength=nent)
    wsum = np.bincount(ent_of_term, weights=rt["tval"], minlength=nent)
    diag = pcol == rows
    V = ring + wsum * (c[rows] + c[pcol]) / (d - 1)
    V[diag] = 0.0
    V[diag] = -np.bincount(rows, weights=V, minlength=len(prow) - 1)
    assert toff[-1] == len(rt["tval"])
    return rows, V


@pytest.mark.parametrize("name", list(CASES))
def test_row_terms_rebuild_the_weighted_stiffness_and_mass(driver, name):
    case = CASES[name]()
    lay = build_layout(case)
    rts = _run(driver, case)[:2]
    rng = np.random.default_rng(11)
    for r in (0, 1):
        rt = rts[r]
        Nr = len(rt["prow"]) - 1
        if Nr == 0:
            continue
        c = rng.uniform(1.0, 150.0, size=Nr)
        rows, V = _products(rt, case.dim, c)
        # oracle: element by element, the P1 weight of the region-local nodal values c
        Ki, Kj, Kv = bulk_coo(case, lay, r, weight=c, kind="stiff")
        K = sp.csr_matrix((Kv, (Ki, Kj)), shape=(Nr, Nr))
        want = np.asarray(K[rows, rt["pcol"]]).ravel()
        rowmax = np.maximum.reduceat(np.abs(want), rt["prow"][:-1])
        err = np.abs(V - want) / rowmax[rows]
        assert err.max() <= 1e-12, (r, err.max())
        Mi, Mj, Mv = bulk_coo(case, lay, r, kind="mass")
        M = sp.csr_matrix((Mv, (Mi, Mj)), shape=(Nr, Nr))
        mwant = np.asarray(M[rows, rt["pcol"]]).ravel()
        assert np.allclose(rt["mval"], mwant, rtol=1e-13, atol=1e-15 * np.abs(mwant).max())


@pytest.mark.parametrize("name", list(CASES))
def test_membrane_operators_rebuild_the_membrane_integrals(driver, name):
    """The membrane operators of an order-1 mesh (the product form's, used with the row
    terms): int_Gamma C phi_a phi_b from the terms (C a random P1 membrane field) and the
    membrane mass, per entry of the membrane adjacency, against the oracle's facet
    integrals; each entry's positions in its regions' scalar rows."""
    case = CASES[name]()
    lay = build_layout(case)
    res = _run(driver, case)
    mem = res[2]
    ng = len(mem["gamma"])
    if ng == 0:
        return
    assert np.array_equal(mem["gamma"], lay.gamma)
    grow, gcol = mem["grow"], mem["gcol"]
    nmem = len(gcol)
    a_of = np.repeat(np.arange(ng), np.diff(grow))
    Cm = np.random.default_rng(5).uniform(-2.0, 3.0, size=ng)       # by membrane index
    C = np.zeros(case.xyz.shape[0])
    C[lay.gamma] = Cm
    ent = np.repeat(np.arange(nmem), np.diff(mem["cptr"]))
    got = np.bincount(ent, weights=mem["cval"] * Cm[mem["cnode"]], minlength=nmem)
    n = case.xyz.shape[0]
    for weight, vals in ((C, got), (None, mem["mg"])):
        Gi, Gj, Gv = gamma_coo(case, lay, weight=weight)
        Gm = sp.csr_matrix((Gv, (Gi, Gj)), shape=(n, n))
        want = np.asarray(Gm[mem["gamma"][a_of], gcol]).ravel()
        assert np.abs(vals - want).max() <= 1e-13 * np.abs(want).max()
    for r in (0, 1):
        prow, pcol = res[r]["prow"], res[r]["pcol"]
        la = lay.loc[r][mem["gamma"][a_of]]
        assert np.array_equal(pcol[prow[la] + mem["rpos"][r]], lay.loc[r][gcol])


@pytest.mark.parametrize("name", ["grid3d", "grid2d_moved", "fan40"])
def test_row_groups_cover_the_rows(driver, name):
    case = CASES[name]()
    for rt in _run(driver, case)[:2]:
        prow, g = rt["prow"], rt["groups"]
        Nr = len(prow) - 1
        assert g["row0"][0] == 0 and g["row0"][-1] == Nr
        assert np.all(np.diff(g["row0"]) > 0)
        toff = np.concatenate([[0], np.cumsum(rt["tcount"].astype(np.int64))])
        for k in range(len(g) - 1):
            r0, r1 = int(g["row0"][k]), int(g["row0"][k + 1])
            e0, e1 = int(prow[r0]), int(prow[r1])
            assert 0 < e1 - e0 <= 64
            mask = sum(1 << int(prow[j] - e0) for j in range(r0, r1))
            assert int(g["starts"][k]) == mask
            assert int(g["term0"][k]) == toff[e0]
            assert int(g["tmax"][k]) == int(rt["tcount"][e0:e1].max())
            assert int(g["nmax"][k]) == int(np.diff(prow[r0:r1 + 1]).max())
            # no group could have taken the next row as well
            if r1 < Nr:
                assert prow[r1 + 1] - e0 > 64
        assert int(g["term0"][-1]) == toff[-1]
        # the diagonal carries no terms; slots stay in their row
        rows = np.repeat(np.arange(Nr), np.diff(prow))
        assert np.all(rt["tcount"][rt["pcol"] == rows] == 0)
        ent = np.repeat(np.arange(len(rt["tcount"])), rt["tcount"].astype(np.int64))
        assert np.all(rt["tslot"] < np.diff(prow)[rows[ent]])
