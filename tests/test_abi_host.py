"""Host-side checks of libknp without a GPU: exported symbols and the mesh/DOF/
pattern logic of knp_mesh_upload (host-only context), bit-exact against the
oracle's independent construction, plus argument errors."""
import ctypes
import os
import re

import numpy as np
import pytest

from knp_inputs import config_case, lattice_case, model_a_case
from oracle.mesh import build_layout, structural_pattern
from paper_2403_04491_amd import knp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "knp.h")).read()
    declared = set(re.findall(r"\b(knp_[a-z0-9_]+)\s*\(", header))
    assert declared == set(knp.EXPORTS)
    lib = ctypes.CDLL(knp._LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


CASES = {
    "cfg1": lambda: config_case(1),
    "modelA3d_nx8_hh": lambda: model_a_case(3, 8, "hh", 5e-5, 1),
    "lattice4_pp5": lambda: config_case(3, per_pitch=5),
    "lattice2_pp6_theta": lambda: config_case(4, per_pitch=6),
    "fan40": lambda: __import__("knp_inputs.fan", fromlist=["fan_case"]).fan_case(),
}


@pytest.mark.parametrize("name", list(CASES))
def test_host_layout_bit_exact(name):
    case = CASES[name]()
    ctx = knp.Context(-1)
    info = ctx.mesh_upload(case.dim, case.xyz, case.elem, case.tag, case.pin_vertex)
    rowptr, colidx, dofv = ctx.get_layout()
    lay = build_layout(case)
    rp, ci = structural_pattern(case, lay)
    assert (info.N_i, info.N_e, info.N) == (lay.N_r[0], lay.N_r[1], lay.N)
    assert info.n_gamma == len(lay.gamma) and info.n_facets == len(lay.facets)
    assert info.n_cells == case.n_cells
    assert info.pin_dof == lay.pin_dof
    assert np.array_equal(rowptr, rp)
    assert np.array_equal(colidx, ci)
    exp_v = np.concatenate([np.tile(lay.verts[0], 4), np.tile(lay.verts[1], 4)])
    assert np.array_equal(dofv, exp_v)
    assert np.array_equal(ctx.get_gamma(), lay.gamma)
    # nnz(P_0) = 4 sum_r P_r
    from oracle.mesh import region_pairs
    assert info.nnz_P0 == 4 * sum(len(region_pairs(case, lay, r)) for r in (0, 1))


@pytest.mark.parametrize("d,nx,membrane", [(2, 4, "leak"), (2, 8, "hh"), (3, 4, "hh")])
def test_host_layout_bit_exact_p2(d, nx, membrane):
    """Quadratic elements: node numbering (edges lexicographic after the vertices), DOF
    numbering, membrane nodes and the structural pattern equal the oracle's P2 layout."""
    from oracle.p2 import p2_case
    base = model_a_case(d, nx, membrane, 1e-4, 1)
    case = p2_case(base)
    ctx = knp.Context(-1)
    info = ctx.mesh_upload(base.dim, base.xyz, base.elem, base.tag, base.pin_vertex, order=2)
    rowptr, colidx, dofv = ctx.get_layout()
    lay = build_layout(case)
    rp, ci = structural_pattern(case, lay)
    assert info.n_vert == case.n_vert
    assert (info.N_i, info.N_e, info.N) == (lay.N_r[0], lay.N_r[1], lay.N)
    assert info.n_gamma == len(lay.gamma) and info.n_facets == len(lay.facets)
    assert info.pin_dof == lay.pin_dof
    assert np.array_equal(rowptr, rp)
    assert np.array_equal(colidx, ci)
    exp_v = np.concatenate([np.tile(lay.verts[0], 4), np.tile(lay.verts[1], 4)])
    assert np.array_equal(dofv, exp_v)
    assert np.array_equal(ctx.get_gamma(), lay.gamma)
    assert np.array_equal(ctx.get_edges(), case.edges)


def _expect_arg_error(case, tag=None, pin=0, elem=None):
    ctx = knp.Context(-1)
    with pytest.raises(knp.KnpError) as ei:
        ctx.mesh_upload(case.dim, case.xyz, case.elem if elem is None else elem,
                        case.tag if tag is None else tag, pin)
    assert ei.value.status == 1
    return str(ei.value)


def test_mesh_errors():
    case = model_a_case(2, 8)
    # pin on the membrane
    lay = build_layout(case)
    assert "pin" in _expect_arg_error(case, pin=int(lay.gamma[0]))
    # vertex index out of range
    bad = case.elem.copy()
    bad[0, 0] = case.n_vert + 5
    assert "range" in _expect_arg_error(case, elem=bad)
    # a cell touching the outer boundary
    tag = case.tag.copy()
    tag[-2:] = 1
    assert "boundary" in _expect_arg_error(case, tag=tag)
    # two cells sharing vertices
    tag = case.tag.copy()
    tag[tag == 1] = 1
    first_cell_elem = np.nonzero(tag == 1)[0][0]
    tag[first_cell_elem] = 2
    assert "cells" in _expect_arg_error(case, tag=tag)
    # gap in cell numbering
    tag = case.tag.copy()
    tag[tag == 1] = 2
    assert "tags" in _expect_arg_error(case, tag=tag)


def test_host_only_context_rejects_device_calls():
    case = config_case(1)
    ctx = knp.Context(-1)
    ctx.mesh_upload(case.dim, case.xyz, case.elem, case.tag, 0)
    with pytest.raises(knp.KnpError) as ei:
        ctx.set_params(case.params, case.cell_model, case.cell_stim)
    assert ei.value.status == 2


def test_one_hip_runtime_in_process():
    """The binding loads libknp after torch, so both use torch's HIP runtime."""
    import paper_2403_04491_amd  # noqa: F401
    maps = open("/proc/self/maps").read().splitlines()
    hip = {line.split()[-1] for line in maps if "libamdhip64" in line}
    assert len(hip) == 1, hip


def test_failed_create_reports_reason():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("needs a host without a visible GPU")
    lib = knp.lib()
    c = ctypes.c_void_p()
    st = lib.knp_create(ctypes.byref(c), 0, None)
    assert knp.STATUS[st] == "KNP_E_HIP" and not c.value
    msg = lib.knp_last_error(None).decode()
    assert "hipGetDeviceCount" in msg or "visible" in msg, msg


def test_ctypes_structs_match_the_header(tmp_path):
    """Every struct of the binding has the header's size and field offsets, as the C
    compiler lays them out (a field added on one side only fails here)."""
    import ctypes
    import shutil
    import subprocess
    from pathlib import Path
    from paper_2403_04491_amd import knp as K
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    pairs = {"knp_mesh_info": K.MeshInfo, "knp_params": K.Params, "knp_amg_opts": K.AmgOpts,
             "knp_solve_opts": K.SolveOpts, "knp_solve_info": K.SolveInfo, "knp_timer": K.Timer}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "knp.h"', "int main(void) {"]
    for cname, cls in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    inc = Path(__file__).resolve().parents[1] / "include"
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", f"-I{inc}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, cls in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
