"""Seeded synthetic inputs for the KNP-EMI time-step solve.

This module only *produces inputs*: a structured simplicial mesh with subdomain
tags, per-vertex initial concentrations, per-cell membrane choices, the physical
parameter table and the solver settings.  It holds none of the method's
arithmetic (no degree-of-freedom numbering, no assembly, no membrane model), so
that both the CPU oracle and the GPU library can consume the same case without
sharing any code that computes the method.

Geometry follows the paper's Model A (Sec. "Model A"): the unit square/cube with
one axis-aligned cell, a uniform grid with N_x intervals per side, 2 triangles per
square (diagonal from the lower-left to the upper-right corner, as drawn in the
Model A geometry figure) or 6 tetrahedra per cube.  The 6-tetrahedra split is the
Kuhn (Freudenthal) split, one simplex per axis permutation.  Larger workloads are
lattices of jittered box cells on the same kind of grid; they stand in for the
paper's image-based Models B-D, whose meshes are not available.

Units are SI throughout: coordinates in metres (grid built in micrometres and
scaled by 1e-6), concentrations in mol/m^3 (= mM), potentials in volts.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Case", "physical_params", "model_a_case", "model_a_evolution_case", "lattice_case", "config_case",
           "structured_simplex_mesh", "CONFIG_NAMES", "MEMBRANE_CODES"]


def physical_params() -> dict:
    """Physical parameters and initial values (Table "Physical parameters").

    Values are transcribed in SI units.  The membrane capacitance is printed with
    unit "F"; it is a capacitance per area, 0.02 F/m^2.  Potentials printed in mV
    are stored in volts.  The ion order is (Na+, K+, Cl-) everywhere.
    """
    return {
        "R": 8.314,            # J/(K mol)
        "T": 300.0,            # K
        "F": 9.648e4,          # C/mol
        "C_m": 0.02,           # F/m^2
        "z": [1.0, 1.0, -1.0],
        "D": [1.33e-9, 1.96e-9, 2.03e-9],   # m^2/s, same in both regions
        "g_leak": [1.0, 4.0, 0.0],          # S/m^2
        "gbar_Na": 1200.0,     # S/m^2
        "gbar_K": 360.0,       # S/m^2
        "g_stim_bar": 40.0,    # S/m^2
        "stim_a": 0.002,       # s
        "stim_tau": 0.010,     # s (period between stimuli, Model A)
        "phi_rest": -0.065,    # V
        "phi_M0": -0.06774,    # V
        "gates0": [0.276, 0.0379, 0.688],   # (n0, m0, h0)
        "conc_i0": [12.0, 125.0, 137.0],    # mol/m^3
        "conc_e0": [100.0, 4.0, 104.0],     # mol/m^3
        "n_ode": 25,
        "rho_pump": 1.115e-6,  # mol/(m^2 s), Na/K pump maximum rate
        "P_Na": 10.0,          # mol/m^3, ICS Na+ pump threshold
        "P_K": 1.5,            # mol/m^3, ECS K+ pump threshold
    }


@dataclass
class Case:
    """One synthetic workload: mesh, tags, initial state, parameters, settings."""
    name: str
    dim: int
    shape: tuple                 # intervals per axis
    length_um: tuple             # domain side lengths in micrometres
    xyz: np.ndarray              # float64 [n_vert, dim], metres
    elem: np.ndarray             # int32 [n_elem, dim+1]
    tag: np.ndarray              # int32 [n_elem]; 0 = extracellular, c >= 1 = cell c
    cell_box: np.ndarray         # int64 [n_cells, 2, dim]: grid-index lo, hi per axis
    cell_model: np.ndarray       # int32 [n_cells]; 0 = passive leak, 1 = Hodgkin-Huxley, 2 = Kir-Na/K
    cell_stim: np.ndarray        # int32 [n_cells]; 1 = periodic Na stimulus applies
    theta: np.ndarray            # float64 [n_cells]; multiplies all leak conductances of cell
    conc0: np.ndarray            # float64 [2, 3, n_vert]; region (i, e) x ion x vertex
    phi0: tuple                  # (phi_i^0, phi_e^0) in volts
    params: dict
    dt: float
    n_steps: int
    pin_vertex: int = 0
    probes: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    seeds: dict = field(default_factory=dict)

    @property
    def n_vert(self) -> int:
        return self.xyz.shape[0]

    @property
    def n_elem(self) -> int:
        return self.elem.shape[0]

    @property
    def n_cells(self) -> int:
        return int(self.cell_box.shape[0])


def structured_simplex_mesh(shape, length_um):
    """Uniform grid split into simplices.

    Vertex id  v = i + (n_x+1) * (j + (n_y+1) * k), x fastest.
    Cubes are enumerated with the last axis outermost and x innermost; each cube
    is split into one simplex per axis permutation sigma, in lexicographic order,
    with vertices v0, v0+e_s1, v0+e_s1+e_s2, (v0+1,1,1).  In 2D this yields the
    lower-left to upper-right diagonal.
    Returns (xyz [m], elem int32 [n_cube * d!, d+1]); element e lies in cube e // d!.
    """
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    nv = [s + 1 for s in shape]
    h = [float(L) / s for L, s in zip(length_um, shape)]
    axes = [np.arange(n, dtype=np.float64) * hh for n, hh in zip(nv, h)]
    grids = np.meshgrid(*axes, indexing="ij")          # index order (x, y[, z])
    # flatten with x fastest -> transpose to (z, y, x) order before ravel
    xyz = np.stack([g.transpose(tuple(reversed(range(dim)))).ravel() for g in grids], axis=1)
    xyz = xyz * 1e-6

    strides = [1]
    for a in range(1, dim):
        strides.append(strides[-1] * nv[a - 1])
    # lower-corner vertex of every cube, cubes in (z, y, x) order with x fastest
    v0 = np.zeros([shape[a] for a in reversed(range(dim))], dtype=np.int64)
    for a in range(dim):
        idx = np.arange(shape[a], dtype=np.int64) * strides[a]
        bshape = [1] * dim
        bshape[dim - 1 - a] = shape[a]
        v0 = v0 + idx.reshape(bshape)
    v0 = v0.ravel()
    perms = list(itertools.permutations(range(dim)))
    elem = np.empty((v0.shape[0], len(perms), dim + 1), dtype=np.int32)
    for p, sigma in enumerate(perms):
        cur = v0.copy()
        elem[:, p, 0] = cur
        for q, ax in enumerate(sigma):
            cur = cur + strides[ax]
            elem[:, p, q + 1] = cur
    return xyz, elem.reshape(-1, dim + 1)


def _tags_from_boxes(shape, boxes):
    """Element belongs to cell c when its cube lies inside box c (grid indices)."""
    dim = len(shape)
    cube = np.zeros([shape[a] for a in reversed(range(dim))], dtype=np.int32)   # (z, y, x)
    for c, (lo, hi) in enumerate(boxes):
        sl = tuple(slice(int(lo[a]), int(hi[a])) for a in reversed(range(dim)))
        if np.any(cube[sl] != 0):
            raise ValueError("cells overlap")
        cube[sl] = c + 1
    n_perm = 2 if dim == 2 else 6
    return np.repeat(cube.ravel(), n_perm)


def _initial_concentrations(params, n_vert, seed, noise=0.01):
    """Per-vertex initial concentrations for both regions.

    Na and K are the table values times (1 + U(-noise, noise)); Cl = Na + K keeps
    every node electroneutral.  Draws: numpy PCG64(seed), one array of shape
    (region i/e, ion Na/K, vertex) for *every* grid vertex, so that the draw
    does not depend on which vertices a region owns.  noise = 0 gives the
    table's uniform values.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(-noise, noise, size=(2, 2, n_vert))
    conc = np.empty((2, 3, n_vert), dtype=np.float64)
    for r, base in enumerate((params["conc_i0"], params["conc_e0"])):
        conc[r, 0] = base[0] * (1.0 + u[r, 0])
        conc[r, 1] = base[1] * (1.0 + u[r, 1])
        conc[r, 2] = conc[r, 0] + conc[r, 1]
    return conc


def _strict_ecs_vertices(shape, boxes):
    """Vertices that lie outside every closed cell box (so not on any membrane)."""
    dim = len(shape)
    nv = [s + 1 for s in shape]
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in nv], indexing="ij"), axis=-1)
    idx = idx.transpose(tuple(reversed(range(dim))) + (dim,)).reshape(-1, dim)
    ok = np.ones(idx.shape[0], dtype=bool)
    for lo, hi in boxes:
        ok &= ~np.all((idx >= lo) & (idx <= hi), axis=1)
    return np.nonzero(ok)[0]


MEMBRANE_CODES = {"leak": 0, "hh": 1, "kir": 2}


def model_a_case(dim=2, nx=32, membrane="leak", dt=1e-4, n_steps=10, cfg_id=1,
                 stim=None, name=None, noise=0.01):
    """Model A: [0,1]^d um with one cell [0.25,0.75]^d um (Sec. "Model A").

    membrane: "leak", "hh" or "kir" (the Kir-Na/K passive model); the stimulus
    defaults to on for "hh" only.  noise: relative amplitude of the per-vertex
    perturbation of the initial Na and K concentrations (0 = the table's values).
    """
    if nx % 4 != 0:
        raise ValueError("nx must be divisible by 4 so the cell faces lie on grid planes")
    params = physical_params()
    shape = (nx,) * dim
    xyz, elem = structured_simplex_mesh(shape, (1.0,) * dim)
    boxes = np.array([[[nx // 4] * dim, [3 * nx // 4] * dim]], dtype=np.int64)
    tag = _tags_from_boxes(shape, boxes)
    hh = membrane == "hh"
    if stim is None:
        stim = hh
    seeds = {"conc": 2000 + cfg_id}
    return Case(
        name=name or f"modelA_{dim}d_nx{nx}_{membrane}", dim=dim, shape=shape,
        length_um=(1.0,) * dim, xyz=xyz, elem=elem, tag=tag, cell_box=boxes,
        cell_model=np.array([MEMBRANE_CODES[membrane]], np.int32),
        cell_stim=np.array([1 if stim else 0], np.int32),
        theta=np.ones(1), conc0=_initial_concentrations(params, xyz.shape[0], seeds["conc"], noise),
        phi0=(params["phi_M0"], 0.0), params=params, dt=dt, n_steps=n_steps, seeds=seeds)


def model_a_evolution_case(nx=512, membrane="hh", n_steps=300, dt=1e-4, dim=2):
    """Model A's time evolution (Sec. "Model A" and its iteration-count figure): the
    2D unit square at N_x = 512 (N = 1,056,772 for p = 1), the periodic Na stimulus
    on the whole membrane for every membrane model, the table's uniform initial
    values, N_t = 300 steps of 0.1 ms."""
    return model_a_case(dim, nx, membrane, dt, n_steps, cfg_id=6, stim=True, noise=0.0,
                        name=f"modelA_evolution_{dim}d_nx{nx}_{membrane}")


def lattice_case(cells=(4, 4, 4), pitch_um=(1.0, 1.0, 1.0), per_pitch=33, n_hh=16,
                 dt=5e-5, n_steps=50, cfg_id=3, theta_range=None, n_probes=0,
                 name=None, passive="leak"):
    """Box containing a lattice of jittered box cells on a structured tet grid.

    Per cell (lexicographic lattice order, x fastest), with PCG64(1000+cfg): a
    size factor U(0.95, 1.05) on 0.6*pitch, then per-axis centre offsets
    U(-0.05, 0.05)*pitch.  Faces are snapped to the nearest grid plane and at
    least one interval of extracellular space is kept between cells and from the
    outer boundary.  HH cells: a PCG64(3000+cfg) choice of exactly n_hh cells
    (stimulated); the rest use the passive model named by `passive` ("leak" or
    "kir", the Kir-Na/K model).  Leak factors theta:
    log-uniform in theta_range from PCG64(4000+cfg) (or all 1).  Probes: the same
    generator then picks n_probes distinct vertices strictly in the ECS, not the
    pinned vertex 0.
    """
    params = physical_params()
    dim = len(cells)
    per_axis = [int(round(per_pitch * p / min(pitch_um))) for p in pitch_um]
    shape = tuple(c * n for c, n in zip(cells, per_axis))
    length = tuple(c * p for c, p in zip(cells, pitch_um))
    h = [L / s for L, s in zip(length, shape)]
    xyz, elem = structured_simplex_mesh(shape, length)

    rng_geo = np.random.Generator(np.random.PCG64(1000 + cfg_id))
    lattice = np.stack(np.meshgrid(*[np.arange(c) for c in cells], indexing="ij"), axis=-1)
    lattice = lattice.transpose(tuple(reversed(range(dim))) + (dim,)).reshape(-1, dim)
    boxes = np.zeros((lattice.shape[0], 2, dim), dtype=np.int64)
    for c, li in enumerate(lattice):
        s = rng_geo.uniform(0.95, 1.05)
        off = rng_geo.uniform(-0.05, 0.05, size=dim)
        for a in range(dim):
            centre = (li[a] + 0.5) * pitch_um[a] + off[a] * pitch_um[a]
            half = 0.5 * 0.6 * pitch_um[a] * s
            boxes[c, 0, a] = int(np.floor((centre - half) / h[a] + 0.5))
            boxes[c, 1, a] = int(np.floor((centre + half) / h[a] + 0.5))
    for c in range(boxes.shape[0]):
        if np.any(boxes[c, 0] < 1) or np.any(boxes[c, 1] > np.array(shape) - 1):
            raise ValueError("cell touches the outer boundary; increase per_pitch")
        if np.any(boxes[c, 1] - boxes[c, 0] < 1):
            raise ValueError("degenerate cell; increase per_pitch")
    for c1 in range(boxes.shape[0]):
        for c2 in range(c1 + 1, boxes.shape[0]):
            sep = np.maximum(boxes[c1, 0] - boxes[c2, 1], boxes[c2, 0] - boxes[c1, 1])
            if np.max(sep) < 1:
                raise ValueError("cells closer than one interval; increase per_pitch")
    tag = _tags_from_boxes(shape, boxes)

    n_cells = boxes.shape[0]
    rng_mem = np.random.Generator(np.random.PCG64(3000 + cfg_id))
    model = np.full(n_cells, MEMBRANE_CODES[passive], np.int32)
    if n_hh:
        model[rng_mem.choice(n_cells, size=n_hh, replace=False)] = 1
    rng_par = np.random.Generator(np.random.PCG64(4000 + cfg_id))
    if theta_range is not None:
        lo, hi = theta_range
        theta = np.exp(rng_par.uniform(np.log(lo), np.log(hi), size=n_cells))
    else:
        theta = np.ones(n_cells)
    probes = np.zeros(0, np.int64)
    if n_probes:
        cand = _strict_ecs_vertices(shape, boxes)
        cand = cand[cand != 0]
        probes = np.sort(rng_par.choice(cand, size=n_probes, replace=False)).astype(np.int64)
    seeds = {"geometry": 1000 + cfg_id, "conc": 2000 + cfg_id, "membrane": 3000 + cfg_id,
             "params": 4000 + cfg_id}
    return Case(
        name=name or f"lattice_{'x'.join(map(str, cells))}_pp{per_pitch}", dim=dim,
        shape=shape, length_um=length, xyz=xyz, elem=elem, tag=tag, cell_box=boxes,
        cell_model=model, cell_stim=(model == 1).astype(np.int32), theta=theta,
        conc0=_initial_concentrations(params, xyz.shape[0], 2000 + cfg_id),
        phi0=(params["phi_M0"], 0.0), params=params, dt=dt, n_steps=n_steps,
        probes=probes, seeds=seeds)


CONFIG_NAMES = {
    1: "2D unit square, one cell, 32x32 triangles, passive leak, dt 0.1 ms, 10 steps",
    2: "3D unit cube, one cell, 32^3 x 6 tets, HH + stimulus, dt 0.05 ms, 100 steps",
    3: "3D 4x4x4 lattice of jittered box cells, 132^3 x 6 tets (~1e7 unknowns), 16 HH cells, 50 steps",
    4: "3D 2x2x2 lattice, 78^3 x 6 tets (~2e6 unknowns), leak with per-cell theta, 16 probes, 40 steps",
    5: "3D 8x8x8 lattice of 4:1:1 cells, 736x184x184 x 6 tets (~1e8 unknowns), leak, 10 steps",
}


def config_case(cfg: int, per_pitch=None, n_steps=None, passive="leak"):
    """The five workloads; per_pitch shrinks configs 3-5 to reduced members.  passive
    ("leak" or "kir") is the membrane model of the lattice's non-HH cells (config 3:
    "kir" gives the HH + Kir-Na/K mix of the paper's Model D on the same geometry)."""
    if cfg == 1:
        c = model_a_case(2, 32, "leak", 1e-4, 10, cfg_id=1, name="cfg1")
    elif cfg == 2:
        c = model_a_case(3, 32, "hh", 5e-5, 100, cfg_id=2, name="cfg2")
    elif cfg == 3:
        pp = per_pitch or 33
        c = lattice_case((4, 4, 4), (1.0, 1.0, 1.0), pp, n_hh=16, dt=5e-5, n_steps=50,
                         cfg_id=3, name=f"cfg3_pp{pp}" + ("" if passive == "leak" else f"_{passive}"),
                         passive=passive)
    elif cfg == 4:
        pp = per_pitch or 39
        c = lattice_case((2, 2, 2), (1.0, 1.0, 1.0), pp, n_hh=0, dt=5e-5, n_steps=40,
                         cfg_id=4, theta_range=(0.5, 2.0), n_probes=16, name=f"cfg4_pp{pp}")
    elif cfg == 5:
        pp = per_pitch or 23
        c = lattice_case((8, 8, 8), (4.0, 1.0, 1.0), pp, n_hh=0, dt=5e-5, n_steps=10,
                         cfg_id=5, name=f"cfg5_pp{pp}")
    else:
        raise ValueError(f"unknown config {cfg}")
    if n_steps is not None:
        c.n_steps = n_steps
    return c
