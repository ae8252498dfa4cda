"""A 2D mesh whose centre vertex has more neighbours than a structured grid gives: rings of
``spokes`` vertices around an extracellular centre, one cell on an arc between the first
two rings.  A synthetic input for meshes of high vertex degree (conforming, tagged like the
other cases); it holds no method arithmetic."""
from __future__ import annotations

import numpy as np

from . import Case, physical_params, _initial_concentrations


def fan_case(spokes=40, rings=4, arc=(0, 10), radius_um=1.0, membrane="leak", dt=1e-4, n_steps=2, seed=2099):
    params = physical_params()
    ang = 2.0 * np.pi * np.arange(spokes) / spokes
    xyz = [np.zeros((1, 2))]
    for k in range(1, rings + 1):
        r = radius_um * k / rings
        xyz.append(np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1))
    xyz = np.concatenate(xyz) * 1e-6

    def vid(k, i):              # ring k >= 1, spoke i
        return 1 + (k - 1) * spokes + (i % spokes)

    elem, tag = [], []
    for i in range(spokes):
        elem.append([0, vid(1, i), vid(1, i + 1)])
        tag.append(0)
    for k in range(1, rings):
        for i in range(spokes):
            a, b, c, d = vid(k, i), vid(k, i + 1), vid(k + 1, i + 1), vid(k + 1, i)
            t = 1 if (k == 1 and arc[0] <= i < arc[1]) else 0
            elem += [[a, b, c], [a, c, d]]
            tag += [t, t]
    elem = np.array(elem, np.int32)
    tag = np.array(tag, np.int32)
    n = xyz.shape[0]
    model = {"leak": 0, "hh": 1, "kir": 2}[membrane]
    return Case(name=f"fan{spokes}x{rings}_{membrane}", dim=2, shape=(spokes, rings),
                length_um=(2.0 * radius_um, 2.0 * radius_um), xyz=xyz, elem=elem, tag=tag,
                cell_box=np.zeros((1, 2, 2), np.int64), cell_model=np.array([model], np.int32),
                cell_stim=np.array([1 if membrane == "hh" else 0], np.int32), theta=np.ones(1),
                conc0=_initial_concentrations(params, n, seed), phi0=(params["phi_M0"], 0.0),
                params=params, dt=dt, n_steps=n_steps, pin_vertex=int(vid(rings, spokes // 2)))
