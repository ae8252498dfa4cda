"""GPU tests of the AMG levels below the finest replayed as one HIP graph
(knp_amg_opts.coarse_graph): every replay gives the V-cycle of the kernels launched one by
one, bit for bit (the same kernels on the same buffers), with eager work and host
synchronisations between the replays, after a new setup too, and in whole solves.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from knp_inputs import config_case  # noqa: E402
from paper_2403_04491_amd import KnpSolver, amg_opts, solve_opts  # noqa: E402
from paper_2403_04491_amd.simulate import AMG_BY_GAUGE  # noqa: E402

DEV = torch.device("cuda", 0)


def pair(precision, gauge=0, **kw):
    case = config_case(3, per_pitch=4)
    extra = AMG_BY_GAUGE[gauge]
    sg = KnpSolver(case, gauge=gauge, amg=amg_opts(precision=precision, coarse_graph=1, **extra, **kw))
    se = KnpSolver(case, gauge=gauge, amg=amg_opts(precision=precision, coarse_graph=0, **extra, **kw))
    return sg, se


@pytest.mark.parametrize("precision", [0, 1])
def test_vcycle_replays_equal_launches(precision):
    print(f"[coarse graph] V-cycle replays, precision {precision}", flush=True)
    sg, se = pair(precision)
    for s in (sg, se):
        s.assemble()
    N = sg.info.N
    rng = np.random.default_rng(17)
    for k in range(5):
        x = torch.as_tensor(rng.standard_normal(N), dtype=torch.float64, device=DEV)
        yg = torch.empty_like(x)
        ye = torch.empty_like(x)
        sg.ctx.apply(1, x, yg)
        # eager work and synchronisations between the replays
        w = torch.empty_like(x)
        sg.ctx.apply(0, x, w)
        torch.cuda.synchronize()
        se.ctx.apply(1, x, ye)
        assert torch.equal(yg, ye), (k, float((yg - ye).abs().max()))
        assert float(yg.abs().max()) > 0.0
    # a new setup drops the graph; the next V-cycle captures the new hierarchy's
    for s in (sg, se):
        s.ctx.amg_setup(amg_opts(precision=precision, coarse_graph=1 if s is sg else 0, **AMG_BY_GAUGE[1]))
    for k in range(3):
        x = torch.as_tensor(rng.standard_normal(N), dtype=torch.float64, device=DEV)
        yg = torch.empty_like(x)
        ye = torch.empty_like(x)
        sg.ctx.apply(1, x, yg)
        se.ctx.apply(1, x, ye)
        assert torch.equal(yg, ye), ("after setup", k)


@pytest.mark.parametrize("precision,gauge", [(1, 1), (0, 0)])
def test_solves_with_the_graph_equal_solves_without(precision, gauge):
    print(f"[coarse graph] steps, precision {precision} gauge {gauge}", flush=True)
    sg, se = pair(precision, gauge)
    for n in range(3):
        ig = sg.step()
        ie = se.step()
        assert ig.its == ie.its and ig.rel_res == ie.rel_res, (n, ig.its, ie.its)
        assert torch.equal(sg.u, se.u), n
