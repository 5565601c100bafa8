"""The inter-grid entry points over a matrix of refinement factors and side
conditions against the oracle (FP64): the integration of the scalar (Eq. 20),
Nu_T (Eq. 23) and two coarse steps of M_t = 2 (Fig. 6: time-blended
refinement, steps, integration), with factors 1 to 5 on each axis (M_z = 5
through the three stage kernels) and periodic or walled x and y."""
import numpy as np
import pytest
import torch

from oracle.intergrid import coarse_step, integrate_scalar, thermal_dissipation
from paper_1805_03426_amd import inputs
from tests.test_gpu_parity import FP64_TOL, host, rel_l2, rel_max
from tests.test_gpu_refine_matrix import FACTORS, SIDES
from tests.test_gpu_walls import WallCase

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("walls", SIDES)
@pytest.mark.parametrize("m", FACTORS)
def test_intergrid_matrix(m, walls):
    print("case intergrid matrix", m, walls, flush=True)
    c = WallCase((7, 5, 4), m, walls, dt=1e-4, n_avg=3)
    th0 = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.1, seed=2)
    lv = [c.coarse_velocity(scale=s) for s in (0.2, 0.25, 0.3)]
    mt = 2
    p1, c1, tc1 = coarse_step(c.g, c.p, 0, mt, th0, th0, *lv[0], *lv[1])
    p2, c2, tc2 = coarse_step(c.g, c.p, mt, mt, p1, c1, *lv[1], *lv[2])
    with c.ctx() as ctx:
        # Eq. 20 and Eq. 23 on the initial scalar
        assert rel_max(host(ctx.integrate_scalar(c.d(th0))), integrate_scalar(c.g, th0)) <= FP64_TOL
        _, got = ctx.thermal_dissipation(c.d(th0))
        want = thermal_dissipation(c.g, c.p, th0)
        for k in ("nu_t", "gx2", "gy2", "gz2"):
            assert abs(got[k] - want[k]) <= FP64_TOL * abs(want["nu_t"]), (k, got[k], want[k])
        # two coarse steps
        dlv = []
        for U, V, W in lv:
            Ul, Vl = c.to_lib(U, V)
            dlv.append([c.d(Ul), c.d(Vl), c.d(W)])
        ring = [c.d(th0), ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell)]
        uvw = (ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_w))
        tc = ctx.empty(ctx.shape_coarse)
        prev, cur = ctx.coarse_step(0, mt, *dlv[0], *dlv[1], uvw, ring, 0, 0, tc)
        assert rel_max(host(ring[cur]), c1) <= FP64_TOL and rel_max(host(ring[prev]), p1) <= FP64_TOL
        assert rel_max(host(tc), tc1) <= FP64_TOL
        prev, cur = ctx.coarse_step(mt, mt, *dlv[1], *dlv[2], uvw, ring, prev, cur, tc)
        assert rel_max(host(ring[cur]), c2) <= FP64_TOL and rel_max(host(ring[prev]), p2) <= FP64_TOL
        assert rel_max(host(tc), tc2) <= FP64_TOL
