"""The step over a matrix of method options against the oracle: side walls in
x and/or y, second- or fourth-order faces, an explicit z share of 0 or 1/2,
uniform or stretched x and y, both precisions; ragged x (70 cells), odd y
(9 rows), 36 z levels, Dirichlet bottom and adiabatic top, every step type
(start-up, leapfrog, averaging) from the oracle's own previous levels."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_1805_03426_amd import inputs
from tests.test_gpu_parity import FP32_TOL, FP64_TOL, host, rel_l2, rel_max
from tests.test_gpu_walls import WallCase

pytestmark = pytest.mark.gpu

SIDES = [(False, False), (True, False), (False, True), (True, True)]


class OptCase(WallCase):
    def __init__(self, walls, order, wz, stretched, prec):
        super().__init__((35, 9, 18), (2, 1, 2), walls, precision=prec, bc=("dirichlet", "adiabatic"), n_avg=3,
                         dt=2e-4, gamma=2.0)
        if not stretched:
            self.yf = inputs.uniform_faces(self.g.y.n)
        elif walls[0]:
            self.xf = inputs.tanh_faces(self.g.x.n, 1.2)
        self.g = O.Grid(self.xf, self.yf, self.zf, self.m, periodic=(not walls[0], not walls[1], False))
        self.order, self.wz = order, wz
        self.p = dataclasses.replace(self.p, face_order=order, z_explicit=wz)

    def ctx(self):
        from paper_1805_03426_amd.context import Context
        return Context(self.xf, self.yf, self.zf, self.m, self.ra, self.pr, self.dt, n_avg=self.n_avg,
                       bc_bot=self.bc[0], bc_top=self.bc[1], precision=self.precision,
                       side_x="walls" if self.walls[0] else "periodic",
                       side_y="walls" if self.walls[1] else "periodic", z_explicit=self.wz,
                       face_order=self.order)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("stretched", [False, True])
@pytest.mark.parametrize("wz", [0.0, 0.5])
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("walls", SIDES)
def test_step_matrix(walls, order, wz, stretched, prec):
    print("case step matrix", walls, order, wz, stretched, prec, flush=True)
    c = OptCase(walls, order, wz, stretched, prec)
    u, v, w = c.dense_velocity()
    ul, vl = c.to_lib(u, v)
    prev = cur = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.1, seed=2)
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    with c.ctx() as ctx:
        du, dv_, dw = c.d(ul), c.d(vl), c.d(w)
        out = ctx.empty(ctx.shape_cell)
        for n in range(4):
            want = O.scalar_step(c.g, c.p, n, prev, cur, u, v, w)
            ctx.scalar_step(n, c.d(prev), c.d(cur), out, du, dv_, dw)
            got = host(out)
            assert np.isfinite(got).all(), n
            assert rel_l2(got, want) <= tol, n
            if prec == "fp64":
                assert rel_max(got, want) <= tol, n
            prev, cur = cur, want


class SmallOptCase(OptCase):
    """The same options on a grid small enough for the oracle's discrete adjoint."""

    def __init__(self, walls, order, wz, stretched):
        WallCase.__init__(self, (6, 5, 9), (2, 2, 2), walls, n_avg=3, gamma=1.5, dt=5e-4)
        if not stretched:
            self.yf = inputs.uniform_faces(self.g.y.n)
        elif walls[0]:
            self.xf = inputs.tanh_faces(self.g.x.n, 1.2)
        self.g = O.Grid(self.xf, self.yf, self.zf, self.m, periodic=(not walls[0], not walls[1], False))
        self.order, self.wz = order, wz
        self.p = dataclasses.replace(self.p, face_order=order, z_explicit=wz)


@pytest.mark.parametrize("stretched", [False, True])
@pytest.mark.parametrize("wz", [0.0, 0.5])
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("walls", SIDES)
def test_adjoint_matrix(walls, order, wz, stretched):
    """Refine + 7 steps and the hand-written reverse sweep (seed, reverse steps,
    velocity gradient, transposed refinement) against the oracle's discrete
    adjoint, FP64, every combination of the options."""
    from tests.test_gpu_face4 import _adjoint_vs_oracle
    print("case adjoint matrix", walls, order, wz, stretched, flush=True)
    _adjoint_vs_oracle(SmallOptCase(walls, order, wz, stretched), 7)
