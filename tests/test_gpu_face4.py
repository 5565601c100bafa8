"""GPU parity of the step with fourth-order face values of the advected scalar
(uniform or stretched x and y, stretched z), forward and reverse, against the
oracle through the C ABI."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_03426_amd import inputs
from tests.test_gpu_parity import FP32_TOL, FP64_TOL, host, rel_l2, rel_max
from tests.test_gpu_walls import WallCase

pytestmark = pytest.mark.gpu
PERIODIC = (False, False)
SIDES = [(True, False), (False, True), (True, True)]


class Case4(WallCase):
    """WallCase with fourth-order faces: uniform x and y widths, or with
    stretched=True wall-clustered x on a walled axis (random widths on a
    periodic one) and random y widths."""

    def __init__(self, nc, m, walls, z_explicit=0.0, stretched=False, **kw):
        super().__init__(nc, m, walls, **kw)
        if stretched:
            nx = self.g.x.n
            if walls[0]:
                self.xf = inputs.tanh_faces(nx, 1.2)
            else:
                hx = self.rng.uniform(0.6, 1.5, nx)
                self.xf = np.concatenate([[0.0], np.cumsum(hx)]) / hx.sum()
        else:
            self.yf = inputs.uniform_faces(self.g.y.n)
        self.g = O.Grid(self.xf, self.yf, self.zf, m, periodic=(not walls[0], not walls[1], False))
        self.z_explicit = z_explicit
        self.p = dataclasses.replace(self.p, face_order=4, z_explicit=z_explicit)

    def ctx(self):
        from paper_1805_03426_amd.context import Context
        return Context(self.xf, self.yf, self.zf, self.m, self.ra, self.pr, self.dt, n_avg=self.n_avg,
                       bc_bot=self.bc[0], bc_top=self.bc[1], precision=self.precision,
                       side_x="walls" if self.walls[0] else "periodic",
                       side_y="walls" if self.walls[1] else "periodic", z_explicit=self.z_explicit,
                       face_order=4)


def _steps(c, nsteps, tol):
    """Every step from the oracle's own previous levels."""
    u, v, w = c.dense_velocity()
    ul, vl = c.to_lib(u, v)
    prev = cur = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.1, seed=2)
    with c.ctx() as ctx:
        du, dv_, dw = c.d(ul), c.d(vl), c.d(w)
        out = ctx.empty(ctx.shape_cell)
        for n in range(nsteps):
            want = O.scalar_step(c.g, c.p, n, prev, cur, u, v, w)
            ctx.scalar_step(n, c.d(prev), c.d(cur), out, du, dv_, dw)
            got = host(out)
            assert rel_l2(got, want) <= tol, n
            if c.precision == "fp64":
                assert rel_max(got, want) <= tol, n
            prev, cur = cur, want


def _adjoint_vs_oracle(c, N):
    walls = c.walls
    U, V, W = c.coarse_velocity()
    th0 = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.1, seed=2)
    target = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.1, seed=3)
    _, w0, wU, wV, wW = O.rollout_loss_grad(c.g, c.p, th0, U, V, W, N, target)
    Ul, Vl = c.to_lib(U, V)
    with c.ctx() as ctx:
        u, v, w = ctx.interpolate_velocity(c.d(Ul), c.d(Vl), c.d(W))
        th = [c.d(th0)]
        for n in range(N):
            out = ctx.empty(ctx.shape_cell)
            ctx.scalar_step(n, th[n - 1] if n else th[0], th[n], out, u, v, w)
            th.append(out)
        mu = [None] * (N + 1)
        mu[N - 1] = ctx.empty(ctx.shape_cell)
        ctx.adjoint_seed(N - 1, th[N] - c.d(target), mu[N - 1])
        g0 = ctx.empty(ctx.shape_cell)
        for n in range(N - 1, -1, -1):
            out = ctx.empty(ctx.shape_cell) if n > 0 else g0
            ctx.scalar_step_backward(n, mu[n + 1], mu[n], None, out, u, v, w)
            if n > 0:
                mu[n - 1] = out
        gu, gv, gw = torch.zeros_like(u), torch.zeros_like(v), torch.zeros_like(w)
        ctx.velocity_grad(list(range(N)), th[:N], mu[:N], gu, gv, gw)
        gU, gV, gW = (host(t) for t in ctx.interpolate_velocity_backward(gu, gv, gw))
        g0 = host(g0)
    assert rel_max(g0, w0) <= 1e-11
    assert rel_max(gW, wW) <= 1e-11
    if walls[0]:
        assert rel_max(gU[:, :, 1:], wU[:, :, 1:-1]) <= 1e-11
    else:
        assert rel_max(gU, wU) <= 1e-11
    if walls[1]:
        assert rel_max(gV[:, 1:], wV[:, 1:-1]) <= 1e-11
    else:
        assert rel_max(gV, wV) <= 1e-11


def _velocity_grad_vs_oracle(c, walls):
    th = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.2, seed=4)
    mu = c.rng.standard_normal(th.shape)
    n = 2
    tau = O.step_kind(n, c.n_avg, c.dt)[0]
    gu_o, gv_o, gw_o = O.scalar._advection_velocity_transpose(c.g, mu, th, 4)
    with c.ctx() as ctx:
        gu = torch.zeros(ctx.shape_cell, dtype=torch.float64, device="cuda")
        gv, gw = torch.zeros_like(gu), torch.zeros(ctx.shape_w, dtype=torch.float64, device="cuda")
        ctx.velocity_grad([n], [c.d(th)], [c.d(mu)], gu, gv, gw)
        gu, gv, gw = host(gu), host(gv), host(gw)
    want_u = tau * gu_o[:, :, :-1] if walls[0] else tau * gu_o
    want_v = tau * gv_o[:, :-1] if walls[1] else tau * gv_o
    if walls[0]:
        assert np.all(gu[:, :, 0] == 0)
    if walls[1]:
        assert np.all(gv[:, 0] == 0)
    assert rel_max(gu, want_u) <= FP64_TOL
    assert rel_max(gv, want_v) <= FP64_TOL
    assert rel_max(gw, tau * gw_o) <= FP64_TOL


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_step_parity_face4(prec):
    """x ragged against the patch width, odd y rows, 70 z levels (a ragged
    last chunk), Dirichlet bottom and adiabatic top, every step type."""
    print("case face4 step", prec, flush=True)
    c = Case4((35, 9, 35), (2, 1, 2), PERIODIC, precision=prec, bc=("dirichlet", "adiabatic"), n_avg=3,
              gamma=2.0)
    _steps(c, 6, FP64_TOL if prec == "fp64" else FP32_TOL)


@pytest.mark.parametrize("nc,m", [((3, 2, 1), (1, 1, 1)), ((4, 3, 2), (1, 1, 1)), ((5, 3, 3), (1, 1, 1)),
                                  ((3, 3, 160), (5, 1, 4)), ((40, 3, 6), (2, 2, 2))])
def test_step_parity_face4_small_and_large(nc, m):
    """Axes shorter than the four-cell stencil (x of 3 cells, y of 2 rows, one
    to three z levels), the largest z (640 levels: 16 chunks of 40), x wider
    than a patch row."""
    print("case face4 sizes", nc, m, flush=True)
    c = Case4(nc, m, PERIODIC, n_avg=2, gamma=2.5 if nc[2] * m[2] > 3 else 0.0)
    _steps(c, 3, FP64_TOL)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nc", [(1, 1, 1), (4, 1, 3), (2, 5, 2)])
def test_step_parity_face4_single_cells_and_rows(nc, prec):
    """A single cell (every stencil cell is itself), a single y row and two-cell
    x, in both patch shapes (FP64 two-row patches, FP32 one-row)."""
    print("case face4 tiny", nc, prec, flush=True)
    c = Case4(nc, (1, 1, 1), PERIODIC, precision=prec, n_avg=2, gamma=0.0)
    _steps(c, 3, FP64_TOL if prec == "fp64" else FP32_TOL)


@pytest.mark.parametrize("walls", SIDES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_step_parity_face4_with_walls(walls, prec):
    print("case face4 walls", walls, prec, flush=True)
    c = Case4((35, 9, 5), (2, 1, 2), walls, precision=prec, n_avg=3)
    _steps(c, 4, FP64_TOL if prec == "fp64" else FP32_TOL)


@pytest.mark.parametrize("walls", [(True, True)])
def test_step_parity_face4_walled_short_axes(walls):
    """Walled axes of 2 and 3 cells: the two-cell mean and three-cell faces."""
    print("case face4 short walled axes", flush=True)
    c = Case4((3, 2, 4), (1, 1, 1), walls, n_avg=3)
    _steps(c, 3, FP64_TOL)


def test_step_parity_face4_with_explicit_share():
    print("case face4 + explicit z share", flush=True)
    c = Case4((33, 6, 20), (2, 2, 2), PERIODIC, z_explicit=0.5, n_avg=3, gamma=2.0)
    _steps(c, 4, FP64_TOL)


@pytest.mark.parametrize("walls,wz", [(PERIODIC, 0.0), ((True, True), 0.0), (PERIODIC, 0.5)])
def test_adjoint_parity_face4(walls, wz):
    """Reverse sweep through refine + 7 steps (every step type) against the
    oracle's discrete adjoint with fourth-order faces."""
    print("case face4 adjoint", walls, wz, flush=True)
    c = Case4((6, 5, 9), (2, 2, 2), walls, z_explicit=wz, n_avg=3, gamma=1.5)
    _adjoint_vs_oracle(c, 7)


def test_velocity_grad_face4_matches_oracle():
    """The dense-face gradient of one step alone (no refinement in between)."""
    print("case face4 velocity gradient", flush=True)
    c = Case4((9, 6, 7), (2, 2, 2), (True, False), n_avg=3)
    _velocity_grad_vs_oracle(c, (True, False))

STRETCHED_SIDES = [PERIODIC, (True, True), (True, False), (False, True)]


@pytest.mark.parametrize("walls", STRETCHED_SIDES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_step_parity_face4_stretched_xy(walls, prec):
    """Stretched x and y (wall-clustered x beside walls, random widths
    otherwise): the per-face weight tables of both axes, every step type."""
    print("case face4 stretched xy", walls, prec, flush=True)
    c = Case4((35, 9, 12), (2, 1, 2), walls, stretched=True, precision=prec, n_avg=3, dt=2e-4, gamma=1.5)
    _steps(c, 5, FP64_TOL if prec == "fp64" else FP32_TOL)


@pytest.mark.parametrize("nc,walls", [((3, 2, 3), PERIODIC), ((1, 3, 3), PERIODIC), ((3, 4, 3), (True, True))])
def test_step_parity_face4_stretched_short_axes(nc, walls):
    """Stretched axes shorter than the stencil: a periodic stencil that wraps
    onto itself with the period added, and walled axes of three and four cells."""
    print("case face4 stretched short axes", nc, walls, flush=True)
    c = Case4(nc, (1, 1, 1), walls, stretched=True, n_avg=2, dt=2e-4)
    _steps(c, 3, FP64_TOL)


@pytest.mark.parametrize("walls,wz", [(PERIODIC, 0.0), ((True, True), 0.0), ((True, False), 0.5)])
def test_adjoint_parity_face4_stretched(walls, wz):
    """Reverse sweep through refine + 7 steps on stretched x and y against the
    oracle's discrete adjoint (the transposed faces use the weights of the
    faces one beyond each side)."""
    print("case face4 stretched adjoint", walls, wz, flush=True)
    c = Case4((6, 5, 9), (2, 2, 2), walls, z_explicit=wz, stretched=True, n_avg=3, gamma=1.5, dt=5e-4)
    _adjoint_vs_oracle(c, 7)


def test_velocity_grad_face4_stretched_matches_oracle():
    print("case face4 stretched velocity gradient", flush=True)
    for walls in [(True, False), (False, True), PERIODIC]:
        c = Case4((9, 6, 7), (2, 2, 2), walls, stretched=True, n_avg=3, dt=5e-4)
        _velocity_grad_vs_oracle(c, walls)
