"""GPU parity of the step with a share w of the z diffusion explicit on the
lagged level (w = 1/2: Crank-Nicolson across the step's time span), forward
and reverse, against the oracle through the C ABI."""
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


class ZCase(WallCase):
    def __init__(self, nc, m, walls, z_explicit, **kw):
        super().__init__(nc, m, walls, **kw)
        self.z_explicit = z_explicit
        self.p = dataclasses.replace(self.p, z_explicit=z_explicit)

    def ctx(self):
        from paper_1805_03426_amd.context import Context
        return Context(self.xf, self.yf, self.zf, self.m, self.ra, self.pr, self.dt, n_avg=self.n_avg,
                       bc_bot=self.bc[0], bc_top=self.bc[1], precision=self.precision,
                       side_x="walls" if self.walls[0] else "periodic",
                       side_y="walls" if self.walls[1] else "periodic", z_explicit=self.z_explicit)


def _steps(c, nsteps, tol):
    """Every step from the oracle's own previous levels; all three step types."""
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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("wz", [0.5, 0.2])
def test_step_parity_explicit_share(prec, wz):
    """Several z chunks with a ragged last one (nz = 70), x ragged against the
    patch width, Dirichlet bottom and adiabatic top, N_p = 3."""
    print("case zweight step", prec, wz, flush=True)
    c = ZCase((35, 9, 35), (2, 1, 2), PERIODIC, wz, precision=prec, bc=("dirichlet", "adiabatic"),
              n_avg=3, gamma=2.0)
    _steps(c, 6, FP64_TOL if prec == "fp64" else FP32_TOL)


@pytest.mark.parametrize("nc,m", [((4, 3, 1), (2, 2, 1)), ((3, 3, 160), (5, 1, 4)), ((6, 5, 12), (2, 2, 2))])
def test_step_parity_explicit_share_z_extremes(nc, m):
    """One z level, the largest z (640 levels: 16 chunks of 40), a short column."""
    print("case zweight z extremes", nc, m, flush=True)
    c = ZCase(nc, m, PERIODIC, 0.5, n_avg=2, gamma=2.5 if nc[2] > 1 else 0.0)
    _steps(c, 3, FP64_TOL)


@pytest.mark.parametrize("walls", [(True, False), (True, True)])
def test_step_parity_explicit_share_with_walls(walls):
    print("case zweight walls", walls, flush=True)
    c = ZCase((35, 9, 5), (2, 1, 2), walls, 0.5, n_avg=3)
    _steps(c, 4, FP64_TOL)


def test_conduction_fixed_point_with_explicit_share():
    print("case zweight conduction", flush=True)
    c = ZCase((8, 6, 20), (2, 2, 2), PERIODIC, 0.5, n_avg=3, gamma=2.0)
    th = np.broadcast_to(1.0 - c.g.z.c[:, None, None], c.g.shape).copy()
    with c.ctx() as ctx:
        ring = [c.d(th)] + [ctx.empty(ctx.shape_cell) for _ in range(3)]
        u, v = ctx.empty(ctx.shape_cell).zero_(), ctx.empty(ctx.shape_cell).zero_()
        w = torch.zeros((c.g.z.n + 1, c.g.y.n, c.g.x.n), dtype=torch.float64, device=u.device)
        run = ctx.step_runner(ring, u, v, w)
        prev = cur = 0
        for n in range(7):
            out = 1 + n % 3
            run.step(n, prev, cur, out)
            prev, cur = cur, out
        assert np.abs(host(ring[cur]) - th).max() < 1e-13


@pytest.mark.parametrize("walls", [PERIODIC, (True, True)])
def test_adjoint_parity_explicit_share(walls):
    """Reverse sweep through refine + 7 steps (every step type) against the
    oracle's discrete adjoint with w = 1/2."""
    print("case zweight adjoint", walls, flush=True)
    c = ZCase((6, 5, 9), (2, 2, 2), walls, 0.5, n_avg=3, gamma=1.5)
    U, V, W = c.coarse_velocity()
    th0 = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.1, seed=2)
    target = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.1, seed=3)
    N = 7
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
