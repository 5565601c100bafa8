"""NaN canaries around every field an entry point touches.

Each input and output is a view into a larger buffer whose other elements are
NaN.  A read outside an input carries NaN into an output, a write outside an
output overwrites a canary, and an output element that is never written keeps
its NaN.  Ragged sizes (x not a multiple of 64, odd y rows, z not a multiple of
the line solver's chunk), both precisions, the fused line solver and the column
sweeps, the variant kernels (side walls, fourth-order faces, explicit z share),
columns taller than the line solver's, and views that start 16-byte aligned or
one element off it (the reductions then take their one-cell-a-lane paths)."""
import numpy as np
import pytest
import torch

from paper_1805_03426_amd import inputs
from tests.test_gpu_parity import Case

pytestmark = pytest.mark.gpu

GUARD = 256   # canary elements after each view


class Guards:
    def __init__(self, offset):
        self.offset = offset
        self.bufs = []

    def view(self, shape, dtype, fill=None):
        n = int(np.prod(shape))
        buf = torch.full((self.offset + n + GUARD,), float("nan"), dtype=dtype, device="cuda")
        v = buf[self.offset:self.offset + n].view(shape)
        if fill is not None:
            v.copy_(fill)
        self.bufs.append((buf, n))
        return v

    def check(self):
        torch.cuda.synchronize()
        for q, (buf, n) in enumerate(self.bufs):
            h = buf.cpu()
            assert torch.isnan(h[:self.offset]).all(), "canary before buffer %d overwritten" % q
            assert torch.isnan(h[self.offset + n:]).all(), "canary after buffer %d overwritten" % q


def finite(t, what):
    torch.cuda.synchronize()
    assert torch.isfinite(t).all(), "%s holds a non-finite value" % what


def _run(c, ctx, offset):
    g = Guards(offset)
    dt = c.dtype
    U, V, W = (g.view(x.shape, dt, c.d(x)) for x in (c.U, c.V, c.W))
    u, v, w = g.view(ctx.shape_cell, dt), g.view(ctx.shape_cell, dt), g.view(ctx.shape_w, dt)
    ctx.interpolate_velocity(U, V, W, out=(u, v, w))
    for t, name in ((u, "u"), (v, "v"), (w, "w")):
        finite(t, name)
    div = g.view((2,), torch.float64)
    ctx.divergence(u, v, w, out=div)
    finite(div, "divergence")
    th0 = g.view(ctx.shape_cell, dt, c.d(c.th0))
    N = 4
    th = [th0] + [g.view(ctx.shape_cell, dt) for _ in range(N)]
    ctx.scalar_steps(0, None, th0, th[1:], u, v, w)
    for q in range(1, N + 1):
        finite(th[q], "theta^%d" % q)
    prof = g.view((ctx.nz + 6,), torch.float64)
    ctx.nusselt(th[N], w, profile=prof, sync=False)
    finite(prof, "Nusselt profile")
    diss = g.view((4,), torch.float64)
    ctx.thermal_dissipation(th[N], out=diss, sync=False)
    finite(diss, "Nu_T")
    tc = g.view(ctx.shape_coarse, dt)
    ctx.integrate_scalar(th[N], out=tc)
    finite(tc, "coarse theta")
    # reverse: seed, reverse steps N-1 .. 1 as one sequence, the start-up step's reverse
    lam = g.view(ctx.shape_cell, dt, th[N] - th[N - 1])
    mu = [None] * N
    mu[N - 1] = g.view(ctx.shape_cell, dt)
    ctx.adjoint_seed(N - 1, lam, mu[N - 1])
    finite(mu[N - 1], "seed")
    outs = [g.view(ctx.shape_cell, dt) for _ in range(N - 1)]
    ctx.scalar_steps_backward(N - 1, None, mu[N - 1], outs, u, v, w)
    for q, o in enumerate(outs):
        mu[N - 2 - q] = o
        finite(o, "mu^%d" % (N - 2 - q))
    g0 = g.view(ctx.shape_cell, dt)
    ctx.scalar_step_backward(0, mu[1], mu[0], None, g0, u, v, w)
    finite(g0, "dL/dtheta^0")
    gu, gv = g.view(ctx.shape_cell, dt, torch.zeros(ctx.shape_cell)), g.view(ctx.shape_cell, dt, torch.zeros(ctx.shape_cell))
    gw = g.view(ctx.shape_w, dt, torch.zeros(ctx.shape_w))
    ctx.velocity_grad(list(range(N)), th[:N], mu, gu, gv, gw)
    for t, name in ((gu, "g_u"), (gv, "g_v"), (gw, "g_w")):
        finite(t, name)
    gU, gV = g.view(ctx.shape_coarse, dt), g.view(ctx.shape_coarse, dt)
    gW = g.view(ctx.shape_coarse_w, dt)
    ctx.interpolate_velocity_backward(gu, gv, gw, out=(gU, gV, gW))
    for t, name in ((gU, "g_U"), (gV, "g_V"), (gW, "g_W")):
        finite(t, name)
    # the time-blended refinement and a coarse step of M_t = 2
    U1, V1, W1 = (g.view(x.shape, dt, 0.5 * x) for x in (U, V, W))
    ut, vt, wt = g.view(ctx.shape_cell, dt), g.view(ctx.shape_cell, dt), g.view(ctx.shape_w, dt)
    ctx.interpolate_velocity_time(U, V, W, U1, V1, W1, 1, 3, out=(ut, vt, wt))
    for t, name in ((ut, "u(t)"), (vt, "v(t)"), (wt, "w(t)")):
        finite(t, name)
    ring = [g.view(ctx.shape_cell, dt, th0), g.view(ctx.shape_cell, dt), g.view(ctx.shape_cell, dt)]
    tcs = g.view(ctx.shape_coarse, dt)
    prev, cur = ctx.coarse_step(0, 2, U, V, W, U1, V1, W1, (ut, vt, wt), ring, 0, 0, tcs)
    finite(ring[prev], "coarse step theta^1")
    finite(ring[cur], "coarse step theta^2")
    finite(tcs, "coarse step coarse theta")
    g.check()


@pytest.mark.parametrize("offset", [64, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["line", "sweep"])
def test_canaries_plain(method, prec, offset):
    print("case canaries", method, prec, offset, flush=True)
    c = Case((35, 9, 35), (2, 1, 2), 2.0, n_avg=3, precision=prec)
    with c.ctx(step_method=method) as ctx:
        assert ctx.step_method == method
        _run(c, ctx, offset)


@pytest.mark.parametrize("offset", [64, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_canaries_variants(prec, offset):
    """Side walls in x and y, fourth-order faces and an explicit z share of 1/2
    (the line solver's variant kernels and the walled refinement)."""
    print("case canaries variants", prec, offset, flush=True)
    from paper_1805_03426_amd.context import Context
    from tests.test_gpu_walls import WallCase
    c = WallCase((35, 9, 35), (2, 1, 2), (True, True), precision=prec, n_avg=3, dt=2e-4)
    c.th0 = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.1, seed=2)
    c.U, c.V, c.W = c.coarse_velocity()
    c.U, c.V = c.to_lib(c.U, c.V)
    with Context(c.xf, c.yf, c.zf, c.m, c.ra, c.pr, c.dt, n_avg=c.n_avg, precision=prec, side_x="walls",
                 side_y="walls", face_order=4, z_explicit=0.5) as ctx:
        assert ctx.step_method == "line"
        _run(c, ctx, offset)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_canaries_tall_columns(prec):
    """700 levels: beyond the line solver, so the steps, the reverse steps, the
    start-up step's reverse and the seed run as column sweeps and column solves."""
    print("case canaries tall", prec, flush=True)
    c = Case((32, 4, 350), (2, 2, 2), 2.0, kmax=1, n_avg=3, precision=prec, dt=1e-5)
    with c.ctx() as ctx:
        assert ctx.step_method == "sweep"
        _run(c, ctx, 64)
