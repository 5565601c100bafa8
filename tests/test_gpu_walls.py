"""GPU parity with adiabatic no-slip side walls (x, y or both) against the
oracle, through the C ABI.

Array conventions differ only in the stored wall faces: the oracle keeps both
wall faces of a walled axis (n + 1 faces), the library keeps n faces with face
0 the low wall and the high wall implicit.  The helpers below convert."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.intergrid import thermal_dissipation
from paper_1805_03426_amd import inputs
from tests.test_gpu_parity import FP32_TOL, FP64_TOL, dev, host, rel_l2, rel_max

pytestmark = pytest.mark.gpu
SIDES = [(True, False), (False, True), (True, True)]   # (walls in x, walls in y)


def lib_to_oracle(a, axis):
    """Append the (zero) high wall face along ``axis``."""
    pad = [(0, 0)] * a.ndim
    pad[axis] = (0, 1)
    return np.pad(a, pad)


def oracle_to_lib(a, axis):
    """Drop the high wall face along ``axis``."""
    return np.take(a, np.arange(a.shape[axis] - 1), axis=axis)


class WallCase:
    def __init__(self, nc, m, walls, gamma=1.5, precision="fp64", seed=1, dt=2e-3, ra=1e5, pr=1.0,
                 n_avg=5, bc=("dirichlet", "dirichlet")):
        self.nc, self.m, self.walls = nc, m, walls
        nx, ny, nz = (c * q for c, q in zip(nc, m))
        rng = np.random.default_rng(seed)
        self.xf = inputs.uniform_faces(nx)
        hy = rng.uniform(0.7, 1.4, ny)
        self.yf = np.concatenate([[0.0], np.cumsum(hy)]) / hy.sum()
        self.zf = inputs.tanh_faces(nz, gamma)
        self.g = O.Grid(self.xf, self.yf, self.zf, m, periodic=(not walls[0], not walls[1], False))
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.p = O.ScalarParams.from_ra_pr(ra, pr, dt, n_avg=n_avg, bc_bot=bc[0], bc_top=bc[1])
        self.ra, self.pr, self.dt, self.n_avg, self.bc = ra, pr, dt, n_avg, bc
        self.rng = rng

    def ctx(self):
        from paper_1805_03426_amd.context import Context
        return Context(self.xf, self.yf, self.zf, self.m, self.ra, self.pr, self.dt, n_avg=self.n_avg,
                       bc_bot=self.bc[0], bc_top=self.bc[1], precision=self.precision,
                       side_x="walls" if self.walls[0] else "periodic",
                       side_y="walls" if self.walls[1] else "periodic")

    def d(self, x):
        return dev(x, self.dtype)

    # oracle-shaped random velocity with zero wall faces
    def coarse_velocity(self, scale=0.2):
        g = self.g
        U = scale * self.rng.standard_normal((g.z.nc, g.y.nc, g.x.ncfaces()))
        V = scale * self.rng.standard_normal((g.z.nc, g.y.ncfaces(), g.x.nc))
        W = scale * self.rng.standard_normal((g.z.nc + 1, g.y.nc, g.x.nc))
        W[0] = W[-1] = 0.0
        if self.walls[0]:
            U[:, :, 0] = U[:, :, -1] = 0.0
        if self.walls[1]:
            V[:, 0] = V[:, -1] = 0.0
        return U, V, W

    def dense_velocity(self, scale=0.2):
        g = self.g
        u = scale * self.rng.standard_normal((g.z.n, g.y.n, g.x.nfaces()))
        v = scale * self.rng.standard_normal((g.z.n, g.y.nfaces(), g.x.n))
        w = scale * self.rng.standard_normal((g.z.n + 1, g.y.n, g.x.n))
        w[0] = w[-1] = 0.0
        if self.walls[0]:
            u[:, :, 0] = u[:, :, -1] = 0.0
        if self.walls[1]:
            v[:, 0] = v[:, -1] = 0.0
        return u, v, w

    def to_lib(self, u, v):
        if self.walls[0]:
            u = oracle_to_lib(u, 2)
        if self.walls[1]:
            v = oracle_to_lib(v, 1)
        return u, v

    def to_oracle(self, u, v):
        if self.walls[0]:
            u = lib_to_oracle(u, 2)
        if self.walls[1]:
            v = lib_to_oracle(v, 1)
        return u, v


@pytest.mark.parametrize("walls", SIDES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_refine_parity_with_walls(walls, prec):
    print("case walls refine", walls, prec, flush=True)
    c = WallCase((7, 5, 4), (2, 3, 2), walls, precision=prec)
    U, V, W = c.coarse_velocity()
    want = O.refine_velocity(c.g, U, V, W)
    Ul, Vl = c.to_lib(U, V)
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    with c.ctx() as ctx:
        got = [host(t) for t in ctx.interpolate_velocity(c.d(Ul), c.d(Vl), c.d(W))]
    gu, gv = c.to_oracle(got[0], got[1])
    for a, b in zip((gu, gv, got[2]), want):
        assert rel_max(a, b) <= tol
    if walls[0]:
        assert np.all(got[0][:, :, 0] == 0)
    if walls[1]:
        assert np.all(got[1][:, 0] == 0)


@pytest.mark.parametrize("nc,m", [((33, 9, 4), (2, 2, 2)), ((33, 11, 4), (2, 2, 2)), ((3, 3, 3), (3, 3, 2)),
                                  ((65, 13, 3), (1, 3, 4)), ((22, 13, 3), (3, 2, 2))])
def test_refine_parity_with_walls_tile_edges(nc, m):
    """Walled sizes whose last refinement tile would hold a single coarse cell
    (33 columns in tiles of 32, 11 rows in tiles of 5, 22 columns in tiles of
    21, 13 rows in tiles of 6): the launcher narrows the tiles so that the
    one-sided wall stencils stay in the halo.  65 x 13 with M_x = 1 takes the
    three stage kernels (a one-row fused tile is too narrow for the walls)."""
    print("case walls refine tile edges", nc, m, flush=True)
    c = WallCase(nc, m, (True, True))
    U, V, W = c.coarse_velocity()
    want = O.refine_velocity(c.g, U, V, W)
    Ul, Vl = c.to_lib(U, V)
    with c.ctx() as ctx:
        got = [host(t) for t in ctx.interpolate_velocity(c.d(Ul), c.d(Vl), c.d(W))]
    gu, gv = c.to_oracle(got[0], got[1])
    for a, b in zip((gu, gv, got[2]), want):
        assert rel_max(a, b) <= FP64_TOL


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nc,m,walls", [((35, 9, 4), (2, 1, 2), (True, True)), ((35, 10, 4), (2, 1, 2), (False, True)),
                                        ((40, 7, 3), (1, 2, 2), (True, False)), ((40, 7, 3), (1, 1, 2), (True, False))])
def test_refine_parity_with_walls_unit_factor(nc, m, walls, prec):
    """A walled axis refined by 1 (R = [0 1 0] on the centred stencil, whose
    table entries wrap even beside a wall) in the fused kernel: M_y = 1 with y
    walls (a ragged last tile of rows), M_x = 1 with x walls (one-row tiles)."""
    print("case walls refine unit factor", nc, m, walls, prec, flush=True)
    c = WallCase(nc, m, walls, precision=prec)
    U, V, W = c.coarse_velocity()
    want = O.refine_velocity(c.g, U, V, W)
    Ul, Vl = c.to_lib(U, V)
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    with c.ctx() as ctx:
        got = [host(t) for t in ctx.interpolate_velocity(c.d(Ul), c.d(Vl), c.d(W))]
    gu, gv = c.to_oracle(got[0], got[1])
    for a, b in zip((gu, gv, got[2]), want):
        assert rel_max(a, b) <= tol


def _stream_field(c):
    """Coarse velocity of psi(x, z) = sin(pi x) sin(pi z) (no flow through the
    x walls or the plates; divergence-free by Stokes), oracle layout."""
    g = c.g
    X, Z = g.x.cf, g.z.cf
    psi = np.sin(np.pi * X)[None, :] * np.sin(np.pi * Z)[:, None]
    Uxz = (psi[1:, :] - psi[:-1, :]) / np.diff(Z)[:, None]
    Wxz = -(psi[:, 1:] - psi[:, :-1]) / np.diff(X)[None, :]
    nfx = g.x.ncfaces()
    U = np.broadcast_to(Uxz[:, None, :nfx], (g.z.nc, g.y.nc, nfx)).copy()
    V = np.zeros((g.z.nc, g.y.ncfaces(), g.x.nc))
    W = np.broadcast_to(Wxz[:, None, :], (g.z.nc + 1, g.y.nc, g.x.nc)).copy()
    return U, V, W


@pytest.mark.parametrize("walls", [(True, False), (True, True)])
def test_walled_refinement_is_divergence_free_and_keeps_constants(walls):
    print("case walls divergence", walls, flush=True)
    c = WallCase((8, 6, 6), (2, 2, 2), walls, bc=("adiabatic", "adiabatic"))
    U, V, W = _stream_field(c)
    Ul, Vl = c.to_lib(U, V)
    with c.ctx() as ctx:
        u, v, w = ctx.interpolate_velocity(c.d(Ul), c.d(Vl), c.d(W))
        dv = host(ctx.divergence(u, v, w))
        assert dv[1] < 64 * np.finfo(np.float64).eps
        ring = [c.d(np.full(c.g.shape, 0.625))] + [ctx.empty(ctx.shape_cell) for _ in range(3)]
        run = ctx.step_runner(ring, u, v, w)
        prev = cur = 0
        for n in range(6):
            out = 1 + n % 3
            run.step(n, prev, cur, out)
            prev, cur = cur, out
        assert np.abs(host(ring[cur]) - 0.625).max() < 1e-13


@pytest.mark.parametrize("walls", SIDES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_step_parity_with_walls(walls, prec):
    """Ragged sizes (odd ny for the two-row FP64 patches, nx not a multiple of
    the patch width), every step type, Dirichlet bottom and adiabatic top."""
    print("case walls step", walls, prec, flush=True)
    c = WallCase((35, 9, 5), (2, 1, 2), walls, precision=prec, bc=("dirichlet", "adiabatic"), n_avg=3)
    u, v, w = c.dense_velocity()
    th0 = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.1, seed=2)
    th1 = th0 + 0.05 * c.rng.standard_normal(th0.shape)
    ul, vl = c.to_lib(u, v)
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    with c.ctx() as ctx:
        du, dv_, dw = c.d(ul), c.d(vl), c.d(w)
        for n in (0, 1, 2):
            out = ctx.empty(ctx.shape_cell)
            ctx.scalar_step(n, c.d(th0), c.d(th1), out, du, dv_, dw)
            want = O.scalar_step(c.g, c.p, n, th0, th1, u, v, w)
            assert rel_l2(host(out), want) <= tol, n
            if prec == "fp64":
                assert rel_max(host(out), want) <= tol, n


@pytest.mark.parametrize("walls", SIDES)
def test_adjoint_parity_with_walls(walls):
    """Reverse sweep through refine + 6 steps against the oracle's discrete
    adjoint: interior coarse faces match; the low wall faces get zero."""
    print("case walls adjoint", walls, flush=True)
    c = WallCase((6, 5, 5), (2, 2, 2), walls, n_avg=3)
    U, V, W = c.coarse_velocity()
    th0 = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.1, seed=2)
    target = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.1, seed=3)
    N = 6
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
        assert np.all(gU[:, :, 0] == 0)
        assert rel_max(gU[:, :, 1:], wU[:, :, 1:-1]) <= 1e-11
    else:
        assert rel_max(gU, wU) <= 1e-11
    if walls[1]:
        assert np.all(gV[:, 0] == 0)
        assert rel_max(gV[:, 1:], wV[:, 1:-1]) <= 1e-11
    else:
        assert rel_max(gV, wV) <= 1e-11


@pytest.mark.parametrize("walls", SIDES)
def test_dissipation_parity_with_walls(walls):
    print("case walls Nu_T", walls, flush=True)
    c = WallCase((9, 7, 6), (2, 3, 2), walls)
    th = inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.2, seed=5)
    want = thermal_dissipation(c.g, c.p, th)
    with c.ctx() as ctx:
        _, got = ctx.thermal_dissipation(c.d(th))
    for k in ("nu_t", "gx2", "gy2", "gz2"):
        assert abs(got[k] - want[k]) <= FP64_TOL * want["nu_t"], k
