"""GPU parity: every entry point of the HIP library against the FP64 oracle on
the same seeded inputs, through the C ABI.  Tolerances: relative L2 (and
max-norm) <= 1e-12 for FP64, <= 1e-5 per step for the FP32 tier."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_03426_amd import inputs
from paper_1805_03426_amd.configs import WORKLOADS

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5
# The conduction profile 1 - z dominates the norm of theta, so the FP32 tier is
# also held to bounds on what the step changes: the relative L2 error of the
# fluctuation theta - (1 - z_c) and of the step's increment theta^{n+1} - theta^n
# (the GPU's increment taken from its own FP32 input).  A correct FP32 step
# differs from the oracle by a few units of FP32 rounding of theta (the cast
# inputs and the stored result), about 1e-7 absolute; the fluctuation (rms
# 0.02) and the increment (about 5e-3 per step here) turn that into relative
# errors of order 1e-6 and 1e-5.  Measured worst over the FP32 parity cases:
# fluctuation 1.9e-6, increment 3.1e-5; the bounds are 5x and 10x those.
FP32_FLUCT_TOL = 1e-5
FP32_INCR_TOL = 3e-4
EPS = np.finfo(np.float64).eps


def _ctx_cls():
    from paper_1805_03426_amd.context import Context
    return Context


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def rel_max(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


class Case:
    """A grid with its oracle geometry, coarse velocity and initial scalar."""

    def __init__(self, nc, m, gamma, ra=1e6, pr=4.38, kmax=4, n_avg=50, precision="fp64",
                 bc=("dirichlet", "dirichlet"), seed=1, stretch_x=False, dt=None, random_velocity=False):
        self.m = m
        nx, ny, nz = (c * q for c, q in zip(nc, m))
        if stretch_x:
            rng = np.random.default_rng(77)
            hx = rng.uniform(0.6, 1.6, nx)
            self.xf = np.concatenate([[0.0], np.cumsum(hx)]) / hx.sum()
        else:
            self.xf = inputs.uniform_faces(nx)
        self.yf = inputs.uniform_faces(ny)
        self.zf = inputs.tanh_faces(nz, gamma)
        self.g = O.Grid(self.xf, self.yf, self.zf, m)
        if random_velocity:
            # any face velocity is a valid input of the step (no divergence constraint)
            rng = np.random.default_rng(seed)
            cs = (nc[2], nc[1], nc[0])
            self.U = 0.2 * rng.standard_normal(cs)
            self.V = 0.2 * rng.standard_normal(cs)
            self.W = 0.2 * rng.standard_normal((nc[2] + 1, nc[1], nc[0]))
            self.W[0] = self.W[-1] = 0.0
        else:
            self.U, self.V, self.W = inputs.divergence_free_velocity(self.g.x.cf, self.g.y.cf, self.g.z.cf,
                                                                     kmax, 0.2, seed)
        self.th0 = inputs.theta_initial(self.zf, nx, ny)
        self.dt = dt if dt is not None else inputs.cfl_dt(self.U, self.V, self.W, self.xf, self.yf,
                                                           self.zf, m)
        self.ra, self.pr, self.n_avg, self.bc = ra, pr, n_avg, bc
        self.p = O.ScalarParams.from_ra_pr(ra, pr, self.dt, n_avg=n_avg, bc_bot=bc[0], bc_top=bc[1])
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32

    def ctx(self, step_method="auto"):
        return _ctx_cls()(self.xf, self.yf, self.zf, self.m, self.ra, self.pr, self.dt, n_avg=self.n_avg,
                          bc_bot=self.bc[0], bc_top=self.bc[1], precision=self.precision, step_method=step_method)

    def d(self, x):
        return dev(x, self.dtype)


@pytest.fixture(scope="module")
def c1():
    w = WORKLOADS["rb64-m2-fp64"]
    case = Case(w.nc, w.m, w.gamma, ra=w.ra, pr=w.pr, kmax=w.kmax)
    case.uvw = O.refine_velocity(case.g, case.U, case.V, case.W)
    return case


# ------------------------------------------------------------------ refinement
def test_refine_parity_rb64(c1):
    print("case rb64 refine fp64", flush=True)
    with c1.ctx() as ctx:
        out = ctx.interpolate_velocity(c1.d(c1.U), c1.d(c1.V), c1.d(c1.W))
        torch.cuda.synchronize()
        for got, want in zip(out, c1.uvw):
            assert rel_max(host(got), want) <= FP64_TOL
        dv = host(ctx.divergence(*out))
        assert dv[1] < 64 * EPS and dv[0] < 1e-15


@pytest.mark.parametrize("nc,m,gamma", [((5, 3, 7), (3, 1, 2), 1.0), ((3, 4, 3), (2, 3, 4), 2.0),
                                        ((7, 6, 5), (1, 1, 1), 0.5), ((4, 3, 9), (5, 2, 3), 1.5)])
def test_refine_parity_ragged(nc, m, gamma):
    """Odd sizes: x not a multiple of the 64-lane tile, 3 coarse cells, M = 1, M = 5."""
    print("case refine ragged", nc, m, flush=True)
    case = Case(nc, m, gamma, kmax=1, stretch_x=True)
    want = O.refine_velocity(case.g, case.U, case.V, case.W)
    with case.ctx() as ctx:
        got = ctx.interpolate_velocity(case.d(case.U), case.d(case.V), case.d(case.W))
        for a, b in zip(got, want):
            assert rel_max(host(a), b) <= FP64_TOL
        if m == (1, 1, 1):
            for a, b in zip(got, (case.U, case.V, case.W)):
                assert np.array_equal(host(a), b)


def test_refine_random_field_closure():
    """Non-divergence-free coarse input: parity, and the GPU divergence check
    reports the oracle's maximum."""
    print("case refine random", flush=True)
    rng = np.random.default_rng(5)
    case = Case((6, 5, 6), (2, 2, 3), 1.2, kmax=1)
    U = rng.standard_normal(case.U.shape)
    V = rng.standard_normal(case.V.shape)
    W = rng.standard_normal(case.W.shape)
    want = O.refine_velocity(case.g, U, V, W)
    div, tot = O.divergence(case.g, *want)
    with case.ctx() as ctx:
        got = ctx.interpolate_velocity(case.d(U), case.d(V), case.d(W))
        for a, b in zip(got, want):
            assert rel_max(host(a), b) <= FP64_TOL
        dv = host(ctx.divergence(*[case.d(x) for x in want]))
        assert abs(dv[0] - np.abs(div).max()) <= 1e-12 * np.abs(div).max()
        assert abs(dv[1] - np.max(np.abs(div) / tot)) <= 1e-12


# ------------------------------------------------------------------ step
def fp32_fine_errors(got, want, cur_in, cur, zc):
    """Relative L2 errors of the fluctuation theta - (1 - z_c) and of the step's
    increment (the GPU's from its FP32 input cur_in, the oracle's from cur)."""
    prof = (1.0 - zc)[:, None, None]
    return rel_l2(got - prof, want - prof), rel_l2(got - cur_in, want - cur)


def _step_parity(case, nsteps, tol, uvw=None, report=None):
    """Run nsteps on the GPU, each step from the oracle's own previous levels
    (cast to the tier), and compare with the oracle's step.  FP32 steps are
    also held to the fluctuation and increment bounds."""
    g, p = case.g, case.p
    if uvw is None:
        uvw = O.refine_velocity(g, case.U, case.V, case.W)
    u, v, w = uvw
    prev = cur = case.th0
    worst = 0.0
    fine = [0.0, 0.0]
    with case.ctx() as ctx:
        du, dv_, dw = (case.d(x) for x in uvw)
        out = ctx.empty(ctx.shape_cell)
        for n in range(nsteps):
            want = O.scalar_step(g, p, n, prev, cur, u, v, w)
            dcur = case.d(cur)
            ctx.scalar_step(n, case.d(prev), dcur, out, du, dv_, dw)
            got = host(out)
            err = rel_l2(got, want)
            worst = max(worst, err)
            assert err <= tol, (n, err)
            if case.precision == "fp32":
                ef, ei = fp32_fine_errors(got, want, host(dcur), cur, g.z.c)
                fine = [max(fine[0], ef), max(fine[1], ei)]
                assert ef <= FP32_FLUCT_TOL and ei <= FP32_INCR_TOL, (n, ef, ei)
            prev, cur = cur, want
    if case.precision == "fp32":
        print("fp32 step errors: theta %.2e, fluctuation %.2e, increment %.2e" % (worst, *fine), flush=True)
    if report is not None:
        report.append(worst)
    return worst


def test_step_parity_rb64(c1):
    print("case rb64 steps fp64", flush=True)
    _step_parity(c1, 10, FP64_TOL, c1.uvw)


def test_step_parity_averaging_and_adiabatic():
    """N_p = 3 exercises the averaging step; adiabatic top wall."""
    print("case step averaging", flush=True)
    case = Case((8, 6, 10), (2, 2, 2), 2.0, kmax=2, n_avg=3, bc=("dirichlet", "adiabatic"))
    _step_parity(case, 8, FP64_TOL)


@pytest.mark.parametrize("nc,m,gamma", [((5, 3, 7), (3, 1, 2), 1.0), ((4, 4, 1), (2, 2, 1), 0.0),
                                        ((3, 3, 160), (5, 1, 4), 2.5), ((33, 3, 3), (3, 2, 3), 1.0),
                                        ((1, 1, 1), (1, 1, 1), 0.0), ((1, 2, 2), (1, 1, 1), 0.5),
                                        ((3, 3, 275), (4, 1, 2), 2.0)])
def test_step_parity_ragged(nc, m, gamma):
    """x not a multiple of 64, a single z level, the largest z (640 levels:
    16 chunks of 40), 550 levels (16 chunks of 36, the last one ragged), a
    ragged last chunk, stretched x, a single cell (its own periodic neighbour
    on every side) and single-column grids."""
    print("case step ragged", nc, m, flush=True)
    case = Case(nc, m, gamma, kmax=1, stretch_x=True, n_avg=2, random_velocity=True)
    _step_parity(case, 4, FP64_TOL)


@pytest.mark.parametrize("ncz,mz", [(150, 2), (275, 2), (128, 2)])
def test_step_and_adjoint_parity_deep_columns(ncz, mz):
    """Uniform x and y with columns of 300 and 550 levels (10 chunks of 32, 16
    of 36): the FP64 one-row layout for columns of more than 8 chunks, forward
    (every step type) and reverse; 256 levels (8 chunks) keeps two-row patches."""
    print("case deep columns", ncz, mz, flush=True)
    case = Case((5, 3, ncz), (2, 2, mz), 2.0, kmax=1, n_avg=2, random_velocity=True, dt=1e-4)
    _step_parity(case, 4, FP64_TOL)
    target = inputs.theta_initial(case.zf, case.g.x.n, case.g.y.n, seed=3)
    _, w0, wU, wV, wW = O.rollout_loss_grad(case.g, case.p, case.th0, case.U, case.V, case.W, 4, target)
    g0, gU, gV, gW = _gpu_loss_grad(case, 4, target)
    assert rel_max(g0, w0) <= 1e-11
    for a, b in zip((gU, gV, gW), (wU, wV, wW)):
        assert rel_max(a, b) <= 1e-11


def test_step_fp32_tier_rb64(c1):
    print("case rb64 steps fp32", flush=True)
    case = Case((32, 32, 32), (2, 2, 2), 0.0, ra=1e6, pr=4.38, kmax=8, precision="fp32")
    _step_parity(case, 10, FP32_TOL, c1.uvw)


def test_step_conduction_fixed_point_gpu():
    """u = 0 and theta = 1 - z_c: the GPU step keeps it to rounding."""
    print("case conduction", flush=True)
    case = Case((4, 4, 32), (2, 2, 2), 2.0, random_velocity=True)
    th = np.broadcast_to((1.0 - case.g.z.c)[:, None, None], case.g.shape).copy()
    z = np.zeros(case.g.shape)
    zw = np.zeros((case.g.z.n + 1,) + case.g.shape[1:])
    with case.ctx() as ctx:
        a, b, c = case.d(th), case.d(th), ctx.empty(ctx.shape_cell)
        for n in range(5):
            ctx.scalar_step(n, a, b, c, case.d(z), case.d(z), case.d(zw))
            assert np.abs(host(c) - th).max() < 1e-14
            a, b, c = b, c, a


def test_step_deterministic(c1):
    print("case determinism", flush=True)
    with c1.ctx() as ctx:
        du, dv_, dw = (c1.d(x) for x in c1.uvw)
        th = c1.d(c1.th0)
        o1, o2 = ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell)
        ctx.scalar_step(0, th, th, o1, du, dv_, dw)
        ctx.scalar_step(0, th, th, o2, du, dv_, dw)
        assert torch.equal(o1, o2)
        p1, _ = ctx.nusselt(o1, dw)
        p2, _ = ctx.nusselt(o1, dw)
        assert torch.equal(p1, p2)


# ------------------------------------------------------------------ Nusselt
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nusselt_parity(c1, precision):
    print("case nusselt", precision, flush=True)
    th = O.rollout(c1.g, c1.p, c1.th0, *c1.uvw, 3)
    w = c1.uvw[2]
    if precision == "fp32":
        th = th.astype(np.float32).astype(np.float64)
        w = w.astype(np.float32).astype(np.float64)
    prof, summ = O.nusselt(c1.g, c1.p, th, w)
    case = Case((32, 32, 32), (2, 2, 2), 0.0, kmax=8, precision=precision)
    with case.ctx() as ctx:
        dprof, dsum = ctx.nusselt(case.d(th), case.d(w))
        gp = host(dprof)
    scale = np.abs(prof).max()
    assert np.abs(gp[:-5] - prof).max() <= 1e-12 * scale
    for k, key in enumerate(["nu_bot", "nu_top", "nu_vol", "nu_paper", "mean_theta"]):
        assert abs(dsum[key] - summ[key]) <= 1e-12 * max(1.0, abs(summ[key])), key
        assert gp[-5 + k] == dsum[key]


def test_nusselt_conduction_gpu():
    print("case nusselt conduction", flush=True)
    case = Case((4, 5, 40), (2, 2, 2), 2.5, random_velocity=True)
    th = np.broadcast_to((1.0 - case.g.z.c)[:, None, None], case.g.shape).copy()
    w = np.zeros((case.g.z.n + 1,) + case.g.shape[1:])
    with case.ctx() as ctx:
        prof, s = ctx.nusselt(case.d(th), case.d(w))
    assert np.abs(host(prof)[:-5] - 1.0).max() < 1e-12
    assert abs(s["mean_theta"] - 0.5) < 1e-15


# ------------------------------------------------------------------ adjoint
def _gpu_loss_grad(case, nsteps, target):
    """Plain reverse sweep through the C ABI (no checkpointing)."""
    with case.ctx() as ctx:
        U, V, W = case.d(case.U), case.d(case.V), case.d(case.W)
        u, v, w = ctx.interpolate_velocity(U, V, W)
        th = [case.d(case.th0)]
        for n in range(nsteps):
            out = ctx.empty(ctx.shape_cell)
            ctx.scalar_step(n, th[n - 1] if n else th[0], th[n], out, u, v, w)
            th.append(out)
        lam = th[nsteps] - case.d(target)
        mu = [None] * (nsteps + 1)
        mu[nsteps - 1] = ctx.empty(ctx.shape_cell)
        ctx.adjoint_seed(nsteps - 1, lam, mu[nsteps - 1])
        g0 = ctx.empty(ctx.shape_cell)
        for n in range(nsteps - 1, -1, -1):
            out = ctx.empty(ctx.shape_cell) if n > 0 else g0
            ctx.scalar_step_backward(n, mu[n + 1], mu[n], None, out, u, v, w)
            if n > 0:
                mu[n - 1] = out
        gu = torch.zeros_like(u)
        gv = torch.zeros_like(v)
        gw = torch.zeros_like(w)
        for s0 in range(0, nsteps, 16):
            idx = list(range(s0, min(nsteps, s0 + 16)))
            ctx.velocity_grad(idx, [th[n] for n in idx], [mu[n] for n in idx], gu, gv, gw)
        gU, gV, gW = ctx.interpolate_velocity_backward(gu, gv, gw)
        torch.cuda.synchronize()
        return host(g0), host(gU), host(gV), host(gW)


@pytest.mark.parametrize("nsteps,n_avg,stretch_x", [(6, 3, False), (18, 50, False), (6, 3, True)])
def test_adjoint_parity(nsteps, n_avg, stretch_x):
    """Reverse sweep on the GPU vs the oracle's discrete adjoint (FP64), on
    uniform x and y (the uniform-width kernels) and on stretched x."""
    print("case adjoint", nsteps, n_avg, stretch_x, flush=True)
    case = Case((8, 6, 7), (2, 3, 2), 1.5, ra=1e4, kmax=2, n_avg=n_avg, stretch_x=stretch_x)
    target = inputs.theta_initial(case.zf, case.g.x.n, case.g.y.n, seed=3)
    _, w0, wU, wV, wW = O.rollout_loss_grad(case.g, case.p, case.th0, case.U, case.V, case.W, nsteps, target)
    g0, gU, gV, gW = _gpu_loss_grad(case, nsteps, target)
    assert rel_max(g0, w0) <= 1e-11
    for a, b in zip((gU, gV, gW), (wU, wV, wW)):
        assert rel_max(a, b) <= 1e-11


@pytest.mark.parametrize("stretch_x", [False, True])
def test_adjoint_parity_fp32(stretch_x):
    """FP32 reverse sweep (the uniform-width kernels with two levels of
    prefetch, and the general kernels on stretched x) against the oracle's
    FP64 discrete adjoint: relative L2 within the FP32 step bar."""
    print("case adjoint fp32", stretch_x, flush=True)
    case = Case((8, 6, 7), (2, 3, 2), 1.5, ra=1e4, kmax=2, n_avg=3, precision="fp32", stretch_x=stretch_x)
    target = inputs.theta_initial(case.zf, case.g.x.n, case.g.y.n, seed=3)
    _, w0, wU, wV, wW = O.rollout_loss_grad(case.g, case.p, case.th0, case.U, case.V, case.W, 6, target)
    got = _gpu_loss_grad(case, 6, target)
    for a, b in zip(got, (w0, wU, wV, wW)):
        assert rel_l2(a, b) <= FP32_TOL


@pytest.mark.parametrize("nsteps,ckpt,method", [(7, 3, "auto"), (7, 1, "auto"), (7, 16, "auto"), (6, 3, "auto"),
                                                (1, 3, "auto"), (5, 5, "auto"), (20, 18, "auto"), (7, 3, "sweep"),
                                                (20, 6, "sweep"), (2, 1, "sweep")])
def test_rollout_checkpoint_segments(nsteps, ckpt, method):
    """The autograd rollout (checkpoint pairs and the last segment kept by the
    forward pass, the other segments recomputed; the forward pass and each
    recomputation one step sequence) against the oracle's discrete adjoint,
    for segment counts of one to seven, a ragged last segment, a single step
    and segments longer than one velocity-gradient call (FP64), with the
    sequences on the line solver and on the column sweeps."""
    print("case rollout", nsteps, ckpt, method, flush=True)
    from paper_1805_03426_amd.autograd import rollout
    case = Case((8, 6, 7), (2, 3, 2), 1.5, ra=1e4, kmax=2, n_avg=3)
    target = inputs.theta_initial(case.zf, case.g.x.n, case.g.y.n, seed=3)
    _, w0, wU, wV, wW = O.rollout_loss_grad(case.g, case.p, case.th0, case.U, case.V, case.W, nsteps, target)
    with case.ctx(method) as ctx:
        assert ctx.step_method == ("sweep" if method == "sweep" else "line")
        th = case.d(case.th0).requires_grad_(True)
        U, V, W = (case.d(a).requires_grad_(True) for a in (case.U, case.V, case.W))
        out = rollout(ctx, th, U, V, W, nsteps, ckpt)
        torch.autograd.backward(out, out.detach() - case.d(target))
        got = [host(t.grad) for t in (th, U, V, W)]
    for a, b in zip(got, (w0, wU, wV, wW)):
        assert rel_max(a, b) <= 1e-11


def test_refine_transpose_dot_product():
    """<P x, y> = <x, P^T y> on the GPU (FP64), ragged grid."""
    print("case refine transpose", flush=True)
    rng = np.random.default_rng(9)
    case = Case((5, 4, 6), (3, 2, 2), 2.0, kmax=1)
    xs = [rng.standard_normal(s) for s in (case.U.shape, case.V.shape, case.W.shape)]
    g = case.g
    ys = [rng.standard_normal(s) for s in ((g.z.n, g.y.n, g.x.n), (g.z.n, g.y.n, g.x.n), (g.z.n + 1, g.y.n, g.x.n))]
    with case.ctx() as ctx:
        Px = [host(t) for t in ctx.interpolate_velocity(*[case.d(x) for x in xs])]
        PTy = [host(t) for t in ctx.interpolate_velocity_backward(*[case.d(y) for y in ys])]
    want = O.refine_velocity_transpose(g, *ys)
    for a, b in zip(PTy, want):
        assert rel_max(a, b) <= FP64_TOL
    lhs = sum(np.vdot(a, b) for a, b in zip(Px, ys))
    rhs = sum(np.vdot(a, b) for a, b in zip(xs, PTy))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ------------------------------------------------------------------ full size
def test_full_size_rb256_fp64():
    """The 128^3 -> 256^3 workload at full size in the benchmark's launch
    configuration: refinement and the first two steps (start-up, leapfrog)
    against the oracle on the whole field, plus an averaging step."""
    print("case rb256 full size", flush=True)
    w = WORKLOADS["rb256-m2-fp64"]
    d = inputs.workload_inputs(w)
    g = O.Grid(d["xf"], d["yf"], d["zf"], w.m)
    p = O.ScalarParams.from_ra_pr(w.ra, w.pr, d["dt"], n_avg=w.n_avg)
    uvw = O.refine_velocity(g, d["U"], d["V"], d["W"])
    Context = _ctx_cls()
    with Context(d["xf"], d["yf"], d["zf"], w.m, w.ra, w.pr, d["dt"], n_avg=w.n_avg) as ctx:
        du = ctx.interpolate_velocity(dev(d["U"]), dev(d["V"]), dev(d["W"]))
        for a, b in zip(du, uvw):
            assert rel_max(host(a), b) <= FP64_TOL
        dv = host(ctx.divergence(*du))
        assert dv[1] < 64 * EPS
        th0 = d["theta0"]
        t1 = O.scalar_step(g, p, 0, th0, th0, *uvw)
        out = ctx.empty(ctx.shape_cell)
        ctx.scalar_step(0, dev(th0), dev(th0), out, *du)
        assert rel_l2(host(out), t1) <= FP64_TOL
        t2 = O.scalar_step(g, p, 1, th0, t1, *uvw)
        ctx.scalar_step(1, dev(th0), dev(t1), out, *du)
        assert rel_l2(host(out), t2) <= FP64_TOL
        t50 = O.scalar_step(g, p, 49, th0, t1, *uvw)
        ctx.scalar_step(49, dev(th0), dev(t1), out, *du)
        assert rel_l2(host(out), t50) <= FP64_TOL
        prof, s = O.nusselt(g, p, t1, uvw[2])
        dprof, ds = ctx.nusselt(dev(t1), du[2])
        assert np.abs(host(dprof)[:-5] - prof).max() <= 1e-12 * np.abs(prof).max()
