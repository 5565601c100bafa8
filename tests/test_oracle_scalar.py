"""Pins of the oracle's scalar step, Nusselt diagnostics and adjoint to closed
forms, invariants, library solvers and a brute-force face-loop assembly."""
import math

import numpy as np
import pytest
from scipy.linalg import solve_banded

import oracle as O
from oracle.scalar import ADIABATIC, DIRICHLET
from paper_1805_03426_amd import inputs

EPS = np.finfo(np.float64).eps


def _grid(n, gamma=0.0, rng=None, m=(1, 1, 1)):
    nx, ny, nz = n
    if rng is None:
        xf, yf = inputs.uniform_faces(nx), inputs.uniform_faces(ny)
    else:
        hx = rng.uniform(0.6, 1.6, nx)
        hy = rng.uniform(0.6, 1.6, ny)
        xf = np.concatenate([[0], np.cumsum(hx)]) / hx.sum()
        yf = np.concatenate([[0], np.cumsum(hy)]) / hy.sum()
    zf = inputs.tanh_faces(nz, gamma)
    return O.Grid(xf, yf, zf, m)


def _dense_velocity(g, kmax=2, seed=1, urms=0.2):
    return inputs.divergence_free_velocity(g.x.faces, g.y.faces, g.z.faces, kmax, urms, seed)


# -------------------------------------------------------------------- Thomas
def test_thomas_matches_solve_banded():
    rng = np.random.default_rng(0)
    n = 37
    sub = rng.uniform(-1, 0, n)
    sup = rng.uniform(-1, 0, n)
    diag = 1.0 + np.abs(sub) + np.abs(sup) + rng.uniform(0, 1, n)
    sub[0] = 0.0
    sup[-1] = 0.0
    r = rng.standard_normal((n, 3, 4))
    ab = np.zeros((3, n))
    ab[0, 1:] = sup[:-1]
    ab[1] = diag
    ab[2, :-1] = sub[1:]
    want = solve_banded((1, 1), ab, r.reshape(n, -1)).reshape(r.shape)
    np.testing.assert_allclose(O.thomas(sub, diag, sup, r), want, rtol=1e-13, atol=1e-14)


# ------------------------------------------------------------------- stepper
def test_step_kind_schedule():
    """Start-up at n = 0, averaging when (n+1) mod N_p = 0 (Eq. 7), else leapfrog (Eq. 6)."""
    dt = 0.01
    kinds = [O.step_kind(n, 50, dt)[3] for n in range(101)]
    assert kinds[0] == "startup"
    assert [n for n, k in enumerate(kinds) if k == "average"] == [49, 99]
    assert O.step_kind(5, 50, dt)[:3] == (2 * dt, 1.0, 0.0)
    assert O.step_kind(49, 50, dt)[:3] == (1.5 * dt, 0.5, 0.5)
    assert O.step_kind(0, 50, dt)[:3] == (dt, 0.0, 1.0)
    assert all(O.step_kind(n, 0, dt)[3] != "average" for n in range(1, 200))


@pytest.mark.parametrize("gamma", [0.0, 2.0])
def test_conduction_is_fixed_point(gamma):
    """theta = 1 - z_c with u = 0 is a steady solution on any z grid, for every step type."""
    g = _grid((6, 5, 16), gamma)
    p = O.ScalarParams.from_ra_pr(1e4, 1.0, dt=0.01, n_avg=3)
    th = np.broadcast_to((1.0 - g.z.c)[:, None, None], g.shape).copy()
    u = np.zeros(g.shape)
    w = np.zeros((g.z.n + 1,) + g.shape[1:])
    prev = cur = th
    for n in range(6):
        nxt = O.scalar_step(g, p, n, prev, cur, u, u, w)
        np.testing.assert_allclose(nxt, th, atol=1e-14)
        prev, cur = cur, nxt


def _mode_field(g, kx, ky, kz):
    return (np.cos(2 * np.pi * kx * g.x.c)[None, None, :] * np.cos(2 * np.pi * ky * g.y.c)[None, :, None]
            * np.sin(np.pi * kz * g.z.c)[:, None, None])


@pytest.mark.parametrize("kvec", [(1, 2, 1), (3, 0, 2), (2, 1, 5)])
def test_fourier_mode_decay_closed_form(kvec):
    """Pure diffusion on a uniform grid: conduction + a cos.cos.sin mode is an
    eigen-solution; its amplitude follows the exact discrete recurrences of the
    start-up, leapfrog and averaging steps with the eigenvalues
    lambda_x = -4 sin^2(pi kx/Nx)/hx^2 (same for y), lambda_z = -4 sin^2(pi kz/(2Nz))/hz^2."""
    kx, ky, kz = kvec
    nx, ny, nz = 12, 10, 14
    g = _grid((nx, ny, nz))
    kappa = 3e-3
    dt = 0.02
    p = O.ScalarParams(kappa=kappa, dt=dt, n_avg=4)
    lx = -4 * math.sin(math.pi * kx / nx) ** 2 * nx * nx
    ly = -4 * math.sin(math.pi * ky / ny) ** 2 * ny * ny
    lz = -4 * math.sin(math.pi * kz / (2 * nz)) ** 2 * nz * nz
    lh = lx + ly
    base = np.broadcast_to((1.0 - g.z.c)[:, None, None], g.shape)
    mode = _mode_field(g, kx, ky, kz)
    a = [0.37]
    th = [base + a[0] * mode]
    u = np.zeros(g.shape)
    w = np.zeros((nz + 1, ny, nx))
    for n in range(10):
        tau, ap, ac, kind = O.step_kind(n, p.n_avg, dt)
        if kind == "startup":
            nxt = a[0] * (1 + dt * kappa * lh) / (1 - dt * kappa * lz)
        elif kind == "leapfrog":
            nxt = a[n - 1] * (1 + 2 * dt * kappa * lh) / (1 - 2 * dt * kappa * lz)
        else:
            nxt = (0.5 * (a[n - 1] + a[n]) + 1.5 * dt * kappa * lh * a[n - 1]) / (1 - 1.5 * dt * kappa * lz)
        a.append(nxt)
        prev = th[n - 1] if n > 0 else th[0]
        th.append(O.scalar_step(g, p, n, prev, th[n], u, u, w))
        np.testing.assert_allclose(th[-1], base + a[-1] * mode, rtol=0, atol=1e-14)


def test_stretched_z_mode_follows_recurrence():
    """Stretched z: an eigenvector of the z operator (numpy.linalg.eig of
    (I - tk Lz0) with adiabatic walls) times a horizontal cosine mode follows the
    same exact amplitude recurrences."""
    nx, ny, nz = 8, 6, 20
    g = _grid((nx, ny, nz), gamma=2.0)
    kappa, dt = 2e-3, 0.01
    p = O.ScalarParams(kappa=kappa, dt=dt, n_avg=5, bc_bot=ADIABATIC, bc_top=ADIABATIC)
    sub, diag, sup, _ = O.z_matrix(g, 1.0, p)    # I - Lz0  ->  Lz0 = I - that
    T = np.diag(diag) + np.diag(sub[1:], -1) + np.diag(sup[:-1], 1)
    Lz0 = np.eye(nz) - T
    ev, vec = np.linalg.eig(Lz0)
    order = np.argsort(-ev.real)
    lz = ev.real[order[3]]
    ez = vec[:, order[3]].real
    lx = -4 * math.sin(math.pi * 1 / nx) ** 2 * nx * nx
    mode = ez[:, None, None] * np.cos(2 * np.pi * g.x.c)[None, None, :] * np.ones((1, ny, 1))
    a = [1.0]
    th = [mode.copy()]
    u = np.zeros(g.shape)
    w = np.zeros((nz + 1, ny, nx))
    for n in range(8):
        tau, ap, ac, kind = O.step_kind(n, p.n_avg, dt)
        lag = a[n] if n == 0 else a[n - 1]
        prev = 0.0 if n == 0 else a[n - 1]
        a.append((ap * prev + ac * a[n] + tau * kappa * lx * lag) / (1 - tau * kappa * lz))
        th.append(O.scalar_step(g, p, n, th[n - 1] if n else th[0], th[n], u, u, w))
        np.testing.assert_allclose(th[-1], a[-1] * mode, atol=1e-13)


def test_advection_translation_closed_form():
    """Uniform u = c in x, kappa = 0: a Fourier mode in x is advected with the
    central-difference eigenvalue lambda = -i c sin(2 pi k hx)/hx; the complex
    amplitude follows a1 = a0 (1 + dt lambda), a_{n+1} = a_{n-1} + 2 dt lambda a_n."""
    nx, ny, nz = 16, 4, 6
    g = _grid((nx, ny, nz), gamma=1.0)
    c, k, dt = 0.8, 3, 0.01
    p = O.ScalarParams(kappa=0.0, dt=dt, n_avg=0, bc_bot=ADIABATIC, bc_top=ADIABATIC)
    lam = -1j * c * math.sin(2 * math.pi * k / nx) * nx
    e = np.exp(2j * np.pi * k * g.x.c)
    a = [0.5 + 0.2j]
    th = [np.broadcast_to((a[0] * e).real[None, None, :], g.shape).copy()]
    u = np.full(g.shape, c)
    v = np.zeros(g.shape)
    w = np.zeros((nz + 1, ny, nx))
    for n in range(12):
        a.append(a[0] * (1 + dt * lam) if n == 0 else a[n - 1] + 2 * dt * lam * a[n])
        th.append(O.scalar_step(g, p, n, th[n - 1] if n else th[0], th[n], u, v, w))
        want = np.broadcast_to((a[-1] * e).real[None, None, :], g.shape)
        np.testing.assert_allclose(th[-1], want, atol=1e-14)


def test_zero_diffusivity_adiabatic_invariants():
    """kappa = 0, adiabatic walls, divergence-free u: the leapfrog pairs keep
    sum V theta^n theta^{n+1} (skew-symmetric central flux) and sum V theta."""
    rng = np.random.default_rng(1)
    g = _grid((10, 8, 12), gamma=1.5, rng=rng)
    u, v, w = _dense_velocity(g, kmax=2)
    p = O.ScalarParams(kappa=0.0, dt=0.02, n_avg=0, bc_bot=ADIABATIC, bc_top=ADIABATIC)
    th0 = rng.standard_normal(g.shape)
    lev = O.rollout(g, p, th0, u, v, w, 12, keep=True)
    V = g.vol()
    q = [np.sum(V * lev[n] * lev[n + 1]) for n in range(1, 12)]
    np.testing.assert_allclose(q, q[0], rtol=1e-13)
    mass = [np.sum(V * t) for t in lev]
    np.testing.assert_allclose(mass, mass[0], atol=1e-14 * np.sum(V * np.abs(th0)))


def test_adiabatic_conserves_total_scalar_with_diffusion():
    """Adiabatic walls, kappa > 0, all step types: sum V theta is conserved
    (start-up, leapfrog pairs, and averaging of two equal totals)."""
    rng = np.random.default_rng(2)
    g = _grid((8, 8, 10), gamma=2.0, rng=rng)
    u, v, w = _dense_velocity(g, kmax=2)
    p = O.ScalarParams(kappa=5e-3, dt=0.01, n_avg=4, bc_bot=ADIABATIC, bc_top=ADIABATIC)
    lev = O.rollout(g, p, rng.standard_normal(g.shape), u, v, w, 9, keep=True)
    mass = [math.fsum((g.vol() * t).ravel()) for t in lev]
    np.testing.assert_allclose(mass, mass[0], atol=1e-14)


def test_free_stream_preserved():
    """A constant scalar stays constant under a divergence-free velocity when
    both walls hold the same constant."""
    g = _grid((8, 6, 10), gamma=1.0)
    u, v, w = _dense_velocity(g)
    p = O.ScalarParams(kappa=1e-2, dt=0.01, n_avg=3, t_bot=0.7, t_top=0.7)
    th = np.full(g.shape, 0.7)
    lev = O.rollout(g, p, th, u, v, w, 6, keep=True)
    for t in lev:
        np.testing.assert_allclose(t, 0.7, atol=1e-14)


# ------------------------------------------------- brute-force face-loop step
def _brute_force_step(g, p, n, th_prev, th_cur, u, v, w):
    """One step assembled cell by cell from an explicit loop over the six faces
    of every cell, the implicit system solved as a dense matrix."""
    nz, ny, nx = g.shape
    tau, ap, ac, _ = O.step_kind(n, p.n_avg, p.dt)
    lag = th_cur if n == 0 else th_prev
    N = nx * ny * nz
    idx = lambda k, j, i: (k * ny + j) * nx + i
    A = np.eye(N)
    rhs = np.zeros(N)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = idx(k, j, i)
                hx, hy, hz = g.x.h[i], g.y.h[j], g.z.h[k]
                vol = hx * hy * hz
                flux_in = 0.0    # advective volume-integrated inflow
                diff = 0.0       # explicit horizontal diffusive inflow
                # x faces: left face i (neighbour i-1), right face i+1 (neighbour i+1)
                for side, face_i, nb in ((-1, i, (i - 1) % nx), (+1, (i + 1) % nx, (i + 1) % nx)):
                    dcx = g.x.dc[face_i]
                    area = hy * hz
                    theta_f = 0.5 * (th_cur[k, j, i] + th_cur[k, j, nb])
                    flux_in += -side * u[k, j, face_i] * theta_f * area
                    diff += (lag[k, j, nb] - lag[k, j, i]) / dcx * area
                for side, face_j, nb in ((-1, j, (j - 1) % ny), (+1, (j + 1) % ny, (j + 1) % ny)):
                    dcy = g.y.dc[face_j]
                    area = hx * hz
                    theta_f = 0.5 * (th_cur[k, j, i] + th_cur[k, nb, i])
                    flux_in += -side * v[k, face_j, i] * theta_f * area
                    diff += (lag[k, nb, i] - lag[k, j, i]) / dcy * area
                # z faces: advection on interior faces only; diffusion implicit
                area = hx * hy
                for side, face_k, nb in ((-1, k, k - 1), (+1, k + 1, k + 1)):
                    if 0 <= nb < nz:
                        theta_f = 0.5 * (th_cur[k, j, i] + th_cur[nb, j, i])
                        flux_in += -side * w[face_k, j, i] * theta_f * area
                        coef = tau * p.kappa * area / g.z.dc[face_k] / vol
                        A[r, r] += coef
                        A[r, idx(nb, j, i)] -= coef
                    else:
                        wall_is_bot = nb < 0
                        bc = p.bc_bot if wall_is_bot else p.bc_top
                        if bc == DIRICHLET:
                            tw = p.t_bot if wall_is_bot else p.t_top
                            coef = tau * p.kappa * area / g.z.dc[face_k] / vol
                            A[r, r] += coef
                            rhs[r] += coef * tw
                rhs[r] += ac * th_cur[k, j, i] + (ap * th_prev[k, j, i] if n > 0 else 0.0)
                rhs[r] += tau * (flux_in + p.kappa * diff) / vol
    return np.linalg.solve(A, rhs).reshape(g.shape)


@pytest.mark.parametrize("n", [0, 1, 3])
def test_step_matches_brute_force(n):
    """Non-uniform x, y and z widths, Dirichlet bottom, adiabatic top."""
    rng = np.random.default_rng(10 + n)
    g = _grid((5, 4, 6), gamma=1.5, rng=rng)
    u, v, w = (rng.standard_normal(g.shape), rng.standard_normal(g.shape),
               rng.standard_normal((g.z.n + 1,) + g.shape[1:]))
    p = O.ScalarParams(kappa=0.05, dt=0.03, n_avg=4, t_bot=0.9, bc_top=ADIABATIC)
    tp, tc = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    got = O.scalar_step(g, p, n, tp, tc, u, v, w)
    want = _brute_force_step(g, p, n, tp, tc, u, v, w)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-13)


# ------------------------------------------------------------------- Nusselt
@pytest.mark.parametrize("gamma", [0.0, 2.5])
def test_nusselt_conduction_is_one(gamma):
    """theta = 1 - z_c: Nu = 1 on every face, both plates included; the mean
    scalar is exactly 1/2 (sum of z_c h_z telescopes to 1/2)."""
    g = _grid((6, 5, 24), gamma)
    p = O.ScalarParams.from_ra_pr(1e8, 4.38, dt=1.0)
    th = np.broadcast_to((1.0 - g.z.c)[:, None, None], g.shape).copy()
    w = np.zeros((g.z.n + 1,) + g.shape[1:])
    prof, out = O.nusselt(g, p, th, w)
    np.testing.assert_allclose(prof, 1.0, atol=1e-12)
    for key in ("nu_bot", "nu_top", "nu_vol", "nu_paper"):
        assert abs(out[key] - 1.0) < 1e-12
    assert abs(out["mean_theta"] - 0.5) < 1e-15


def test_nusselt_convective_closed_form():
    """theta = 1 - z_c + a cos(2 pi x_c), w = b cos(2 pi x_c) on interior faces:
    Nu_k = 1 + (Ra Pr)^(1/2) a b / 2 exactly (discrete mean of cos^2 is 1/2)."""
    g = _grid((12, 3, 10), 1.0)
    ra, pr = 1e6, 7.0
    p = O.ScalarParams.from_ra_pr(ra, pr, dt=1.0)
    a, b = 0.03, 0.2
    cx = np.cos(2 * np.pi * g.x.c)[None, None, :]
    th = (1.0 - g.z.c)[:, None, None] + a * cx * np.ones((1, 3, 1))
    w = b * cx * np.ones((g.z.n + 1, 3, 1))
    w[0] = w[-1] = 0.0
    prof, out = O.nusselt(g, p, th, w)
    want = 1.0 + math.sqrt(ra * pr) * a * b / 2
    np.testing.assert_allclose(prof[1:-1], want, rtol=1e-13)
    np.testing.assert_allclose([prof[0], prof[-1]], 1.0, atol=1e-12)


def test_nusselt_volume_identity():
    """Nu_vol = 1 + (Ra Pr)^(1/2) sum_k h_k <w_k theta_f>: the gradient part
    telescopes to T_bot - T_top = 1 for any scalar field."""
    rng = np.random.default_rng(3)
    g = _grid((7, 6, 15), 2.0, rng=rng)
    p = O.ScalarParams.from_ra_pr(1e7, 3.0, dt=1.0)
    th = rng.standard_normal(g.shape)
    w = rng.standard_normal((g.z.n + 1,) + g.shape[1:])
    w[0] = w[-1] = 0.0
    prof, out = O.nusselt(g, p, th, w)
    area = g.area_xy()
    conv = [np.sum(w[k] * 0.5 * (th[k - 1] + th[k]) * area) / area.sum() for k in range(1, g.z.n)]
    want = 1.0 + math.sqrt(1e7 * 3.0) * sum(g.z.dc[k] * conv[k - 1] for k in range(1, g.z.n))
    assert abs(out["nu_vol"] - want) < 1e-10 * abs(want)


# ------------------------------------------------------------------- adjoint
def _step_jacobian_apply(g, p, n, tp, tc, u, v, w, dtp, dtc, du, dv, dw):
    """J @ (dtp, dtc, du) of the step: exact by linearity (theta-part affine,
    velocity-part linear in u for fixed theta)."""
    base = O.scalar_step(g, p, n, tp, tc, u, v, w)
    jt = O.scalar_step(g, p, n, tp + dtp, tc + dtc, u, v, w) - base
    ju = O.scalar_step(g, p, n, tp, tc, u + du, v + dv, w + dw) - base
    return jt + ju


@pytest.mark.parametrize("n", [0, 1, 4])
def test_step_vjp_dot_product(n):
    rng = np.random.default_rng(20 + n)
    g = _grid((8, 7, 9), 1.5, rng=rng)
    u, v, w = _dense_velocity(g)
    p = O.ScalarParams(kappa=0.02, dt=0.02, n_avg=5)
    tp, tc = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    d = [rng.standard_normal(g.shape) for _ in range(4)] + [rng.standard_normal(w.shape)]
    d[4][0] = d[4][-1] = 0.0
    y = rng.standard_normal(g.shape)
    lhs = np.vdot(_step_jacobian_apply(g, p, n, tp, tc, u, v, w, *d), y)
    gp, gc, gu, gv, gw = O.step_vjp(g, p, n, tc, u, v, w, y)
    rhs = np.vdot(gp, d[0]) + np.vdot(gc, d[1]) + np.vdot(gu, d[2]) + np.vdot(gv, d[3]) + np.vdot(gw, d[4])
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1e-3)


def test_step_vjp_brute_force_matrix():
    """Tiny grid: the VJP equals the transpose of the Jacobian assembled column
    by column from the forward step (theta parts and velocity parts)."""
    rng = np.random.default_rng(7)
    g = _grid((3, 3, 4), 2.0, rng=rng)
    u, v, w = rng.standard_normal(g.shape), rng.standard_normal(g.shape), rng.standard_normal((5, 3, 3))
    p = O.ScalarParams(kappa=0.1, dt=0.05, n_avg=3, bc_top=ADIABATIC)
    tp, tc = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    n = 2        # averaging step: both alphas non-zero
    shapes = [g.shape, g.shape, g.shape, g.shape, w.shape]
    sizes = [int(np.prod(s)) for s in shapes]
    cols = []
    for c in range(sum(sizes)):
        e = np.zeros(sum(sizes))
        e[c] = 1.0
        parts, o = [], 0
        for s, k in zip(shapes, sizes):
            parts.append(e[o:o + k].reshape(s))
            o += k
        cols.append(_step_jacobian_apply(g, p, n, tp, tc, u, v, w, *parts).ravel())
    J = np.stack(cols, axis=1)
    y = rng.standard_normal(g.shape)
    got = np.concatenate([a.ravel() for a in O.step_vjp(g, p, n, tc, u, v, w, y)])
    want = J.T @ y.ravel()
    # the z-wall faces carry no advective flux: their velocity columns are zero
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-11)


def test_rollout_gradient_finite_differences():
    """Loss gradient of refine + N steps vs central differences (eps = 1e-3,
    FP64): exact for theta_0 directions (the loss is quadratic), O(eps^2) for
    velocity directions (divergence-free coarse curls)."""
    m = (2, 2, 2)
    g = O.Grid(inputs.uniform_faces(12), inputs.uniform_faces(10), inputs.tanh_faces(10, 1.5), m)
    U, V, W = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=2, seed=1)
    th0 = inputs.theta_initial(g.z.faces, g.x.n, g.y.n, seed=2)
    tgt = inputs.theta_initial(g.z.faces, g.x.n, g.y.n, seed=3)
    p = O.ScalarParams.from_ra_pr(1e4, 4.38, dt=0.02, n_avg=3)
    N = 6
    loss, g0, gU, gV, gW = O.rollout_loss_grad(g, p, th0, U, V, W, N, tgt)
    rng = np.random.default_rng(4)
    eps = 1e-3
    for trial in range(3):
        dth = rng.standard_normal(th0.shape)
        dU, dV, dW = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=2, seed=40 + trial)
        # theta_0 direction: the loss is quadratic, central differences are exact
        f = lambda s: O.rollout_loss_grad(g, p, th0 + s * dth, U, V, W, N, tgt)[0]
        fd = (f(eps) - f(-eps)) / (2 * eps)
        ad = np.vdot(g0, dth)
        assert abs(fd - ad) <= 1e-9 * abs(ad)
        # velocity direction: O(eps^2) truncation, removed by one Richardson step
        f = lambda s: O.rollout_loss_grad(g, p, th0, U + s * dU, V + s * dV, W + s * dW, N, tgt)[0]
        fd1 = (f(eps) - f(-eps)) / (2 * eps)
        fd2 = (f(eps / 2) - f(-eps / 2)) / eps
        ad = np.vdot(gU, dU) + np.vdot(gV, dV) + np.vdot(gW, dW)
        assert abs(fd1 - ad) <= 1e-5 * abs(ad)
        assert abs((4 * fd2 - fd1) / 3 - ad) <= 1e-9 * abs(ad)
