"""Pins of the oracle's scalar step with adiabatic no-slip side walls in x
and/or y (the paper's cube, Sec. 4): closed-form Neumann modes, conservation,
free stream on a refined walled velocity, a brute-force face loop, adjoint
dot products, and Nu_T."""
import math

import numpy as np
import pytest

import oracle as O
from oracle.intergrid import thermal_dissipation
from oracle.scalar import ADIABATIC, DIRICHLET
from paper_1805_03426_amd import inputs

EPS = np.finfo(np.float64).eps
WALLS = [(False, True), (True, False), (False, False)]   # (periodic x, periodic y)


def _faces(n, rng):
    if rng is None:
        return inputs.uniform_faces(n)
    h = rng.uniform(0.6, 1.6, n)
    return np.concatenate([[0.0], np.cumsum(h)]) / h.sum()


def _grid(n, per, gamma=1.5, rng=None, m=(1, 1, 1)):
    nx, ny, nz = n
    return O.Grid(_faces(nx, rng), _faces(ny, rng), inputs.tanh_faces(nz, gamma), m,
                  periodic=(per[0], per[1], False))


def _random_velocity(g, rng, zero_walls=True):
    u = rng.standard_normal((g.z.n, g.y.n, g.x.nfaces()))
    v = rng.standard_normal((g.z.n, g.y.nfaces(), g.x.n))
    w = rng.standard_normal((g.z.n + 1, g.y.n, g.x.n))
    w[0] = w[-1] = 0.0
    if zero_walls:
        if not g.x.periodic:
            u[:, :, 0] = u[:, :, -1] = 0.0
        if not g.y.periodic:
            v[:, 0] = v[:, -1] = 0.0
    return u, v, w


# ------------------------------------------------------------ closed forms
@pytest.mark.parametrize("k", [1, 3, 7])
def test_neumann_cosine_mode_is_an_eigenvector(k):
    """On a uniform walled axis, cos(pi k x / L) sampled at the cell centres is
    an eigenvector of the adiabatic finite-volume Laplacian with eigenvalue
    -4 sin^2(pi k / (2 n)) / h^2 (closed form of the Neumann second difference)."""
    n = 16
    g = _grid((n, n, 4), (False, False), gamma=0.0)
    h = 1.0 / n
    lam = -4.0 * math.sin(math.pi * k / (2 * n)) ** 2 / h ** 2
    thx = np.broadcast_to(np.cos(math.pi * k * g.x.c)[None, None, :], g.shape).copy()
    np.testing.assert_allclose(O.lap_h(g, thx), lam * thx, rtol=0, atol=1e-11 * abs(lam))
    thy = np.broadcast_to(np.cos(math.pi * k * g.y.c)[None, :, None], g.shape).copy()
    np.testing.assert_allclose(O.lap_h(g, thy), lam * thy, rtol=0, atol=1e-11 * abs(lam))


def test_neumann_mode_decays_by_the_step_recurrence():
    """At rest with adiabatic plates, a cos(pi x)cos(pi y) mode decays by the
    exact start-up and leapfrog amplification factors of the step."""
    n = 12
    g = _grid((n, n, 5), (False, False), gamma=0.0)
    h = 1.0 / n
    lam_h = 2 * (-4.0 * math.sin(math.pi / (2 * n)) ** 2 / h ** 2)
    p = O.ScalarParams(kappa=0.01, dt=0.004, n_avg=0, bc_bot=ADIABATIC, bc_top=ADIABATIC)
    mode = np.cos(math.pi * g.x.c)[None, None, :] * np.cos(math.pi * g.y.c)[None, :, None]
    th0 = np.broadcast_to(mode, g.shape).copy()
    u, v, w = np.zeros((5, n, n + 1)), np.zeros((5, n + 1, n)), np.zeros((6, n, n))
    levels = O.rollout(g, p, th0, u, v, w, 4, keep=True)
    a = [1.0, 1.0 + p.dt * p.kappa * lam_h]
    for _ in range(3):
        a.append(a[-2] * (1.0 + 2 * p.dt * p.kappa * lam_h))
    for q in range(5):
        np.testing.assert_allclose(levels[q], a[q] * th0, rtol=0, atol=1e-13)


# -------------------------------------------------------------- invariants
@pytest.mark.parametrize("per", WALLS)
def test_walls_conserve_total_scalar(per):
    """Adiabatic side walls and plates: sum V theta is unchanged by every step
    type for any face velocity (fluxes telescope, walls carry none), even with
    non-zero values stored on the wall faces."""
    rng = np.random.default_rng(3)
    g = _grid((6, 5, 7), per, rng=rng)
    u, v, w = _random_velocity(g, rng, zero_walls=False)
    p = O.ScalarParams(kappa=0.03, dt=0.01, n_avg=3, bc_bot=ADIABATIC, bc_top=ADIABATIC)
    th0 = rng.standard_normal(g.shape)
    vol = g.vol()
    total = math.fsum((th0 * vol).ravel())
    for lvl in O.rollout(g, p, th0, 0.1 * u, 0.1 * v, 0.1 * w, 6, keep=True):
        assert abs(math.fsum((lvl * vol).ravel()) - total) < 1e-13 * math.fsum(np.abs(th0 * vol).ravel())


@pytest.mark.parametrize("per", [(False, True), (False, False)])
def test_free_stream_on_refined_walled_velocity(per):
    """A coarse field from a stream function that vanishes on the x walls and the
    plates (no flow through any wall), refined with walled axes, keeps a uniform
    scalar uniform: every dense cell must be divergence-free and no wall may
    carry flux."""
    g = _grid((8, 6, 6), per, m=(2, 2, 2))
    X, Z = g.x.cf, g.z.cf
    ncx, ncy, ncz = g.x.nc, g.y.nc, g.z.nc
    # psi(x, z) = sin(pi x) sin(pi z) on the coarse edges: u = dpsi/dz, w = -dpsi/dx (Stokes)
    psi = np.sin(np.pi * X)[None, :] * np.sin(np.pi * Z)[:, None]          # (ncz+1, ncx+1)
    Uxz = (psi[1:, :] - psi[:-1, :]) / np.diff(Z)[:, None]                 # x faces (ncz, ncx+1)
    Wxz = -(psi[:, 1:] - psi[:, :-1]) / np.diff(X)[None, :]                # z faces (ncz+1, ncx)
    U = np.broadcast_to(Uxz[:, None, :], (ncz, ncy, ncx + 1)).copy()
    V = np.zeros((ncz, g.y.ncfaces(), ncx))
    W = np.broadcast_to(Wxz[:, None, :], (ncz + 1, ncy, ncx)).copy()
    u, v, w = O.refine_velocity(g, U, V, W)
    div, tot = O.divergence(g, u, v, w)
    assert np.max(np.abs(div) / tot) < 64 * EPS
    p = O.ScalarParams(kappa=1e-3, dt=0.01, n_avg=4, bc_bot=ADIABATIC, bc_top=ADIABATIC)
    out = O.rollout(g, p, np.full(g.shape, 0.625), u, v, w, 5)
    assert np.abs(out - 0.625).max() < 1e-14


@pytest.mark.parametrize("per", WALLS)
def test_conduction_fixed_point_with_walls(per):
    g = _grid((5, 4, 8), per, gamma=2.0)
    p = O.ScalarParams(kappa=0.02, dt=0.01, n_avg=3)
    th = np.broadcast_to(1.0 - g.z.c[:, None, None], g.shape).copy()
    rng = np.random.default_rng(4)
    u, v, w = _random_velocity(g, rng)
    for n in range(4):
        out = O.scalar_step(g, p, n, th, th, 0 * u, 0 * v, 0 * w)
        assert np.abs(out - th).max() < 1e-14


# -------------------------------------------------------------- brute force
def _brute_force_step(g, p, n, th_prev, th_cur, u, v, w):
    """One step from an explicit loop over the six faces of every cell: a face
    on a side wall carries nothing; the implicit z system solved densely."""
    nz, ny, nx = g.shape
    px, py = g.x.periodic, g.y.periodic
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
                flux_in = 0.0
                diff = 0.0
                for side in (-1, +1):
                    # x face: index of the face and of the neighbour across it
                    face = i if side < 0 else i + 1
                    nb = i + side
                    if px:
                        face %= nx
                        nb %= nx
                    if 0 <= nb < nx:
                        area = hy * hz
                        flux_in += -side * u[k, j, face] * 0.5 * (th_cur[k, j, i] + th_cur[k, j, nb]) * area
                        diff += (lag[k, j, nb] - lag[k, j, i]) / g.x.dc[face] * area
                    face = j if side < 0 else j + 1
                    nb = j + side
                    if py:
                        face %= ny
                        nb %= ny
                    if 0 <= nb < ny:
                        area = hx * hz
                        flux_in += -side * v[k, face, i] * 0.5 * (th_cur[k, j, i] + th_cur[k, nb, i]) * area
                        diff += (lag[k, nb, i] - lag[k, j, i]) / g.y.dc[face] * area
                area = hx * hy
                for side, face_k, nb in ((-1, k, k - 1), (+1, k + 1, k + 1)):
                    if 0 <= nb < nz:
                        flux_in += -side * w[face_k, j, i] * 0.5 * (th_cur[k, j, i] + th_cur[nb, j, i]) * area
                        coef = tau * p.kappa * area / g.z.dc[face_k] / vol
                        A[r, r] += coef
                        A[r, idx(nb, j, i)] -= coef
                    else:
                        bot = nb < 0
                        if (p.bc_bot if bot else p.bc_top) == DIRICHLET:
                            coef = tau * p.kappa * area / g.z.dc[face_k] / vol
                            A[r, r] += coef
                            rhs[r] += coef * (p.t_bot if bot else p.t_top)
                rhs[r] += ac * th_cur[k, j, i] + (ap * th_prev[k, j, i] if n > 0 else 0.0)
                rhs[r] += tau * (flux_in + p.kappa * diff) / vol
    return np.linalg.solve(A, rhs).reshape(g.shape)


@pytest.mark.parametrize("per,n", [((False, True), 0), ((True, False), 1), ((False, False), 2)])
def test_step_matches_brute_force_with_walls(per, n):
    rng = np.random.default_rng(30 + n)
    g = _grid((5, 4, 6), per, rng=rng)
    u, v, w = _random_velocity(g, rng)
    p = O.ScalarParams(kappa=0.05, dt=0.03, n_avg=3, t_bot=0.9, bc_top=ADIABATIC)
    tp, tc = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    got = O.scalar_step(g, p, n, tp, tc, u, v, w)
    want = _brute_force_step(g, p, n, tp, tc, u, v, w)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-13)


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("per,n", [((False, True), 0), ((True, False), 1), ((False, False), 4)])
def test_step_vjp_dot_product_with_walls(per, n):
    rng = np.random.default_rng(40 + n)
    g = _grid((7, 6, 8), per, rng=rng)
    u, v, w = _random_velocity(g, rng)
    p = O.ScalarParams(kappa=0.02, dt=0.02, n_avg=5)
    tp, tc = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    d = [rng.standard_normal(g.shape), rng.standard_normal(g.shape)]
    du, dv, dw = _random_velocity(g, rng)
    y = rng.standard_normal(g.shape)
    base = O.scalar_step(g, p, n, tp, tc, u, v, w)
    jt = O.scalar_step(g, p, n, tp + d[0], tc + d[1], u, v, w) - base
    ju = O.scalar_step(g, p, n, tp, tc, u + du, v + dv, w + dw) - base
    lhs = np.vdot(jt + ju, y)
    gp, gc, gu, gv, gw = O.step_vjp(g, p, n, tc, u, v, w, y)
    rhs = np.vdot(gp, d[0]) + np.vdot(gc, d[1]) + np.vdot(gu, du) + np.vdot(gv, dv) + np.vdot(gw, dw)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1e-3)
    # wall faces carry no flux, so their velocity gradient is zero
    if not per[0]:
        assert np.all(gu[:, :, 0] == 0) and np.all(gu[:, :, -1] == 0)
    if not per[1]:
        assert np.all(gv[:, 0] == 0) and np.all(gv[:, -1] == 0)


# ---------------------------------------------------------------------- Nu_T
@pytest.mark.parametrize("per", WALLS)
def test_dissipation_with_walls(per):
    """Conduction gives Nu_T = 1; the face sum obeys summation by parts with the
    walled diffusion operators and the plate fluxes."""
    rng = np.random.default_rng(9)
    g = _grid((5, 4, 7), per, rng=rng)
    p = O.ScalarParams.from_ra_pr(1e7, 2.0, 1e-3, t_bot=1.3, t_top=-0.2)
    cond = np.broadcast_to(1.0 - g.z.c[:, None, None], g.shape).copy()
    pc = O.ScalarParams.from_ra_pr(1e7, 2.0, 1e-3)
    assert abs(thermal_dissipation(g, pc, cond)["nu_t"] - 1.0) < 32 * EPS
    th = rng.standard_normal(g.shape)
    vol = g.vol()
    sub, diag, sup, bz = O.z_matrix(g, 1.0, p)
    lz0 = th - diag[:, None, None] * th
    lz0[1:] -= sub[1:, None, None] * th[:-1]
    lz0[:-1] -= sup[:-1, None, None] * th[1:]
    lth = O.lap_h(g, th) + lz0 + bz[:, None, None]
    _, nu = O.nusselt(g, p, th, np.zeros((g.z.n + 1, g.y.n, g.x.n)))
    atot = math.fsum(g.area_xy().ravel())
    rhs = -math.fsum((th * lth * vol).ravel()) + atot * (p.t_bot * nu["nu_bot"] - p.t_top * nu["nu_top"])
    d = thermal_dissipation(g, p, th)
    lhs = (d["gx2"] + d["gy2"] + d["gz2"]) * math.fsum(vol.ravel())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
