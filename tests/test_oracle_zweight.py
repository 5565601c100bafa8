"""Pins of the oracle's partly explicit z diffusion: a share w of the vertical
diffusion taken explicit on the lagged level (w = 1/2 is Crank-Nicolson across
the step's time span; w = 0 is the default fully implicit step)."""
import math

import numpy as np
import pytest

import oracle as O
from oracle.scalar import ADIABATIC, DIRICHLET, lz0, lz0_transpose
from paper_1805_03426_amd import inputs

W_HALF = 0.5


def _grid(n, gamma=0.0, rng=None, periodic=(True, True, False)):
    nx, ny, nz = n
    if rng is None:
        xf, yf = inputs.uniform_faces(nx), inputs.uniform_faces(ny)
    else:
        hx, hy = rng.uniform(0.6, 1.6, nx), rng.uniform(0.6, 1.6, ny)
        xf = np.concatenate([[0], np.cumsum(hx)]) / hx.sum()
        yf = np.concatenate([[0], np.cumsum(hy)]) / hy.sum()
    return O.Grid(xf, yf, inputs.tanh_faces(nz, gamma), (1, 1, 1), periodic)


def test_lz0_is_the_face_form_and_its_transpose():
    """Lz0 theta + bz is the face-flux divergence of the z diffusion (Dirichlet
    wall at half a cell), and lz0_transpose is the transpose of the assembled
    matrix (not symmetric on a stretched grid)."""
    rng = np.random.default_rng(1)
    g = _grid((3, 2, 9), gamma=2.0)
    p = O.ScalarParams(kappa=1.0, dt=1.0, t_bot=0.8, t_top=0.1, bc_top=ADIABATIC)
    th = rng.standard_normal(g.shape)
    hz, dc = g.z.h, g.z.dc
    nz = g.z.n
    want = np.zeros_like(th)
    for k in range(nz):
        up = (th[k + 1] - th[k]) / dc[k + 1] if k < nz - 1 else 0.0 * th[k]
        if k > 0:
            dn = (th[k] - th[k - 1]) / dc[k]
        else:
            dn = (th[0] - p.t_bot) / dc[0]
        want[k] = (up - dn) / hz[k]
    _, _, _, bz = O.z_matrix(g, 1.0, p)
    np.testing.assert_allclose(lz0(g, p, th) + bz[:, None, None], want, rtol=1e-13, atol=1e-12)
    M = np.stack([lz0(g, p, np.eye(nz)[:, q][:, None, None] * np.ones((1, 1, 1)))[:, 0, 0] for q in range(nz)], axis=1)
    MT = np.stack([lz0_transpose(g, p, np.eye(nz)[:, q][:, None, None] * np.ones((1, 1, 1)))[:, 0, 0]
                   for q in range(nz)], axis=1)
    np.testing.assert_allclose(MT, M.T, rtol=1e-14, atol=1e-12)
    assert np.abs(M - M.T).max() > 1.0          # really not symmetric here


@pytest.mark.parametrize("kvec", [(1, 2, 1), (2, 1, 5)])
def test_fourier_mode_recurrence_with_explicit_share(kvec):
    """Uniform grid, pure diffusion: conduction + a cos.cos.sin mode follows the
    theta-weighted recurrences
      start-up  a1 = a0 (1 + dt k lh + w dt k lz) / (1 - (1-w) dt k lz)
      leapfrog  a_{n+1} = a_{n-1} (1 + 2dt k lh + w 2dt k lz) / (1 - (1-w) 2dt k lz)
      averaging a_{n+1} = [(a_{n-1} + a_n)/2 + 1.5dt k (lh + w lz) a_{n-1}] / (1 - (1-w) 1.5dt k lz)."""
    kx, ky, kz = kvec
    nx, ny, nz = 12, 10, 14
    g = _grid((nx, ny, nz))
    kappa, dt, wz = 3e-3, 0.02, W_HALF
    p = O.ScalarParams(kappa=kappa, dt=dt, n_avg=4, z_explicit=wz)
    lh = -4 * math.sin(math.pi * kx / nx) ** 2 * nx * nx - 4 * math.sin(math.pi * ky / ny) ** 2 * ny * ny
    lz = -4 * math.sin(math.pi * kz / (2 * nz)) ** 2 * nz * nz
    base = np.broadcast_to((1.0 - g.z.c)[:, None, None], g.shape)
    mode = (np.cos(2 * np.pi * kx * g.x.c)[None, None, :] * np.cos(2 * np.pi * ky * g.y.c)[None, :, None]
            * np.sin(np.pi * kz * g.z.c)[:, None, None])
    a = [0.37]
    th = [base + a[0] * mode]
    u = np.zeros(g.shape)
    w = np.zeros((nz + 1, ny, nx))
    for n in range(10):
        tau, ap, ac, kind = O.step_kind(n, p.n_avg, dt)
        tk = tau * kappa
        lag = a[0] if n == 0 else a[n - 1]
        prev = 0.0 if n == 0 else a[n - 1]
        a.append((ap * prev + ac * a[n] + tk * (lh + wz * lz) * lag) / (1 - (1 - wz) * tk * lz))
        th.append(O.scalar_step(g, p, n, th[n - 1] if n else th[0], th[n], u, u, w))
        np.testing.assert_allclose(th[-1], base + a[-1] * mode, rtol=0, atol=1e-14)


def test_crank_nicolson_is_second_order_in_time():
    """With w = 1/2 the amplification over a leapfrog interval matches
    exp(2 dt k lz) to O(dt^3) (one order better than w = 0)."""
    nz = 16
    lz = -4 * math.sin(math.pi / (2 * nz)) ** 2 * nz * nz
    kappa = 1e-2
    errs = {0.0: [], W_HALF: []}
    for dt in (0.04, 0.02, 0.01):
        x = 2 * dt * kappa * lz
        for wz in errs:
            amp = (1 + wz * x) / (1 - (1 - wz) * x)
            errs[wz].append(abs(amp - math.exp(x)))
    ratio_half = errs[W_HALF][0] / errs[W_HALF][1], errs[W_HALF][1] / errs[W_HALF][2]
    ratio_zero = errs[0.0][0] / errs[0.0][1], errs[0.0][1] / errs[0.0][2]
    assert all(7.0 < r < 9.0 for r in ratio_half) and all(3.5 < r < 4.5 for r in ratio_zero)


@pytest.mark.parametrize("n", [0, 1, 3])
def test_conduction_fixed_point_and_conservation(n):
    g = _grid((5, 4, 9), gamma=2.0)
    p = O.ScalarParams(kappa=0.02, dt=0.01, n_avg=4, z_explicit=W_HALF, t_bot=1.0, t_top=0.0)
    th = np.broadcast_to(1.0 - g.z.c[:, None, None], g.shape).copy()
    zero = np.zeros(g.shape), np.zeros(g.shape), np.zeros((g.z.n + 1,) + g.shape[1:])
    assert np.abs(O.scalar_step(g, p, n, th, th, *zero) - th).max() < 1e-14
    rng = np.random.default_rng(2)
    pa = O.ScalarParams(kappa=0.02, dt=0.01, n_avg=4, z_explicit=W_HALF, bc_bot=ADIABATIC, bc_top=ADIABATIC)
    t0, t1 = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    vol = g.vol()
    out = O.scalar_step(g, pa, n, t0, t1, *zero)
    _, ap, ac, _ = O.step_kind(n, 4, 0.01)
    # closed plates: the volume integral only carries the time weights over
    want = math.fsum((ac * t1 * vol).ravel()) + (math.fsum((ap * t0 * vol).ravel()) if n else 0.0)
    assert abs(math.fsum((out * vol).ravel()) - want) < 1e-12


def _brute_force_step(g, p, n, th_prev, th_cur, u, v, w):
    """Face-loop step with the z diffusion split: (1-w) implicit on the new
    level, w explicit on the lagged level; dense solve."""
    nz, ny, nx = g.shape
    tau, ap, ac, _ = O.step_kind(n, p.n_avg, p.dt)
    lag = th_cur if n == 0 else th_prev
    wz = p.z_explicit
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
                flux_in, diff = 0.0, 0.0
                for side, fi, nb in ((-1, i, (i - 1) % nx), (+1, (i + 1) % nx, (i + 1) % nx)):
                    flux_in += -side * u[k, j, fi] * 0.5 * (th_cur[k, j, i] + th_cur[k, j, nb]) * hy * hz
                    diff += (lag[k, j, nb] - lag[k, j, i]) / g.x.dc[fi] * hy * hz
                for side, fj, nb in ((-1, j, (j - 1) % ny), (+1, (j + 1) % ny, (j + 1) % ny)):
                    flux_in += -side * v[k, fj, i] * 0.5 * (th_cur[k, j, i] + th_cur[k, nb, i]) * hx * hz
                    diff += (lag[k, nb, i] - lag[k, j, i]) / g.y.dc[fj] * hx * hz
                area = hx * hy
                for side, fk, nb in ((-1, k, k - 1), (+1, k + 1, k + 1)):
                    coef = tau * p.kappa * area / g.z.dc[fk] / vol
                    if 0 <= nb < nz:
                        flux_in += -side * w[fk, j, i] * 0.5 * (th_cur[k, j, i] + th_cur[nb, j, i]) * area
                        A[r, r] += (1 - wz) * coef
                        A[r, idx(nb, j, i)] -= (1 - wz) * coef
                        rhs[r] += wz * coef * (lag[nb, j, i] - lag[k, j, i])
                    else:
                        bot = nb < 0
                        if (p.bc_bot if bot else p.bc_top) == DIRICHLET:
                            tw = p.t_bot if bot else p.t_top
                            A[r, r] += (1 - wz) * coef
                            rhs[r] += (1 - wz) * coef * tw + wz * coef * (tw - lag[k, j, i])
                rhs[r] += ac * th_cur[k, j, i] + (ap * th_prev[k, j, i] if n > 0 else 0.0)
                rhs[r] += tau * (flux_in + p.kappa * diff) / vol
    return np.linalg.solve(A, rhs).reshape(g.shape)


@pytest.mark.parametrize("n", [0, 1, 3])
def test_step_matches_brute_force_with_explicit_share(n):
    rng = np.random.default_rng(40 + n)
    g = _grid((5, 4, 6), gamma=1.5, rng=rng)
    u, v, w = (rng.standard_normal(g.shape), rng.standard_normal(g.shape),
               rng.standard_normal((g.z.n + 1,) + g.shape[1:]))
    p = O.ScalarParams(kappa=0.05, dt=0.03, n_avg=4, t_bot=0.9, bc_top=ADIABATIC, z_explicit=0.3)
    tp, tc = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    np.testing.assert_allclose(O.scalar_step(g, p, n, tp, tc, u, v, w),
                               _brute_force_step(g, p, n, tp, tc, u, v, w), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("n", [0, 1, 4])
def test_step_vjp_dot_product_with_explicit_share(n):
    rng = np.random.default_rng(50 + n)
    g = _grid((7, 6, 9), gamma=1.5, rng=rng)
    u, v = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    w = rng.standard_normal((g.z.n + 1,) + g.shape[1:])
    w[0] = w[-1] = 0.0
    p = O.ScalarParams(kappa=0.02, dt=0.02, n_avg=5, z_explicit=W_HALF, t_bot=0.7)
    tp, tc = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    d = [rng.standard_normal(g.shape) for _ in range(4)] + [rng.standard_normal(w.shape)]
    d[4][0] = d[4][-1] = 0.0
    y = rng.standard_normal(g.shape)
    base = O.scalar_step(g, p, n, tp, tc, u, v, w)
    jt = O.scalar_step(g, p, n, tp + d[0], tc + d[1], u, v, w) - base
    ju = O.scalar_step(g, p, n, tp, tc, u + d[2], v + d[3], w + d[4]) - base
    lhs = np.vdot(jt + ju, y)
    gp, gc, gu, gv, gw = O.step_vjp(g, p, n, tc, u, v, w, y)
    rhs = np.vdot(gp, d[0]) + np.vdot(gc, d[1]) + np.vdot(gu, d[2]) + np.vdot(gv, d[3]) + np.vdot(gw, d[4])
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1e-3)
