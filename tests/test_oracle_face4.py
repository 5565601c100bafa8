"""Pins of the oracle's fourth-order face values of the advected scalar
(Sec. 2.2: the paper's code interpolates face values to fourth order), read as
the value at the face of the polynomial whose means over the stencil cells
equal their values."""
import math

import numpy as np
import pytest
from numpy.polynomial import polynomial as P

import oracle as O
from oracle.grid import Axis
from oracle.scalar import ADIABATIC, DIRICHLET, face_values, face_weights
from paper_1805_03426_amd import inputs


def _random_faces(rng, n, lo=0.5, hi=1.8):
    h = rng.uniform(lo, hi, n)
    return np.concatenate([[0.0], np.cumsum(h)]) / h.sum()


def _dense_weights(ax, order):
    """(nf, n) matrix of the face interpolation."""
    cells, wts = face_weights(ax, order)
    M = np.zeros((cells.shape[0], ax.n))
    for f in range(cells.shape[0]):
        for s in range(4):
            M[f, cells[f, s]] += wts[f, s]
    return M


def test_uniform_weights_closed_form():
    """Uniform widths h, face at 0.  Two cells each side, cells [-2h,-h] ..
    [h,2h], cubic a + bx + cx^2 + dx^3: the four cell means give
    a = (-T0 + 7 T1 + 7 T2 - T3)/12.  Three cells [-h,0], [0,h], [h,2h],
    quadratic: T1 - T0 = b h, T2 - T1 = b h + 2 c h^2 and
    T0 = a - b h/2 + c h^2/3 give a = (2 T0 + 5 T1 - T2)/6.  Two cells: a = (T0 + T1)/2."""
    n = 8
    per = Axis(inputs.uniform_faces(n), 1, True)
    M = _dense_weights(per, 4)
    for f in range(n):
        want = np.zeros(n)
        for c, wt in zip((f - 2, f - 1, f, f + 1), (-1, 7, 7, -1)):
            want[c % n] += wt / 12
        np.testing.assert_allclose(M[f], want, atol=1e-14)
    n = 6
    wal = Axis(inputs.uniform_faces(n), 1, False)
    M = _dense_weights(wal, 4)
    assert np.all(M[0] == 0) and np.all(M[n] == 0)
    np.testing.assert_allclose(M[1, :3], np.array([2, 5, -1]) / 6, atol=1e-14)
    np.testing.assert_allclose(M[n - 1, n - 3:], np.array([-1, 5, 2]) / 6, atol=1e-14)
    for f in range(2, n - 1):
        np.testing.assert_allclose(M[f, f - 2:f + 2], np.array([-1, 7, 7, -1]) / 12, atol=1e-14)
    M2 = _dense_weights(Axis(inputs.uniform_faces(2), 1, False), 4)
    np.testing.assert_allclose(M2[1], [0.5, 0.5], atol=1e-15)
    # order 2 is the plain mean
    M = _dense_weights(per, 2)
    np.testing.assert_allclose(M[3, 2:4], [0.5, 0.5], atol=0)


def _cell_means(poly, faces):
    """Exact cell means of a polynomial (coefficients low to high) from its antiderivative."""
    F = P.polyint(poly)
    return (P.polyval(faces[1:], F) - P.polyval(faces[:-1], F)) / np.diff(faces)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_walled_faces_exact_for_cubics_and_quadratics(seed):
    rng = np.random.default_rng(seed)
    n = 9
    faces = _random_faces(rng, n)
    ax = Axis(faces, 1, False)
    cubic = rng.standard_normal(4)
    quad = rng.standard_normal(3)
    for poly, faces_exact in ((cubic, range(2, n - 1)), (quad, range(1, n))):
        got = face_values(ax, _cell_means(poly, faces), 0, 4)
        for f in faces_exact:
            assert abs(got[f] - P.polyval(faces[f], poly)) < 1e-12
    # the faces next to a wall cell use three cells: a cubic is not exact there
    got = face_values(ax, _cell_means(cubic, faces), 0, 4)
    assert abs(got[1] - P.polyval(faces[1], cubic)) > 1e-6
    assert abs(got[n - 1] - P.polyval(faces[n - 1], cubic)) > 1e-6


def test_periodic_faces_exact_for_cubics_away_from_the_seam():
    rng = np.random.default_rng(5)
    n = 10
    faces = _random_faces(rng, n)
    ax = Axis(faces, 1, True)
    cubic = rng.standard_normal(4)
    got = face_values(ax, _cell_means(cubic, faces), 0, 4)
    for f in range(2, n - 1):                       # stencils f-2..f+1 inside 0..n-1
        assert abs(got[f] - P.polyval(faces[f], cubic)) < 1e-12


def _mapped_periodic_faces(n, a=0.12):
    xi = np.arange(n + 1) / n
    return xi + a * np.sin(2 * np.pi * xi) / (2 * np.pi)


def test_fourth_order_convergence_on_a_stretched_periodic_axis():
    """Exact cell means of sin(2 pi x) + cos(4 pi x) on a smooth stretched
    periodic grid: the face error falls by ~16 per halving (4th order) across
    the seam too; the mean (order 2) falls by ~4."""
    F = lambda x: -np.cos(2 * np.pi * x) / (2 * np.pi) + np.sin(4 * np.pi * x) / (4 * np.pi)
    f = lambda x: np.sin(2 * np.pi * x) + np.cos(4 * np.pi * x)
    errs = {2: [], 4: []}
    for n in (32, 64, 128):
        faces = _mapped_periodic_faces(n)
        means = (F(faces[1:]) - F(faces[:-1])) / np.diff(faces)
        ax = Axis(faces, 1, True)
        for order in errs:
            errs[order].append(np.abs(face_values(ax, means, 0, order) - f(faces[:-1])).max())
    r4 = [errs[4][i] / errs[4][i + 1] for i in range(2)]
    r2 = [errs[2][i] / errs[2][i + 1] for i in range(2)]
    assert all(13 < r < 19 for r in r4), r4
    assert all(3.5 < r < 4.5 for r in r2), r2


def _primitive_face_value(faces_c, vals, xf):
    """Independent construction: the primitive P(x) = integral of the
    reconstruction from the first stencil edge is known at every stencil edge
    (cumulative sums of mean * width); the face value is P'(xf) of the
    interpolating polynomial through those edge points."""
    edges = np.asarray(faces_c, dtype=np.float64)
    cum = np.concatenate([[0.0], np.cumsum(np.asarray(vals) * np.diff(edges))])
    scale = edges[-1] - edges[0]
    t = (edges - xf) / scale
    coef = np.polyfit(t, cum, len(edges) - 1)
    return np.polyval(np.polyder(coef), 0.0) / scale


def _independent_faces(ax, q):
    """Face values along axis 0 of a 1-D q by the primitive construction."""
    n, f = ax.n, ax.faces
    nf = n if ax.periodic else n + 1
    out = np.zeros(nf)
    for face in range(nf):
        if not ax.periodic and face in (0, n):
            continue
        lo, hi = face - 2, face + 1
        if not ax.periodic:
            lo, hi = max(lo, 0), min(hi, n - 1)
        edges, vals = [], []
        for c in range(lo, hi + 1):
            wrap, cell = divmod(c, n)
            edges.append(f[cell] + wrap * ax.length)
            vals.append(q[cell])
        edges.append(f[(hi % n) + 1] + (hi // n) * ax.length)
        out[face] = _primitive_face_value(edges, vals, f[face])
    return out


@pytest.mark.parametrize("n,periodic", [(1, True), (2, True), (3, True), (7, True),
                                        (2, False), (3, False), (4, False), (8, False)])
def test_weights_match_the_primitive_construction(n, periodic):
    rng = np.random.default_rng(10 + n)
    ax = Axis(_random_faces(rng, n), 1, periodic)
    q = rng.standard_normal(n)
    np.testing.assert_allclose(face_values(ax, q, 0, 4), _independent_faces(ax, q), rtol=0, atol=1e-12)


def _grid(n, periodic=(True, True, False), gamma=1.5, seed=0):
    rng = np.random.default_rng(seed)
    xf = _random_faces(rng, n[0]) if not periodic[0] else inputs.uniform_faces(n[0])
    yf = _random_faces(rng, n[1])
    return O.Grid(xf, yf, inputs.tanh_faces(n[2], gamma), (1, 1, 1), periodic)


def _random_velocity(g, rng):
    nz, ny, nx = g.shape
    u = rng.standard_normal((nz, ny, g.x.nfaces()))
    v = rng.standard_normal((nz, g.y.nfaces(), nx))
    w = rng.standard_normal((nz + 1, ny, nx))
    w[0] = w[-1] = 0.0
    if not g.x.periodic:
        u[:, :, 0] = u[:, :, -1] = 0.0
    if not g.y.periodic:
        v[:, 0] = v[:, -1] = 0.0
    return u, v, w


@pytest.mark.parametrize("periodic", [(True, True, False), (False, True, False), (False, False, False)])
def test_advection4_conserves_and_keeps_constants(periodic):
    """Flux form: sum V C(theta) = 0 for any velocity (no flux through walls).
    The weights of every face sum to 1, so a constant's face values are the
    constant: C(const) = -const div(u)/V for any velocity, the same as with the
    mean, and zero for a divergence-free one."""
    rng = np.random.default_rng(3)
    g = _grid((7, 6, 9), periodic)
    u, v, w = _random_velocity(g, rng)
    th = rng.standard_normal(g.shape)
    c = O.advection(g, th, u, v, w, order=4)
    assert abs(math.fsum((c * g.vol()).ravel())) < 1e-11 * np.abs(c * g.vol()).sum()
    const = np.full(g.shape, 0.37)
    np.testing.assert_allclose(O.advection(g, const, u, v, w, order=4), O.advection(g, const, u, v, w),
                               rtol=0, atol=1e-12 * np.abs(O.advection(g, const, u, v, w)).max())
    if periodic[0] and periodic[1]:
        gr = O.Grid(inputs.uniform_faces(16), inputs.uniform_faces(12), inputs.tanh_faces(12, 1.5), (2, 2, 2))
        U, V, W = inputs.divergence_free_velocity(gr.x.cf, gr.y.cf, gr.z.cf, 2, 0.2, 4)
        uu, vv, ww = O.refine_velocity(gr, U, V, W)
        c = O.advection(gr, np.full(gr.shape, 0.37), uu, vv, ww, order=4)
        assert np.abs(c).max() < 1e-12


def test_advection4_of_a_mode_is_fourth_order():
    """Uniform u on a uniform periodic x grid, exact cell means of cos(2 pi k x):
    C theta matches the exact rate -u d/dx of the mean to O(h^4) (O(h^2) for
    the mean face value)."""
    errs = {2: [], 4: []}
    k = 3
    for nx in (32, 64, 128):
        xf = inputs.uniform_faces(nx)
        g = O.Grid(xf, inputs.uniform_faces(2), inputs.uniform_faces(2), (1, 1, 1))
        F = lambda x: np.sin(2 * np.pi * k * x) / (2 * np.pi * k)
        means = (F(xf[1:]) - F(xf[:-1])) * nx
        th = np.broadcast_to(means, g.shape).copy()
        u = np.full(g.shape, 0.7)
        v = np.zeros(g.shape)
        w = np.zeros((3, 2, nx))
        exact = -0.7 * (np.cos(2 * np.pi * k * xf[1:]) - np.cos(2 * np.pi * k * xf[:-1])) * nx
        for order in errs:
            errs[order].append(np.abs(O.advection(g, th, u, v, w, order)[0, 0] - exact).max())
    r4 = [errs[4][i] / errs[4][i + 1] for i in range(2)]
    r2 = [errs[2][i] / errs[2][i + 1] for i in range(2)]
    assert all(14 < r < 18 for r in r4), r4
    assert all(3.5 < r < 4.5 for r in r2), r2


def _brute_force_step4(g, p, n, th_prev, th_cur, u, v, w):
    """Face-loop step: advective face values from the primitive construction,
    diffusion as in the default step; dense solve of the implicit z part."""
    nz, ny, nx = g.shape
    tau, ap, ac, _ = O.step_kind(n, p.n_avg, p.dt)
    lag = th_cur if n == 0 else th_prev
    fx = np.zeros((nz, ny, g.x.nfaces()))
    fy = np.zeros((nz, g.y.nfaces(), nx))
    fz = np.zeros((nz + 1, ny, nx))
    for k in range(nz):
        for j in range(ny):
            fx[k, j] = _independent_faces(g.x, th_cur[k, j, :])
    for k in range(nz):
        for i in range(nx):
            fy[k, :, i] = _independent_faces(g.y, th_cur[k, :, i])
    for j in range(ny):
        for i in range(nx):
            fz[:, j, i] = _independent_faces(g.z, th_cur[:, j, i])
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
                net = 0.0
                ilo, ihi = i, (i + 1) % nx if g.x.periodic else i + 1
                net += (u[k, j, ihi] * fx[k, j, ihi] - u[k, j, ilo] * fx[k, j, ilo]) * hy * hz
                jlo, jhi = j, (j + 1) % ny if g.y.periodic else j + 1
                net += (v[k, jhi, i] * fy[k, jhi, i] - v[k, jlo, i] * fy[k, jlo, i]) * hx * hz
                net += (w[k + 1, j, i] * fz[k + 1, j, i] - w[k, j, i] * fz[k, j, i]) * hx * hy
                diff = 0.0
                # x and y: neighbour across the low face (index c) and the high face (c + 1);
                # no flux through a wall
                for c, nc_, per, area, dcs, nbval in (
                        (i, nx, g.x.periodic, hy * hz, g.x.dc, lambda m: lag[k, j, m]),
                        (j, ny, g.y.periodic, hx * hz, g.y.dc, lambda m: lag[k, m, i])):
                    for nb, face in ((c - 1, c), (c + 1, c + 1)):
                        if per:
                            diff += (nbval(nb % nc_) - nbval(c)) / dcs[face % nc_] * area
                        elif 0 <= nb < nc_:
                            diff += (nbval(nb) - nbval(c)) / dcs[face] * area
                for side, fk, nb in ((-1, k, k - 1), (+1, k + 1, k + 1)):
                    coef = tau * p.kappa * hx * hy / g.z.dc[fk] / vol
                    if 0 <= nb < nz:
                        A[r, r] += coef
                        A[r, idx(nb, j, i)] -= coef
                    elif (p.bc_bot if nb < 0 else p.bc_top) == DIRICHLET:
                        A[r, r] += coef
                        rhs[r] += coef * (p.t_bot if nb < 0 else p.t_top)
                rhs[r] += ac * th_cur[k, j, i] + (ap * th_prev[k, j, i] if n > 0 else 0.0)
                rhs[r] += tau * (-net + p.kappa * diff) / vol
    return np.linalg.solve(A, rhs).reshape(g.shape)


@pytest.mark.parametrize("periodic,n", [((True, True, False), 0), ((True, True, False), 1),
                                        ((False, True, False), 3), ((False, False, False), 1)])
def test_step4_matches_brute_force(periodic, n):
    rng = np.random.default_rng(60 + n)
    g = _grid((6, 5, 6), periodic, seed=n)
    u, v, w = _random_velocity(g, rng)
    p = O.ScalarParams(kappa=0.05, dt=0.02, n_avg=4, t_bot=0.9, bc_top=ADIABATIC, face_order=4)
    tp, tc = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    np.testing.assert_allclose(O.scalar_step(g, p, n, tp, tc, u, v, w),
                               _brute_force_step4(g, p, n, tp, tc, u, v, w), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("periodic,n", [((True, True, False), 0), ((True, True, False), 2),
                                        ((False, False, False), 1), ((True, False, False), 4)])
def test_step4_vjp_dot_product(periodic, n):
    rng = np.random.default_rng(70 + n)
    g = _grid((7, 6, 8), periodic, seed=n)
    u, v, w = _random_velocity(g, rng)
    p = O.ScalarParams(kappa=0.02, dt=0.02, n_avg=5, t_bot=0.7, face_order=4, z_explicit=0.5 if n == 2 else 0.0)
    tp, tc = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    du, dv, dw = _random_velocity(g, rng)
    d = [rng.standard_normal(g.shape), rng.standard_normal(g.shape), du, dv, dw]
    y = rng.standard_normal(g.shape)
    base = O.scalar_step(g, p, n, tp, tc, u, v, w)
    jt = O.scalar_step(g, p, n, tp + d[0], tc + d[1], u, v, w) - base
    ju = O.scalar_step(g, p, n, tp, tc, u + d[2], v + d[3], w + d[4]) - base
    lhs = np.vdot(jt + ju, y)
    gp, gc, gu, gv, gw = O.step_vjp(g, p, n, tc, u, v, w, y)
    rhs = np.vdot(gp, d[0]) + np.vdot(gc, d[1]) + np.vdot(gu, d[2]) + np.vdot(gv, d[3]) + np.vdot(gw, d[4])
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1e-3)
