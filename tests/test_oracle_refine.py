"""Pins of the oracle's refinement (paper Sec. 3.2, Eqs. 12-19) to closed forms,
quadrature, invariants and brute force -- nothing here re-runs the oracle's own
formulas."""
import os

import numpy as np
import pytest
from scipy.integrate import quad

import oracle as O
from oracle.refine import split
from paper_1805_03426_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EPS = np.finfo(np.float64).eps


def _golden_r():
    out = {}
    for line in open(os.path.join(GOLDEN, "r_uniform.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        m, row, a, b, c, d = (int(t) for t in line.split())
        out.setdefault(m, {})[row] = np.array([a, b, c], dtype=np.float64) / d
    return {m: np.stack([rows[r] for r in sorted(rows)]) for m, rows in out.items()}


def _stretched_faces(n, rng, lo=0.0, hi=1.0):
    h = rng.uniform(0.5, 2.0, n)
    f = np.concatenate([[0.0], np.cumsum(h)])
    return lo + (hi - lo) * f / f[-1]


# ----------------------------------------------------------------- R matrices
@pytest.mark.parametrize("m", [2, 3])
@pytest.mark.parametrize("periodic", [True, False])
def test_r_uniform_closed_form(m, periodic):
    """Uniform grid: R equals the hand-derived closed form (interior cells)."""
    want = _golden_r()[m]
    ax = O.Axis(np.linspace(0.0, 1.0, 8 * m + 1), m, periodic)
    cells = range(8) if periodic else range(1, 7)
    for I in cells:
        np.testing.assert_allclose(O.r_matrix(ax, I), want, rtol=0, atol=4 * EPS)


@pytest.mark.parametrize("m", [2, 3, 4])
@pytest.mark.parametrize("periodic", [True, False])
def test_r_reproduces_quadratics_by_quadrature(m, periodic):
    """Random stretched grid: coarse means of a random quadratic, split by R, equal
    its sub-interval means computed by adaptive quadrature (Eqs. 12, 16)."""
    rng = np.random.default_rng(11 + m)
    nc = 7
    faces = _stretched_faces(nc * m, rng)
    ax = O.Axis(faces, m, periodic)
    coef = rng.standard_normal(3)
    f = lambda x: coef[0] + coef[1] * x + coef[2] * x * x
    mean = lambda a, b: quad(f, a, b, epsabs=1e-15, epsrel=1e-13)[0] / (b - a)
    cells = range(1, nc - 1) if periodic else range(nc)   # a periodic stencil wraps the poly
    for I in cells:
        s = O.stencil_start(ax, I)
        q = np.array([mean(ax.cf[s + r], ax.cf[s + r + 1]) for r in range(3)])
        sub = ax.faces[I * m:(I + 1) * m + 1]
        want = np.array([mean(sub[p], sub[p + 1]) for p in range(m)])
        np.testing.assert_allclose(O.r_matrix(ax, I) @ q, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("m", [2, 3, 5])
def test_r_row_sums_and_flux(m):
    """Every row sums to 1 (constants kept); sum_p hs_p R[p,:] = H e_centre
    (the coarse face flux is split without loss, Sec. 3.2)."""
    rng = np.random.default_rng(5)
    for periodic in (True, False):
        ax = O.Axis(_stretched_faces(6 * m, rng), m, periodic)
        for I in range(ax.nc):
            R = O.r_matrix(ax, I)
            np.testing.assert_allclose(R.sum(axis=1), 1.0, atol=1e-13)
            hs = ax.h[I * m:(I + 1) * m]
            centre = I - O.stencil_start(ax, I)
            e = np.zeros(3)
            e[centre] = 1.0
            np.testing.assert_allclose(hs @ R / ax.H[I], e, atol=1e-13)


def test_r_m1_identity():
    ax = O.Axis(np.linspace(0, 1, 9), 1, True)
    for I in range(8):
        assert np.array_equal(O.r_matrix(ax, I), [[0.0, 1.0, 0.0]])


def test_r_periodic_wrap_is_shift_invariant():
    """On a uniform periodic axis R is the same for every cell, wrapped or not."""
    ax = O.Axis(np.linspace(0, 1, 13), 3, True)
    R0 = O.r_matrix(ax, 1)
    for I in (0, 3):
        np.testing.assert_allclose(O.r_matrix(ax, I), R0, atol=4 * EPS)


# ----------------------------------------------------------------- refinement
def _grid(nc, m, gamma=0.0, periodic=(True, True, False), rng=None):
    ncx, ncy, ncz = nc
    mx, my, mz = m
    if rng is None:
        xf = inputs.uniform_faces(ncx * mx)
        yf = inputs.uniform_faces(ncy * my)
    else:
        xf = _stretched_faces(ncx * mx, rng)
        yf = _stretched_faces(ncy * my, rng)
    zf = inputs.tanh_faces(ncz * mz, gamma)
    return O.Grid(xf, yf, zf, m, periodic), (xf, yf, zf)


def _coarse_divergence(g, U, V, W):
    cg = O.Grid(g.x.cf, g.y.cf, g.z.cf, (1, 1, 1), (g.x.periodic, g.y.periodic, False))
    d, _ = O.divergence(cg, U, V, W)
    return d


@pytest.mark.parametrize("m", [(2, 2, 2), (3, 2, 4), (1, 3, 2)])
def test_refined_field_is_divergence_free(m):
    """The generator's coarse field (exactly divergence-free) refines to a dense
    field whose every cell has zero net flux up to rounding (Sec. 3.2 claims
    ~1e-17 absolute in double precision)."""
    nc = (12, 10, 9)
    g, (xf, yf, zf) = _grid(nc, m, gamma=1.5)
    U, V, W = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=4, seed=1)
    assert np.abs(_coarse_divergence(g, U, V, W)).max() < 1e-15
    u, v, w = O.refine_velocity(g, U, V, W)
    div, tot = O.divergence(g, u, v, w)
    assert np.max(np.abs(div) / tot) < 64 * EPS
    assert np.abs(div).max() < 1e-16
    assert np.all(w[0] == 0.0) and np.all(w[-1] == 0.0)


@pytest.mark.parametrize("periodic", [(True, True, False), (False, False, False)])
def test_closure_residual_is_coarse_divergence(periodic):
    """Random (not divergence-free) coarse field: every dense cell but the last
    sub-cell of each coarse cell has zero net flux, and the last one carries the
    coarse cell's divergence (the splits conserve each coarse face's flux)."""
    rng = np.random.default_rng(3)
    m = (2, 3, 2)
    g, _ = _grid((5, 4, 6), m, gamma=1.0, periodic=periodic, rng=rng)
    U = rng.standard_normal((g.z.nc, g.y.nc, g.x.ncfaces()))
    V = rng.standard_normal((g.z.nc, g.y.ncfaces(), g.x.nc))
    W = rng.standard_normal((g.z.nc + 1, g.y.nc, g.x.nc))
    u, v, w = O.refine_velocity(g, U, V, W)
    div, _ = O.divergence(g, u, v, w)
    dc = _coarse_divergence(g, U, V, W)
    mx, my, mz = m
    d6 = div.reshape(g.z.nc, mz, g.y.nc, my, g.x.nc, mx)
    last = d6[:, -1, :, -1, :, -1]
    np.testing.assert_allclose(last, dc, rtol=1e-12, atol=1e-14 * np.abs(dc).max())
    others = d6.copy()
    others[:, -1, :, -1, :, -1] = 0.0
    assert np.abs(others).max() < 1e-13 * np.abs(dc).max()


def test_coarse_face_flux_preserved():
    """Dense fluxes through the sub-faces of a coarse face add up to its flux."""
    rng = np.random.default_rng(8)
    m = (3, 2, 2)
    g, _ = _grid((5, 6, 5), m, gamma=2.0, rng=rng)
    U, V, W = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=2, seed=4)
    u, v, w = O.refine_velocity(g, U, V, W)
    mx, my, mz = m
    fu = (u[:, :, ::mx] * g.y.h[None, :, None] * g.z.h[:, None, None])
    fu = fu.reshape(g.z.nc, mz, g.y.nc, my, g.x.nc).sum(axis=(1, 3))
    np.testing.assert_allclose(fu, U * g.y.H[None, :, None] * g.z.H[:, None, None], atol=1e-15)
    fw = (w[::mz] * g.x.h[None, None, :] * g.y.h[None, :, None])
    fw = fw.reshape(g.z.nc + 1, g.y.nc, my, g.x.nc, mx).sum(axis=(2, 4))
    np.testing.assert_allclose(fw, W * g.x.H[None, None, :] * g.y.H[None, :, None], atol=1e-15)


def test_linear_shear_reproduced_periodic():
    """u = a + b z, v = c + d z, w = 0 (divergence-free, periodic in x and y):
    face averages are the values at the face centroids, on both grids."""
    a, b, c, d = 0.3, -0.7, 0.11, 0.5
    g, _ = _grid((6, 5, 7), (2, 3, 2), gamma=1.7)
    zc_c = 0.5 * (g.z.cf[1:] + g.z.cf[:-1])
    U = np.broadcast_to((a + b * zc_c)[:, None, None], (g.z.nc, g.y.nc, g.x.nc)).copy()
    V = np.broadcast_to((c + d * zc_c)[:, None, None], (g.z.nc, g.y.nc, g.x.nc)).copy()
    W = np.zeros((g.z.nc + 1, g.y.nc, g.x.nc))
    u, v, w = O.refine_velocity(g, U, V, W)
    np.testing.assert_allclose(u, np.broadcast_to((a + b * g.z.c)[:, None, None], u.shape), atol=1e-14)
    np.testing.assert_allclose(v, np.broadcast_to((c + d * g.z.c)[:, None, None], v.shape), atol=1e-14)
    assert np.abs(w).max() < 1e-14


def test_linear_field_reproduced_walled():
    """Walls on all axes: u = G x + c with trace(G) = 0 is reproduced exactly."""
    rng = np.random.default_rng(21)
    G = rng.standard_normal((3, 3))
    G[2, 2] = -(G[0, 0] + G[1, 1])
    c0 = rng.standard_normal(3)
    g, _ = _grid((5, 4, 6), (2, 3, 2), gamma=1.2, periodic=(False, False, False), rng=rng)

    def faces_avg(comp, ax_faces, yy, zz, xx):
        return G[comp, 0] * xx + G[comp, 1] * yy + G[comp, 2] * zz + c0[comp]

    def build(xf, xc, yf, yc, zf, zc):
        U = faces_avg(0, None, yc[None, :, None], zc[:, None, None], xf[None, None, :])
        V = faces_avg(1, None, yf[None, :, None], zc[:, None, None], xc[None, None, :])
        W = faces_avg(2, None, yc[None, :, None], zf[:, None, None], xc[None, None, :])
        return U, V, W

    cc = lambda f: 0.5 * (f[1:] + f[:-1])
    U, V, W = build(g.x.cf, cc(g.x.cf), g.y.cf, cc(g.y.cf), g.z.cf, cc(g.z.cf))
    u, v, w = O.refine_velocity(g, U, V, W)
    ue, ve, we = build(g.x.faces, g.x.c, g.y.faces, g.y.c, g.z.faces, g.z.c)
    np.testing.assert_allclose(u, ue, atol=1e-13)
    np.testing.assert_allclose(v, ve, atol=1e-13)
    np.testing.assert_allclose(w, we, atol=1e-13)


def _gauss(a, b, npts=4):
    """Gauss-Legendre nodes and weights on [a, b] (exact for degree <= 7)."""
    t, wt = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (b - a) * t + 0.5 * (a + b), 0.5 * (b - a) * wt


def _poly_potential_fluxes(coefs, X, Y, Z):
    """Face-average velocities of curl A for a polynomial potential with degree
    <= 2 in each variable, by Stokes' theorem: each face flux is the
    circulation of A around the face, edge integrals by Gauss-Legendre."""
    def A(comp, x, y, z):
        out = 0.0
        for a in range(3):
            for b in range(3):
                for c in range(3):
                    out = out + coefs[comp, a, b, c] * x ** a * y ** b * z ** c
        return out

    gx = np.zeros((Z.size, Y.size, X.size - 1))
    for i in range(X.size - 1):
        pts, wts = _gauss(X[i], X[i + 1])
        for s, wq in zip(pts, wts):
            gx[:, :, i] += wq * A(0, s, Y[None, :], Z[:, None])
    gy = np.zeros((Z.size, Y.size - 1, X.size))
    for j in range(Y.size - 1):
        pts, wts = _gauss(Y[j], Y[j + 1])
        for s, wq in zip(pts, wts):
            gy[:, j, :] += wq * A(1, X[None, :], s, Z[:, None])
    gz = np.zeros((Z.size - 1, Y.size, X.size))
    for k in range(Z.size - 1):
        pts, wts = _gauss(Z[k], Z[k + 1])
        for s, wq in zip(pts, wts):
            gz[k] += wq * A(2, X[None, :], Y[:, None], s)
    fx = (gz[:, 1:, :] - gz[:, :-1, :]) - (gy[1:, :, :] - gy[:-1, :, :])      # (nz, ny, nx+1)
    fy = (gx[1:, :, :] - gx[:-1, :, :]) - (gz[:, :, 1:] - gz[:, :, :-1])      # (nz, ny+1, nx)
    fz = (gy[:, :, 1:] - gy[:, :, :-1]) - (gx[:, 1:, :] - gx[:, :-1, :])      # (nz+1, ny, nx)
    hx, hy, hz = np.diff(X), np.diff(Y), np.diff(Z)
    U = fx / (hy[None, :, None] * hz[:, None, None])
    V = fy / (hz[:, None, None] * hx[None, None, :])
    W = fz / (hx[None, None, :] * hy[None, :, None])
    return U, V, W


def test_triquadratic_divergence_free_field_reproduced():
    """Walls on all axes: the curl of a polynomial potential of degree <= 2 in
    each variable (a divergence-free field of per-variable degree <= 2) is
    refined exactly -- coarse and dense face averages from Stokes' theorem."""
    rng = np.random.default_rng(31)
    coefs = rng.standard_normal((3, 3, 3, 3))
    g, _ = _grid((5, 4, 5), (2, 3, 2), gamma=1.3, periodic=(False, False, False), rng=rng)
    U, V, W = _poly_potential_fluxes(coefs, g.x.cf, g.y.cf, g.z.cf)
    ue, ve, we = _poly_potential_fluxes(coefs, g.x.faces, g.y.faces, g.z.faces)
    u, v, w = O.refine_velocity(g, U, V, W)
    scale = max(np.abs(ue).max(), np.abs(ve).max(), np.abs(we).max())
    np.testing.assert_allclose(u, ue, atol=1e-11 * scale)
    np.testing.assert_allclose(v, ve, atol=1e-11 * scale)
    np.testing.assert_allclose(w, we, atol=1e-11 * scale)


def test_m1_is_identity():
    g, _ = _grid((6, 5, 4), (1, 1, 1), gamma=1.0)
    rng = np.random.default_rng(2)
    U = rng.standard_normal((4, 5, 6))
    V = rng.standard_normal((4, 5, 6))
    W = rng.standard_normal((5, 5, 6))
    u, v, w = O.refine_velocity(g, U, V, W)
    assert np.array_equal(u, U) and np.array_equal(v, V) and np.array_equal(w, W)


def test_linear_in_coarse_field():
    """A linear combination of coarse fields refines to the same combination
    (why time-interpolated coarse fields stay divergence-free, Sec. 3.4)."""
    rng = np.random.default_rng(9)
    g, _ = _grid((5, 5, 5), (2, 2, 3), gamma=1.5)
    f1 = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=2, seed=1)
    f2 = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=2, seed=7)
    a = 0.375
    r1 = O.refine_velocity(g, *f1)
    r2 = O.refine_velocity(g, *f2)
    rc = O.refine_velocity(g, *[(1 - a) * p + a * q for p, q in zip(f1, f2)])
    for x, y, z in zip(r1, r2, rc):
        np.testing.assert_allclose(z, (1 - a) * x + a * y, atol=1e-14)


# ------------------------------------------------------------------- transpose
def _flat(*arrs):
    return np.concatenate([a.ravel() for a in arrs])


@pytest.mark.parametrize("periodic", [(True, True, False), (False, False, False)])
def test_transpose_brute_force(periodic):
    """P^T from the oracle equals the transpose of P assembled column by column
    from the forward refinement on a tiny grid."""
    rng = np.random.default_rng(4)
    g, _ = _grid((3, 3, 3), (2, 3, 2), gamma=1.4, periodic=periodic, rng=rng)
    shapes_c = [(g.z.nc, g.y.nc, g.x.ncfaces()), (g.z.nc, g.y.ncfaces(), g.x.nc),
                (g.z.nc + 1, g.y.nc, g.x.nc)]
    sizes_c = [int(np.prod(s)) for s in shapes_c]
    ncol = sum(sizes_c)

    def unflat(vec, shapes):
        out, o = [], 0
        for s in shapes:
            k = int(np.prod(s))
            out.append(vec[o:o + k].reshape(s))
            o += k
        return out

    cols = []
    for c in range(ncol):
        e = np.zeros(ncol)
        e[c] = 1.0
        cols.append(_flat(*O.refine_velocity(g, *unflat(e, shapes_c))))
    P = np.stack(cols, axis=1)
    y = rng.standard_normal(P.shape[0])
    shapes_d = [(g.z.n, g.y.n, g.x.nfaces()), (g.z.n, g.y.nfaces(), g.x.n), (g.z.n + 1, g.y.n, g.x.n)]
    got = _flat(*O.refine_velocity_transpose(g, *unflat(y, shapes_d)))
    np.testing.assert_allclose(got, P.T @ y, rtol=1e-12, atol=1e-12 * np.abs(P.T @ y).max())


def test_transpose_dot_product_generator_grid():
    """<P x, y> = <x, P^T y> on a tanh grid with M = 3."""
    rng = np.random.default_rng(6)
    g, _ = _grid((7, 6, 8), (3, 3, 3), gamma=2.0)
    x = [rng.standard_normal(s) for s in [(8, 6, 7), (8, 6, 7), (9, 6, 7)]]
    y = [rng.standard_normal(s) for s in [(24, 18, 21), (24, 18, 21), (25, 18, 21)]]
    lhs = sum(np.vdot(a, b) for a, b in zip(O.refine_velocity(g, *x), y))
    rhs = sum(np.vdot(a, b) for a, b in zip(x, O.refine_velocity_transpose(g, *y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_split_matches_r_application_for_all_cells():
    """split() applies R cell by cell with periodic wrap of the stencil."""
    rng = np.random.default_rng(12)
    ax = O.Axis(_stretched_faces(12, rng), 3, True)
    q = rng.standard_normal(4)
    s = split(q[:, None], 0, ax)[:, 0]
    for I in range(4):
        idx = [(I - 1 + r) % 4 for r in range(3)]
        np.testing.assert_allclose(s[3 * I:3 * I + 3], O.r_matrix(ax, I) @ q[idx], atol=1e-15)
