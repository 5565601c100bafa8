"""Oracle results for single dense columns of a large grid, computed on small
windows (test infrastructure).

On a grid that is uniform in x and y, the refinement of the coarse cells
around coarse column (I, J) depends only on coarse columns I-3..I+3 and
J-3..J+3, and one scalar step of dense column (i, j) only on the dense columns
i-1..i+1, j-1..j+1 (all z).  A window of that size, treated as a small
periodic domain with the same spacing, therefore gives the exact oracle
values at its centre: the window's own wrap only touches columns that are
discarded.  The window inputs are slices of the caller's arrays (generator
output), never of GPU results.
"""
import numpy as np

import oracle as O

COARSE_RADIUS = 3


def _take(a, axis, idx):
    return np.take(a, idx, axis=axis, mode="wrap")


def refine_window(U, V, W, m, zf, nx, ny, I, J):
    """Oracle dense (u, v, w) of the dense columns inside coarse columns
    I-1..I+1 and J-1..J+1; returns the dense window arrays and the global
    dense index of their first x and y column."""
    mx, my, mz = m
    ncy, ncx = U.shape[1], U.shape[2]
    r = COARSE_RADIUS
    ci = np.arange(I - r, I + r + 1) % ncx
    cj = np.arange(J - r, J + r + 1) % ncy
    Uw = _take(_take(U, 2, ci), 1, cj)
    Vw = _take(_take(V, 2, ci), 1, cj)
    Ww = _take(_take(W, 2, ci), 1, cj)
    n_win = 2 * r + 1
    xf = np.arange(n_win * mx + 1) / nx
    yf = np.arange(n_win * my + 1) / ny
    g = O.Grid(xf, yf, zf, m)
    u, v, w = O.refine_velocity(g, Uw, Vw, Ww)
    return (u, v, w), ((I - r) * mx, (J - r) * my)


def window3(a, nx, ny, i, j):
    """The nz x 3 x 3 columns of field a around dense column (i, j), wrapped."""
    xs = np.arange(i - 1, i + 2) % nx
    ys = np.arange(j - 1, j + 2) % ny
    return _take(_take(a, 2, xs), 1, ys)


def step_column_windows(tp, tc, uvw_window, origin, zf, nx, ny, params, n, i, j):
    """Oracle scalar step n for dense column (i, j) from nz x 3 x 3 windows
    (centred on the column) of theta^{n-1} and theta^n and the window velocity."""
    u, v, w = uvw_window
    ox, oy = origin
    li, lj = i - ox, j - oy            # position inside the velocity window
    assert 1 <= li < u.shape[2] - 1 and 1 <= lj < u.shape[1] - 1
    sl = (slice(None), slice(lj - 1, lj + 2), slice(li - 1, li + 2))
    g = O.Grid(np.arange(4) / nx, np.arange(4) / ny, zf, (1, 1, 1))
    out = O.scalar_step(g, params, n, tp, tc, u[sl], v[sl], w[sl])
    return out[:, 1, 1]


def step_column(th_prev, th_cur, uvw_window, origin, zf, nx, ny, m, params, n, i, j):
    """Oracle scalar step n for dense column (i, j): a 3x3-column window of the
    scalar levels and of the window velocity around (i, j)."""
    return step_column_windows(window3(th_prev, nx, ny, i, j), window3(th_cur, nx, ny, i, j), uvw_window,
                               origin, zf, nx, ny, params, n, i, j)


def dense_column(uvw_window, origin, i, j):
    """(u, v, w) of dense column (i, j) from a refined window."""
    u, v, w = uvw_window
    li, lj = i - origin[0], j - origin[1]
    return u[:, lj, li], v[:, lj, li], w[:, lj, li]


def sample_columns(nx, ny, mx, my, count, seed):
    """Seeded dense columns (i, j), spread over the grid, including the
    periodic seam (first and last columns)."""
    rng = np.random.default_rng(seed)
    cols = [(0, 0), (nx - 1, ny - 1), (nx - 1, 0)]
    while len(cols) < count:
        cols.append((int(rng.integers(nx)), int(rng.integers(ny))))
    return cols


def z_system_transpose(g, params, n):
    """(sub, diag, sup) of Z_n^T, Z_n = I - (1 - w) tau_n kappa Lz0 the implicit
    z system of step n (the oracle's matrix, transposed)."""
    tau = O.step_kind(n, params.n_avg, params.dt)[0]
    sub, diag, sup, _ = O.z_matrix(g, tau * params.kappa * (1.0 - params.z_explicit), params)
    sub_t, sup_t = np.zeros_like(sub), np.zeros_like(sup)
    sub_t[1:] = sup[:-1]
    sup_t[:-1] = sub[1:]
    return sub_t, diag, sup_t


def _z_t_times(g, params, n, mu):
    """Z_n^T mu column by column: the lam whose transposed solve gives back mu."""
    sub_t, diag, sup_t = z_system_transpose(g, params, n)
    r = diag[:, None, None] * mu
    r[1:] += sub_t[1:, None, None] * mu[:-1]
    r[:-1] += sup_t[:-1, None, None] * mu[1:]
    return r


def reverse_step(g, params, n, mu_next, mu_cur, th_cur, u, v, w):
    """Oracle values of the library's fused reverse step n on a whole (window or
    full) periodic field, from mu^{n+1} (None when no later step exists), mu^n
    and theta^n:

        lam^n = a_p(n+1) mu^{n+1} + tau_{n+1} kappa Lh^T mu^{n+1}
              + a_c(n) mu^n + tau_n C_u^T mu^n,
        out   = Z_{n-1}^{-T} lam^n (n >= 1),  lam^0 + tau_0 kappa Lh^T mu^0 (n = 0),

    with mu^m = Z_m^{-T} dL/dtheta^{m+1}.  Each piece is the oracle's step_vjp
    fed lam = Z_m^T mu^m, so that its own transposed solve returns mu^m.  Also
    returns step n's velocity gradient (gu, gv, gw) on every dense face."""
    _, g_cur, gu, gv, gw = O.step_vjp(g, params, n, th_cur, u, v, w, _z_t_times(g, params, n, mu_cur))
    lam = g_cur
    if mu_next is not None:
        lam = lam + O.step_vjp(g, params, n + 1, th_cur, u, v, w, _z_t_times(g, params, n + 1, mu_next))[0]
    if n >= 1:
        lam = O.thomas(*z_system_transpose(g, params, n - 1), lam)
    return lam, (gu, gv, gw)


def backward_column(mu_next, mu_cur, th_cur, uvw_window, origin, zf, nx, ny, params, n, i, j):
    """``reverse_step`` for dense column (i, j) of a large grid, from 3x3-column
    windows (nz x 3 x 3, centred on the column) of mu^{n+1} (or None), mu^n and
    theta^n: the output column and step n's velocity gradient on the faces of
    the column (x face i, y face j, the z faces).  The transposed stencils reach
    one column out, so the centre of the window is exact."""
    u, v, w = uvw_window
    li, lj = i - origin[0], j - origin[1]
    assert 1 <= li < u.shape[2] - 1 and 1 <= lj < u.shape[1] - 1
    sl = (slice(None), slice(lj - 1, lj + 2), slice(li - 1, li + 2))
    g = O.Grid(np.arange(4) / nx, np.arange(4) / ny, zf, (1, 1, 1))
    out, (gu, gv, gw) = reverse_step(g, params, n, mu_next, mu_cur, th_cur, u[sl], v[sl], w[sl])
    return out[:, 1, 1], (gu[:, 1, 1], gv[:, 1, 1], gw[:, 1, 1])


def seed(g, params, n, lam):
    """mu^n = Z_n^{-T} lam, column by column (lam: one column or a field)."""
    return O.thomas(*z_system_transpose(g, params, n), lam)
