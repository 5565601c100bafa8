"""Divergence-free coarse-to-dense refinement of a staggered velocity.

Follows paper Sec. 3.2 ("Downscale refinement of the velocity field"):

* Mass-conserving split of a coarse face velocity into M sub-face velocities:
  a quadratic f whose means over three neighbouring coarse intervals equal the
  three coarse values (Eqs. 12-15, V = A zeta), integrated over the M
  sub-intervals (Eqs. 16-18, V_s = A_s zeta), so V_s = A_s A^-1 V = R V
  (Eq. 19), R an M x 3 matrix per coarse cell that depends on the grid only.
* Stepwise refinement (Fig. 5a): split the outer normal velocities, then get
  each inner face velocity from zero net outward flux of the sub-cell below
  it, one direction at a time.

Readings where the paper is silent or shows only 2-D (each one also listed in
the design notes): the stages run z, then y, then x; the marches run in
ascending index inside each coarse cell; the last sub-cell's balance is not
imposed (it holds because the splits conserve each coarse face's flux); on a
walled axis the three-cell stencil is shifted inwards at the first and last
coarse cell; for M = 1 the split is the identity; the flux balance uses face
areas (the garbled inner-face formula of the 2-D example is read as zero net
outward flux).

Array conventions: [z][y][x], x fastest.  Coarse U (x-faces) has shape
(ncz, ncy, ncfx), V (ncz, ncfy, ncx), W (ncz+1, ncy, ncx) where ncf = nc on a
periodic axis and nc+1 on a walled one.  Dense u, v, w likewise.
Test infrastructure only.
"""
import numpy as np


# ------------------------------------------------------------------ R matrices
def _interval_means(a, b):
    """Means of 1, x, x^2 over [a, b] (one row of A or A_s, Eqs. 15 and 18)."""
    return np.array([1.0, 0.5 * (a + b), (a * a + a * b + b * b) / 3.0])


def stencil_start(ax, I):
    """First coarse cell of the three-cell stencil of coarse cell I.

    Centred (I-1) on a periodic axis (may be -1, wrapped); on a walled axis the
    stencil is kept inside the domain: 0 for I = 0 and nc-3 for I = nc-1."""
    if ax.periodic:
        return I - 1
    return min(max(I - 1, 0), ax.nc - 3)


def r_matrix(ax, I):
    """R = A_s A^-1 (Eq. 19) of coarse cell I on axis ``ax``, shape (m, 3).

    Coordinates are mapped to xi = (x - centre_I)/H_I first; R is invariant
    under this affine map and A stays well conditioned.  m = 1 gives [0 1 0]."""
    m, nc = ax.m, ax.nc
    if m == 1:
        return np.array([[0.0, 1.0, 0.0]])
    if nc < 3:
        raise ValueError("a three-cell stencil needs at least 3 coarse cells")
    X = ax.cf
    centre = 0.5 * (X[I] + X[I + 1])
    H = X[I + 1] - X[I]
    s = stencil_start(ax, I)
    A = np.empty((3, 3))
    for r in range(3):
        c = s + r
        shift = 0.0
        if ax.periodic:
            shift = ax.length * (c // nc)
            c = c % nc
        A[r] = _interval_means((X[c] + shift - centre) / H, (X[c + 1] + shift - centre) / H)
    sub = ax.faces[I * m:(I + 1) * m + 1]
    As = np.array([_interval_means((sub[q] - centre) / H, (sub[q + 1] - centre) / H)
                   for q in range(m)])
    # R A = A_s  ->  A^T R^T = A_s^T
    return np.linalg.solve(A.T, As.T).T


def r_tables(ax):
    """R of every coarse cell, shape (nc, m, 3), and the stencil cell indices (nc, 3).

    For m = 1 every stencil is centred on its own cell, so R = [0 1 0] picks it."""
    R = np.stack([r_matrix(ax, I) for I in range(ax.nc)])
    idx = np.empty((ax.nc, 3), dtype=np.int64)
    if ax.m == 1:
        for I in range(ax.nc):
            idx[I] = (I - 1) % ax.nc, I, (I + 1) % ax.nc
        return R, idx
    for I in range(ax.nc):
        s = stencil_start(ax, I)
        for r in range(3):
            idx[I, r] = (s + r) % ax.nc if ax.periodic else s + r
    return R, idx


def split(q, axis, ax):
    """Sub-face values qs[I*m + p] = sum_r R_I[p, r] q[s_I + r] along ``axis``.

    ``q`` must hold one value per coarse cell along that axis."""
    R, idx = r_tables(ax)
    q = np.moveaxis(np.asarray(q, dtype=np.float64), axis, 0)
    if q.shape[0] != ax.nc:
        raise ValueError("split expects %d coarse values, got %d" % (ax.nc, q.shape[0]))
    out = np.empty((ax.n,) + q.shape[1:])
    for I in range(ax.nc):
        for p in range(ax.m):
            out[I * ax.m + p] = (R[I, p, 0] * q[idx[I, 0]] + R[I, p, 1] * q[idx[I, 1]]
                                 + R[I, p, 2] * q[idx[I, 2]])
    return np.moveaxis(out, 0, axis)


def split_transpose(g, axis, ax):
    """Transpose of ``split``: scatter sub-face values back with R."""
    R, idx = r_tables(ax)
    g = np.moveaxis(np.asarray(g, dtype=np.float64), axis, 0)
    out = np.zeros((ax.nc,) + g.shape[1:])
    for I in range(ax.nc):
        for p in range(ax.m):
            for r in range(3):
                out[idx[I, r]] += R[I, p, r] * g[I * ax.m + p]
    return np.moveaxis(out, 0, axis)


# -------------------------------------------------------------- face differences
def dface(q, axis, periodic):
    """q[i+1] - q[i] for every cell i along ``axis`` (faces -> cells)."""
    if periodic:
        return np.roll(q, -1, axis=axis) - q
    return np.diff(q, axis=axis)


def dface_transpose(g, axis, periodic):
    """Transpose of ``dface`` (cells -> faces)."""
    if periodic:
        return np.roll(g, 1, axis=axis) - g
    g = np.moveaxis(g, axis, 0)
    n = g.shape[0]
    out = np.zeros((n + 1,) + g.shape[1:])
    out[1:] += g
    out[:-1] -= g
    return np.moveaxis(out, 0, axis)


# -------------------------------------------------------------------- stages
def _stage_z(g, U, V, W):
    x, y, z = g.x, g.y, g.z
    Uz = split(U, 0, z)
    Vz = split(V, 0, z)
    Wz = np.empty((z.n + 1,) + W.shape[1:])
    Wz[::z.m] = W
    dU = dface(Uz, 2, x.periodic)                  # (nz, ncy, ncx)
    dV = dface(Vz, 1, y.periodic)
    HX = x.H[None, :]
    HY = y.H[:, None]
    for K in range(z.nc):
        for p in range(z.m - 1):
            k = K * z.m + p
            hz = z.h[k]
            Wz[k + 1] = Wz[k] - (dU[k] * HY * hz + dV[k] * HX * hz) / (HX * HY)
    return Uz, Vz, Wz


def _stage_y(g, Uz, Vz, Wz):
    x, y, z = g.x, g.y, g.z
    Uzy = split(Uz, 1, y)
    Wzy = split(Wz, 1, y)
    Vzy = np.empty((z.n, y.nfaces(), Vz.shape[2]))
    Vzy[:, ::y.m] = Vz
    dU = dface(Uzy, 2, x.periodic)                 # (nz, ny, ncx)
    dW = Wzy[1:] - Wzy[:-1]                        # (nz, ny, ncx)
    HX = x.H[None, :]
    hz = z.h[:, None]
    for J in range(y.nc):
        for p in range(y.m - 1):
            j = J * y.m + p
            hy = y.h[j]
            Vzy[:, j + 1] = Vzy[:, j] - (dU[:, j] * hy * hz + dW[:, j] * HX * hy) / (HX * hz)
    return Uzy, Vzy, Wzy


def _stage_x(g, Uzy, Vzy, Wzy):
    x, y, z = g.x, g.y, g.z
    v = split(Vzy, 2, x)
    w = split(Wzy, 2, x)
    u = np.empty((z.n, y.n, x.nfaces()))
    u[..., ::x.m] = Uzy
    dV = dface(v, 1, y.periodic)                   # (nz, ny, nx)
    dW = w[1:] - w[:-1]
    hz = z.h[:, None]
    hy = y.h[None, :]
    for I in range(x.nc):
        for p in range(x.m - 1):
            i = I * x.m + p
            hx = x.h[i]
            u[..., i + 1] = u[..., i] - (dV[..., i] * hx * hz + dW[..., i] * hx * hy) / (hy * hz)
    return u, v, w


def refine_velocity(g, U, V, W):
    """Coarse staggered (U, V, W) -> dense (u, v, w), stages z, y, x (Sec. 3.2)."""
    U, V, W = (np.asarray(a, dtype=np.float64) for a in (U, V, W))
    Uz, Vz, Wz = _stage_z(g, U, V, W)
    Uzy, Vzy, Wzy = _stage_y(g, Uz, Vz, Wz)
    return _stage_x(g, Uzy, Vzy, Wzy)


# ---------------------------------------------------------------- transposes
def _suffix_without_self(gq, axis, m):
    """For each coarse cell, a[p] = sum of gq over sub-faces p+1..m-1 (march transpose)."""
    gq = np.moveaxis(gq, axis, 0)
    out = np.zeros_like(gq)
    n = gq.shape[0] - (gq.shape[0] % m)
    for I in range(n // m):
        acc = np.zeros(gq.shape[1:])
        for p in range(m - 1, -1, -1):
            out[I * m + p] = acc
            acc = acc + gq[I * m + p]
    return np.moveaxis(out, 0, axis)


def _coarse_sum(gq, axis, m, ncf):
    """gQ[I] = sum_p gq[I*m + p]; on a walled axis the last coarse face takes the last dense one."""
    gq = np.moveaxis(gq, axis, 0)
    out = np.zeros((ncf,) + gq.shape[1:])
    nc = (gq.shape[0]) // m
    for I in range(nc):
        out[I] = gq[I * m:(I + 1) * m].sum(axis=0)
    if ncf > nc:
        out[nc] = gq[nc * m]
    return np.moveaxis(out, 0, axis)


def refine_velocity_transpose(g, gu, gv, gw):
    """Transpose of ``refine_velocity``: dense face adjoints -> coarse face adjoints.

    Each stage is reversed: a march u[i+1] = u[i] - c_i becomes a reverse
    suffix accumulation, a split becomes an R-transpose scatter."""
    x, y, z = g.x, g.y, g.z
    gu, gv, gw = (np.asarray(a, dtype=np.float64) for a in (gu, gv, gw))
    # ---- stage x
    gc = -_suffix_without_self(gu, 2, x.m)[..., :x.n]   # adjoint of each march increment c_i
    hxv = x.h[None, None, :]
    gdV = gc * hxv / y.h[None, :, None]
    gdW = gc * hxv / z.h[:, None, None]
    gv = gv + dface_transpose(gdV, 1, y.periodic)
    gw_t = gw.copy()
    gw_t[1:] += gdW
    gw_t[:-1] -= gdW
    gUzy = _coarse_sum(gu, 2, x.m, x.ncfaces())
    gVzy = split_transpose(gv, 2, x)
    gWzy = split_transpose(gw_t, 2, x)
    # ---- stage y
    gc = -_suffix_without_self(gVzy, 1, y.m)[:, :y.n]   # (nz, ny, ncx)
    hyv = y.h[None, :, None]
    gdU = gc * hyv / x.H[None, None, :]
    gdW = gc * hyv / z.h[:, None, None]
    gUzy = gUzy + dface_transpose(gdU, 2, x.periodic)
    gWzy = gWzy.copy()
    gWzy[1:] += gdW
    gWzy[:-1] -= gdW
    gVz = _coarse_sum(gVzy, 1, y.m, y.ncfaces())
    gUz = split_transpose(gUzy, 1, y)
    gWz = split_transpose(gWzy, 1, y)
    # ---- stage z
    gc = -_suffix_without_self(gWz[:-1], 0, z.m)   # (nz, ncy, ncx)
    hzv = z.h[:, None, None]
    gdU = gc * hzv / x.H[None, None, :]
    gdV = gc * hzv / y.H[None, :, None]
    gUz = gUz + dface_transpose(gdU, 2, x.periodic)
    gVz = gVz + dface_transpose(gdV, 1, y.periodic)
    gW = _coarse_sum(gWz, 0, z.m, z.nc + 1)
    gU = split_transpose(gUz, 0, z)
    gV = split_transpose(gVz, 0, z)
    return gU, gV, gW


# ----------------------------------------------------------------- divergence
def divergence(g, u, v, w):
    """Net outward volume flux of every dense cell and the sum of |face fluxes|.

    div = (u_{i+1}-u_i) hy hz + (v_{j+1}-v_j) hx hz + (w_{k+1}-w_k) hx hy."""
    x, y, z = g.x, g.y, g.z
    ax = y.h[None, :, None] * z.h[:, None, None]
    ay = x.h[None, None, :] * z.h[:, None, None]
    az = x.h[None, None, :] * y.h[None, :, None]
    div = dface(u, 2, x.periodic) * ax + dface(v, 1, y.periodic) * ay + (w[1:] - w[:-1]) * az

    def absum(q, axis, periodic):
        a = np.abs(q)
        if periodic:
            return a + np.roll(a, -1, axis=axis)
        sl0 = [slice(None)] * 3
        sl1 = [slice(None)] * 3
        sl0[axis] = slice(0, -1)
        sl1[axis] = slice(1, None)
        return a[tuple(sl0)] + a[tuple(sl1)]

    tot = absum(u, 2, x.periodic) * ax + absum(v, 1, y.periodic) * ay + absum(w, 0, False) * az
    return div, tot
