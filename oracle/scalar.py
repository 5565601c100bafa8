"""Finite-volume scalar step on the dense grid, its Nusselt diagnostics and adjoint.

Follows the paper's heat equation (Eq. 2) in integral form (Eq. 5) on the
staggered grid (Sec. 2.2), the Euler-leapfrog step (Eq. 6) with the averaging
step every N_p steps (Eq. 7), and the heat-flux Nusselt number (Eq. 22).

Readings (each also listed in the design notes):
* face value of the advected scalar: second-order central, the arithmetic
  mean of the two neighbouring cells, by default; or fourth order as in the
  paper's code (Sec. 2.2), read as the value at the face of the polynomial
  whose means over the stencil cells equal their values (two cells on each
  side of the face; on a walled axis only the cells that exist);
* diffusion: x and y explicit on the lagged level n-1 as in Eq. 6; the z part
  moved to the new level n+1 and solved line by line (backward Euler over the
  step's time span tau), which keeps the wall-clustered z grid stable;
* the first step (n = 0) is forward Euler over dt with the same implicit z
  part; the averaging step produces theta^{n+1} when (n+1) mod N_p = 0, n >= 1,
  with its diffusion on level n-1 as written in Eq. 7;
* optionally only a fraction 1 - w of the z diffusion is implicit, the rest
  explicit on the lagged level (the level of the x/y diffusion): w = 1/2 is the
  Crank-Nicolson weighting across the step's time span, w = 0 (default) fully
  implicit;
* z walls: Dirichlet (wall value at half a cell from the first centre) or
  adiabatic; x and y periodic, or bounded by adiabatic no-slip side walls (the
  paper's cube, Sec. 4): a wall face carries neither advective nor diffusive
  flux;
* Nu(z) lives on the dense z faces; the plates use the half-cell gradient;
  Nu_paper is the mean over the interior faces, Nu_vol the height-weighted sum.

Array conventions: theta (nz, ny, nx); u (nz, ny, nx) on x-faces i (between
cells i-1 and i, periodic), or (nz, ny, nx+1) with the two wall faces when x
is walled; v likewise on y-faces; w (nz+1, ny, nx) on z-faces.
Test infrastructure only; all arithmetic float64, plain NumPy.
"""
import math
from dataclasses import dataclass

import numpy as np

DIRICHLET = "dirichlet"
ADIABATIC = "adiabatic"


@dataclass
class ScalarParams:
    kappa: float                 # (Ra Pr)^(-1/2), Eq. 2
    dt: float
    n_avg: int = 50              # N_p of Eq. 7 (0 = never average)
    t_bot: float = 1.0
    t_top: float = 0.0
    bc_bot: str = DIRICHLET
    bc_top: str = DIRICHLET
    ra: float = 1.0              # Ra and Pr enter Nu through (Ra Pr)^(1/2)
    pr: float = 1.0
    z_explicit: float = 0.0      # w: share of the z diffusion taken explicit on the lagged level
    face_order: int = 2          # face value of the advected scalar: 2 (mean) or 4

    @staticmethod
    def from_ra_pr(ra, pr, dt, **kw):
        return ScalarParams(kappa=1.0 / math.sqrt(ra * pr), dt=dt, ra=ra, pr=pr, **kw)


def step_kind(n, n_avg, dt):
    """(tau, alpha_prev, alpha_cur, kind) of the step that makes theta^{n+1}.

    n = 0: start-up, forward Euler over dt (Eq. 6 needs two levels);
    (n+1) mod N_p = 0: averaging step of Eq. 7, 1.5 dt and (theta^{n-1}+theta^n)/2;
    otherwise leapfrog of Eq. 6, 2 dt from theta^{n-1}."""
    if n == 0:
        return dt, 0.0, 1.0, "startup"
    if n_avg > 0 and (n + 1) % n_avg == 0:
        return 1.5 * dt, 0.5, 0.5, "average"
    return 2.0 * dt, 1.0, 0.0, "leapfrog"


# ------------------------------------------------------------------ faces
def _sides(q, axis, periodic):
    """Cell values on the low and high side of every face normal to ``axis``:
    periodic, face i lies between cells i-1 and i (n faces); walled, faces
    0..n with the two wall faces seeing the adjacent cell on both sides."""
    if periodic:
        return np.roll(q, 1, axis=axis), q
    q0 = np.moveaxis(q, axis, 0)
    lo = np.concatenate([q0[:1], q0])
    hi = np.concatenate([q0, q0[-1:]])
    return np.moveaxis(lo, 0, axis), np.moveaxis(hi, 0, axis)


def _open(f, axis, periodic):
    """Face array with the wall faces (walled axis) set to zero."""
    if periodic:
        return f
    f = np.array(f, dtype=np.float64, copy=True)
    f0 = np.moveaxis(f, axis, 0)
    f0[0] = 0.0
    f0[-1] = 0.0
    return f


def _net(f, axis, periodic):
    """f[i+1] - f[i] for every cell i from face values (outflow minus inflow)."""
    if periodic:
        return np.roll(f, -1, axis=axis) - f
    return np.diff(f, axis=axis)


def _to_cells(s_lo, s_hi, axis, periodic):
    """Per-cell sums of face contributions: cell i receives s_hi of its low
    face and s_lo of its high face."""
    if periodic:
        return s_hi + np.roll(s_lo, -1, axis=axis)
    n = s_lo.shape[axis] - 1
    return np.take(s_hi, np.arange(n), axis=axis) + np.take(s_lo, np.arange(1, n + 1), axis=axis)


# ------------------------------------------------------- face interpolation
def _interval_means(a, b, npow):
    """Means over [a, b] of x^q, q = 0..npow-1."""
    q = np.arange(npow)
    return (b ** (q + 1) - a ** (q + 1)) / ((q + 1) * (b - a))


def face_weights(ax, order):
    """Stencils of the face value along one axis: (cells, weights), shape (nf, 4).

    The value on face f is sum_s weights[f, s] * theta[cells[f, s]]; unused
    slots have weight 0.  Faces: periodic axis n faces (face i between cells
    i-1 and i); walled axis n+1 faces, whose two wall faces get zero weights.
    order 2: the mean of the two cells.  order 4 (Sec. 2.2, fourth-order face
    values): the stencil is the two cells on each side of the face -- on a
    periodic axis wrapped around with the period added to their coordinates,
    on a walled axis only the cells that exist (three next to a wall cell, two
    when the axis has two cells) -- and the face value is the value at the
    face of the polynomial (degree = cells - 1) whose mean over every stencil
    cell equals that cell's value."""
    n, f = ax.n, ax.faces
    nf = n if ax.periodic else n + 1
    cells = np.zeros((nf, 4), dtype=np.int64)
    wts = np.zeros((nf, 4))
    for face in range(nf):
        if not ax.periodic and (face == 0 or face == n):
            continue
        if order == 2:
            lo, hi = face - 1, face
        elif order == 4:
            lo, hi = face - 2, face + 1
            if not ax.periodic:
                lo, hi = max(lo, 0), min(hi, n - 1)
        else:
            raise ValueError("face order must be 2 or 4")
        xf = f[face]
        h = ax.h[face % n]                       # length scale of the local solve
        rows, idx = [], []
        for c in range(lo, hi + 1):
            wrap, cell = divmod(c, n)            # wrap = periods crossed (periodic axes only)
            shift = wrap * ax.length
            a = (f[cell] + shift - xf) / h
            b = (f[cell + 1] + shift - xf) / h
            rows.append((a, b))
            idx.append(cell)
        m = len(rows)
        A = np.array([_interval_means(a, b, m) for a, b in rows])
        # face value = coefficient of x^0 = e_0 . A^-1 theta  ->  weights = A^-T e_0
        e0 = np.zeros(m)
        e0[0] = 1.0
        wts[face, :m] = np.linalg.solve(A.T, e0)
        cells[face, :m] = idx
    return cells, wts


def face_values(ax, q, axis, order):
    """Face values of q along ``axis`` (faces first as in ``face_weights``)."""
    cells, wts = face_weights(ax, order)
    q0 = np.moveaxis(q, axis, 0)
    out = np.zeros((cells.shape[0],) + q0.shape[1:])
    for s in range(4):
        out += wts[:, s].reshape((-1,) + (1,) * (q0.ndim - 1)) * q0[cells[:, s]]
    return np.moveaxis(out, 0, axis)


def face_values_transpose(ax, t, axis, order):
    """Transpose of ``face_values``: face quantities t -> cells."""
    cells, wts = face_weights(ax, order)
    t0 = np.moveaxis(t, axis, 0)
    out = np.zeros((ax.n,) + t0.shape[1:])
    for face in range(cells.shape[0]):
        for s in range(4):
            if wts[face, s] != 0.0:
                out[cells[face, s]] += wts[face, s] * t0[face]
    return np.moveaxis(out, 0, axis)


# ------------------------------------------------------------------ operators
def _areas(g):
    ax = g.y.h[None, :, None] * g.z.h[:, None, None]       # x-face areas hy*hz
    ay = g.x.h[None, None, :] * g.z.h[:, None, None]       # y-face areas hx*hz
    az = g.x.h[None, :] * g.y.h[:, None]                   # z-face areas hx*hy (ny, nx)
    return ax, ay, az


def advection(g, th, u, v, w, order=2):
    """C(theta) = -(1/V) sum of outward fluxes u_f A_f theta_f, theta_f = mean of the
    two cells (Eq. 5, convective term), or the fourth-order face value of
    ``face_weights`` with order=4; no flux through any wall."""
    if order == 4:
        return _advection4(g, th, u, v, w)
    ax, ay, az = _areas(g)
    px, py = g.x.periodic, g.y.periodic
    if px and py:
        fx = u * 0.5 * (np.roll(th, 1, axis=2) + th) * ax       # face i: cells i-1, i
        fy = v * 0.5 * (np.roll(th, 1, axis=1) + th) * ay
    else:
        lx, hx_ = _sides(th, 2, px)
        ly, hy_ = _sides(th, 1, py)
        fx = _open(u * 0.5 * (lx + hx_) * ax, 2, px)
        fy = _open(v * 0.5 * (ly + hy_) * ay, 1, py)
    nz = th.shape[0]
    fz = np.zeros((nz + 1,) + th.shape[1:])
    fz[1:nz] = w[1:nz] * 0.5 * (th[:-1] + th[1:]) * az[None]
    net = _net(fx, 2, px) + _net(fy, 1, py) + (fz[1:] - fz[:-1])
    return -net / g.vol()


def _advection4(g, th, u, v, w):
    ax, ay, az = _areas(g)
    px, py = g.x.periodic, g.y.periodic
    fx = _open(u * face_values(g.x, th, 2, 4) * ax, 2, px)
    fy = _open(v * face_values(g.y, th, 1, 4) * ay, 1, py)
    fz = _open(w * face_values(g.z, th, 0, 4) * az[None], 0, False)
    net = _net(fx, 2, px) + _net(fy, 1, py) + (fz[1:] - fz[:-1])
    return -net / g.vol()


def lap_h(g, th):
    """Horizontal diffusion (1/V) sum over x and y faces of A_f (theta_R - theta_L)/dc_f;
    no diffusive flux through a side wall (adiabatic)."""
    ax, ay, _ = _areas(g)
    px, py = g.x.periodic, g.y.periodic
    if px and py:
        gx = (th - np.roll(th, 1, axis=2)) / g.x.dc[None, None, :] * ax
        gy = (th - np.roll(th, 1, axis=1)) / g.y.dc[None, :, None] * ay
        return ((np.roll(gx, -1, axis=2) - gx) + (np.roll(gy, -1, axis=1) - gy)) / g.vol()
    lx, hx_ = _sides(th, 2, px)
    ly, hy_ = _sides(th, 1, py)
    gx = _open((hx_ - lx) / g.x.dc[None, None, :] * ax, 2, px)
    gy = _open((hy_ - ly) / g.y.dc[None, :, None] * ay, 1, py)
    return (_net(gx, 2, px) + _net(gy, 1, py)) / g.vol()


def z_matrix(g, tk, p):
    """Tridiagonal (sub, diag, sup) of I - tk*Lz0 and the wall source bz with
    Lz theta = Lz0 theta + bz (vertical diffusion per unit volume), tk = tau*kappa.

    Row k: Lz0 couples theta_{k-1}, theta_k, theta_{k+1} through
    (theta_{k+1}-theta_k)/(hz_k dc_{k+1}) - (theta_k-theta_{k-1})/(hz_k dc_k);
    a Dirichlet wall adds -theta/(hz dc_wall) and the source T_wall/(hz dc_wall)."""
    hz, dc = g.z.h, g.z.dc
    nz = hz.size
    sub = np.zeros(nz)
    sup = np.zeros(nz)
    sub[1:] = -tk / (hz[1:] * dc[1:nz])
    sup[:-1] = -tk / (hz[:-1] * dc[1:nz])
    diag = 1.0 - sub - sup
    bz = np.zeros(nz)
    if p.bc_bot == DIRICHLET:
        diag[0] += tk / (hz[0] * dc[0])
        bz[0] += p.t_bot / (hz[0] * dc[0])
    if p.bc_top == DIRICHLET:
        diag[-1] += tk / (hz[-1] * dc[nz])
        bz[-1] += p.t_top / (hz[-1] * dc[nz])
    return sub, diag, sup, bz


def lz0(g, p, th):
    """Lz0 theta: the vertical diffusion per unit volume without the wall
    source (row k: the coefficients of I - Lz0 from ``z_matrix`` with tk = 1)."""
    sub, diag, sup, _ = z_matrix(g, 1.0, p)
    out = (1.0 - diag)[:, None, None] * th
    out[1:] -= sub[1:, None, None] * th[:-1]
    out[:-1] -= sup[:-1, None, None] * th[1:]
    return out


def lz0_transpose(g, p, mu):
    """Lz0^T mu (the z system is not symmetric on a stretched grid)."""
    sub, diag, sup, _ = z_matrix(g, 1.0, p)
    out = (1.0 - diag)[:, None, None] * mu
    out[:-1] -= sub[1:, None, None] * mu[1:]      # row k+1 couples column k through sub_{k+1}
    out[1:] -= sup[:-1, None, None] * mu[:-1]     # row k-1 couples column k through sup_{k-1}
    return out


def thomas(sub, diag, sup, r):
    """Solve the tridiagonal system along axis 0 of r (classical Thomas algorithm)."""
    n = diag.size
    cp = np.empty(n)
    dp = np.empty_like(r)
    cp[0] = sup[0] / diag[0]
    dp[0] = r[0] / diag[0]
    for k in range(1, n):
        den = diag[k] - sub[k] * cp[k - 1]
        cp[k] = sup[k] / den
        dp[k] = (r[k] - sub[k] * dp[k - 1]) / den
    x = np.empty_like(r)
    x[-1] = dp[-1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def scalar_step(g, p, n, th_prev, th_cur, u, v, w):
    """theta^{n+1} from theta^{n-1}, theta^n (Eqs. 6-7 with implicit z diffusion):

    (I - (1-w) tau kappa Lz0) theta^{n+1} = a_p theta^{n-1} + a_c theta^n
        + tau [C(theta^n) + kappa Lh(theta^lag) + w kappa Lz0(theta^lag) + kappa bz]
    with theta^lag = theta^{n-1} (theta^0 at n = 0), w = p.z_explicit;
    th_prev is ignored at n = 0."""
    tau, ap, ac, _ = step_kind(n, p.n_avg, p.dt)
    lag = th_cur if n == 0 else th_prev
    r = ac * th_cur + tau * (advection(g, th_cur, u, v, w, p.face_order) + p.kappa * lap_h(g, lag))
    if n > 0:
        r = r + ap * th_prev
    wz = p.z_explicit
    if wz:
        r = r + (tau * p.kappa * wz) * lz0(g, p, lag)
    sub, diag, sup, bz = z_matrix(g, tau * p.kappa * (1.0 - wz), p)
    r = r + (tau * p.kappa) * bz[:, None, None]
    return thomas(sub, diag, sup, r)


# ------------------------------------------------------------------- Nusselt
def nusselt(g, p, th, w):
    """Heat-flux Nusselt number on every dense z face (Eq. 22, instantaneous):

    Nu_k = (Ra Pr)^(1/2) <w_k theta_f> - <(theta_k - theta_{k-1})/dc_k>,
    <.> the area-weighted mean over x and y, theta_f the mean of the two cells;
    at the plates the gradient uses the wall value and half a cell.
    Returns (profile[0..nz], dict(nu_bot, nu_top, nu_vol, nu_paper, mean_theta)).
    Sums are exact-rounded (math.fsum)."""
    nz = th.shape[0]
    area = g.area_xy()
    atot = math.fsum(area.ravel())
    dc = g.z.dc
    sq = math.sqrt(p.ra * p.pr)
    prof = np.zeros(nz + 1)
    for k in range(1, nz):
        conv = math.fsum((w[k] * 0.5 * (th[k - 1] + th[k]) * area).ravel()) / atot
        grad = math.fsum(((th[k] - th[k - 1]) / dc[k] * area).ravel()) / atot
        prof[k] = sq * conv - grad
    if p.bc_bot == DIRICHLET:
        prof[0] = -math.fsum(((th[0] - p.t_bot) / dc[0] * area).ravel()) / atot
    if p.bc_top == DIRICHLET:
        prof[nz] = -math.fsum(((p.t_top - th[-1]) / dc[nz] * area).ravel()) / atot
    vol = g.vol()
    out = dict(
        nu_bot=prof[0],
        nu_top=prof[nz],
        nu_vol=math.fsum(dc * prof),
        nu_paper=math.fsum(prof[1:nz]) / (nz - 1),
        mean_theta=math.fsum((th * vol).ravel()) / math.fsum(vol.ravel()),
    )
    return prof, out


# ------------------------------------------------------------------- adjoint
def _lap_h_transpose(g, mu):
    """Lh^T mu, written as the transpose of the face-flux form of ``lap_h``."""
    ax, ay, _ = _areas(g)
    q = mu / g.vol()
    px, py = g.x.periodic, g.y.periodic
    if px and py:
        tx = ax / g.x.dc[None, None, :] * (np.roll(q, 1, axis=2) - q)   # face i: d/d theta_i
        ty = ay / g.y.dc[None, :, None] * (np.roll(q, 1, axis=1) - q)
        return (tx - np.roll(tx, -1, axis=2)) + (ty - np.roll(ty, -1, axis=1))
    # face f (cells lo, hi) carries F_f = w_f (theta_hi - theta_lo), added to lo's
    # balance and subtracted from hi's; sum(q * Lh theta) = sum_f F_f (q_lo - q_hi),
    # so with t_f = w_f (q_lo - q_hi) cell hi receives +t_f and cell lo -t_f
    out = np.zeros_like(mu)
    for axis, d, a, per in ((2, g.x.dc[None, None, :], ax, px), (1, g.y.dc[None, :, None], ay, py)):
        lo, hi = _sides(q, axis, per)
        t = _open(a / d * (lo - hi), axis, per)
        out = out + _to_cells(-t, t, axis, per)
    return out


def _advection_transpose(g, mu, u, v, w, order=2):
    """C_u^T mu: each face f (cells L, R) gives s_f = u_f A_f (q_R - q_L)/2 to both
    cells (order 2), or s_f times its stencil weights to its stencil cells
    (order 4); wall faces give nothing."""
    if order == 4:
        return _advection4_transpose(g, mu, u, v, w)
    ax, ay, az = _areas(g)
    q = mu / g.vol()
    nz = mu.shape[0]
    sz = np.zeros((nz + 1,) + mu.shape[1:])
    sz[1:nz] = 0.5 * w[1:nz] * az[None] * (q[1:] - q[:-1])
    px, py = g.x.periodic, g.y.periodic
    if px and py:
        sx = 0.5 * u * ax * (q - np.roll(q, 1, axis=2))
        sy = 0.5 * v * ay * (q - np.roll(q, 1, axis=1))
        return (sx + np.roll(sx, -1, axis=2)) + (sy + np.roll(sy, -1, axis=1)) + (sz[1:] + sz[:-1])
    out = sz[1:] + sz[:-1]
    for axis, vel, a, per in ((2, u, ax, px), (1, v, ay, py)):
        lo, hi = _sides(q, axis, per)
        sf = _open(0.5 * vel * a * (hi - lo), axis, per)
        out = out + _to_cells(sf, sf, axis, per)
    return out


def _advection4_transpose(g, mu, u, v, w):
    """sum(mu * C(theta)) = sum_f s_f theta_f with s_f = u_f A_f (q_R - q_L), so
    C^T mu is the transposed face interpolation of s."""
    ax, ay, az = _areas(g)
    q = mu / g.vol()
    px, py = g.x.periodic, g.y.periodic
    out = np.zeros_like(mu)
    for axis, vel, a, per, axo in ((2, u, ax, px, g.x), (1, v, ay, py, g.y), (0, w, az[None], False, g.z)):
        lo, hi = _sides(q, axis, per)
        sf = _open(vel * a * (hi - lo), axis, per)
        out = out + face_values_transpose(axo, sf, axis, 4)
    return out


def _advection_velocity_transpose(g, mu, th, order=2):
    """Gradient of sum(mu * C_u(theta)) w.r.t. every dense face velocity:
    A_f theta_f (q_R - q_L) with theta_f the face value of the step's order;
    zero on every wall face."""
    ax, ay, az = _areas(g)
    if order == 4:
        q = mu / g.vol()
        px, py = g.x.periodic, g.y.periodic
        grads = []
        for axis, a, per, axo in ((2, ax, px, g.x), (1, ay, py, g.y), (0, az[None], False, g.z)):
            lo, hi = _sides(q, axis, per)
            grads.append(_open(a * face_values(axo, th, axis, 4) * (hi - lo), axis, per))
        return tuple(grads)
    q = mu / g.vol()
    px, py = g.x.periodic, g.y.periodic
    if px and py:
        gu = ax * 0.5 * (np.roll(th, 1, axis=2) + th) * (q - np.roll(q, 1, axis=2))
        gv = ay * 0.5 * (np.roll(th, 1, axis=1) + th) * (q - np.roll(q, 1, axis=1))
    else:
        tl, th_ = _sides(th, 2, px)
        ql, qh = _sides(q, 2, px)
        gu = _open(ax * 0.5 * (tl + th_) * (qh - ql), 2, px)
        tl, th_ = _sides(th, 1, py)
        ql, qh = _sides(q, 1, py)
        gv = _open(ay * 0.5 * (tl + th_) * (qh - ql), 1, py)
    nz = th.shape[0]
    gw = np.zeros((nz + 1,) + th.shape[1:])
    gw[1:nz] = az[None] * 0.5 * (th[:-1] + th[1:]) * (q[1:] - q[:-1])
    return gu, gv, gw


def step_vjp(g, p, n, th_cur, u, v, w, lam_next):
    """Vector-Jacobian product of ``scalar_step`` at step n.

    Given lam_next = dL/dtheta^{n+1}, returns (g_prev, g_cur, gu, gv, gw) with
    mu = (I - (1-w) tau kappa Lz0)^-T lam_next,
    g_prev = a_p mu + tau kappa (Lh^T + w Lz0^T) mu      (n >= 1; zero at n = 0)
    g_cur  = a_c mu + tau C_u^T mu (+ tau kappa (Lh^T + w Lz0^T) mu at n = 0)
    g_vel  = tau dC/du^T mu on every dense face.
    The tridiagonal transpose is formed explicitly (the matrix is not symmetric
    on a stretched grid)."""
    tau, ap, ac, _ = step_kind(n, p.n_avg, p.dt)
    wz = p.z_explicit
    sub, diag, sup, _ = z_matrix(g, tau * p.kappa * (1.0 - wz), p)
    sub_t = np.zeros_like(sub)
    sup_t = np.zeros_like(sup)
    sub_t[1:] = sup[:-1]
    sup_t[:-1] = sub[1:]
    mu = thomas(sub_t, diag, sup_t, lam_next)
    lh = (tau * p.kappa) * _lap_h_transpose(g, mu)
    if wz:
        lh = lh + (tau * p.kappa * wz) * lz0_transpose(g, p, mu)
    g_cur = ac * mu + tau * _advection_transpose(g, mu, u, v, w, p.face_order)
    if n == 0:
        g_cur = g_cur + lh
        g_prev = np.zeros_like(mu)
    else:
        g_prev = ap * mu + lh
    gu, gv, gw = _advection_velocity_transpose(g, mu, th_cur, p.face_order)
    return g_prev, g_cur, tau * gu, tau * gv, tau * gw


# ------------------------------------------------------------------- rollout
def rollout(g, p, th0, u, v, w, nsteps, keep=False):
    """theta^nsteps from theta^0 with a frozen dense velocity (all levels if keep)."""
    levels = [th0]
    prev, cur = th0, th0
    for n in range(nsteps):
        nxt = scalar_step(g, p, n, prev, cur, u, v, w)
        prev, cur = cur, nxt
        if keep:
            levels.append(nxt)
    return levels if keep else cur


def rollout_loss_grad(g, p, th0, U, V, W, nsteps, target):
    """Loss 0.5*||theta^N - target||^2 of refine + N steps, and its gradient
    w.r.t. theta^0 and the coarse (U, V, W), by the discrete adjoint."""
    from .refine import refine_velocity, refine_velocity_transpose
    u, v, w = refine_velocity(g, U, V, W)
    th = rollout(g, p, th0, u, v, w, nsteps, keep=True)
    resid = th[nsteps] - target
    loss = 0.5 * math.fsum((resid * resid).ravel())
    lam = [np.zeros_like(th0) for _ in range(nsteps + 1)]
    lam[nsteps] = resid.copy()
    gu = np.zeros_like(u)
    gv = np.zeros_like(v)
    gw = np.zeros_like(w)
    for n in range(nsteps - 1, -1, -1):
        g_prev, g_cur, du, dv, dw = step_vjp(g, p, n, th[n], u, v, w, lam[n + 1])
        lam[n] += g_cur
        if n >= 1:
            lam[n - 1] += g_prev
        gu += du
        gv += dv
        gw += dw
    gU, gV, gW = refine_velocity_transpose(g, gu, gv, gw)
    return loss, lam[0], gU, gV, gW
