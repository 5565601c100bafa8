"""Seeded synthetic inputs for the multiple-resolution scalar step.

This module builds the *inputs* that both the HIP library and the CPU oracle
consume; it contains none of the method's arithmetic (no refinement, no flux,
no time stepping).  It makes:

* face coordinates: uniform in x and y, a tanh law in z that clusters faces at
  the walls, with every M-th dense face a coarse face (paper Sec. 3.1);
* a staggered velocity on any such grid that is exactly divergence-free: the
  discrete curl (Stokes' theorem on each face) of a seeded random vector
  potential with Gaussian Fourier modes of amplitude |k|^(-11/6) up to kmax,
  multiplied by sin^2(pi xi) in the computational z coordinate so that the
  normal velocity vanishes at the walls, scaled to a given rms velocity;
* the scalar's initial field, the conduction profile 1 - z plus seeded
  Gaussian noise;
* a fixed time step at a given CFL number, estimated from the coarse face
  velocities and the dense cell widths.

Seeds: velocity 1, scalar noise 2, scalar target 3, finite-difference
directions 4.
"""
import numpy as np

SEED_VELOCITY = 1
SEED_THETA = 2
SEED_TARGET = 3
SEED_DIRECTIONS = 4


# --------------------------------------------------------------------------- grids
def uniform_faces(n):
    """n+1 equally spaced faces on [0, 1]."""
    return np.arange(n + 1, dtype=np.float64) / n


def tanh_faces(n, gamma):
    """n+1 faces on [0, 1] clustered at both ends: z_k = (1 + tanh(g(2k/n-1))/tanh g)/2."""
    if gamma == 0.0:
        return uniform_faces(n)
    s = 2.0 * np.arange(n + 1, dtype=np.float64) / n - 1.0
    z = 0.5 * (1.0 + np.tanh(gamma * s) / np.tanh(gamma))
    z[0], z[-1] = 0.0, 1.0
    return z


def workload_faces(w):
    """Dense face coordinates (xf, yf, zf) of a workload."""
    nx, ny, nz = w.n
    return uniform_faces(nx), uniform_faces(ny), tanh_faces(nz, w.gamma)


# --------------------------------------------------------------------- velocity
def _potential_coefficients(kmax, seed):
    """Complex Gaussian coefficients of the three potential components on the
    integer box |k_i| <= kmax, amplitude |k|^(-11/6), zero outside 1<=|k|<=kmax.
    The draw order is fixed, so a seed gives the same modes on every grid."""
    rng = np.random.default_rng(seed)
    kk = np.arange(-kmax, kmax + 1)
    nk = kk.size
    c = rng.standard_normal((3, nk, nk, nk)) + 1j * rng.standard_normal((3, nk, nk, nk))
    kz, ky, kx = np.meshgrid(kk, kk, kk, indexing="ij")
    mag = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.where((mag >= 1.0) & (mag <= kmax), np.power(np.maximum(mag, 1.0), -11.0 / 6.0), 0.0)
    return c * amp[None], kk


def _evaluate(coef, kk, n3, shift):
    """Real part of sum_k coef_k exp(2 pi i k.(idx + shift)/n) on the lattice of
    n3 = (nz, ny, nx) points (z, y, x order), via one inverse FFT."""
    nz, ny, nx = n3
    kmax = (kk.size - 1) // 2
    if min(n3) < 2 * kmax + 1:
        raise ValueError("lattice too small for kmax=%d" % kmax)
    sz, sy, sx = shift
    spec = np.zeros((nz, ny, nx), dtype=np.complex128)
    pz = np.exp(2j * np.pi * kk * sz / nz)
    py = np.exp(2j * np.pi * kk * sy / ny)
    px = np.exp(2j * np.pi * kk * sx / nx)
    ph = pz[:, None, None] * py[None, :, None] * px[None, None, :]
    iz = (kk % nz)[:, None, None]
    iy = (kk % ny)[None, :, None]
    ix = (kk % nx)[None, None, :]
    spec[iz, iy, ix] = coef * ph
    return np.real(np.fft.ifftn(spec)) * (nx * ny * nz)


def divergence_free_velocity(xf, yf, zf, kmax, urms=0.2, seed=SEED_VELOCITY):
    """Staggered (U, V, W) on the grid with faces xf, yf, zf (x, y periodic).

    U[k, j, i] is the mean normal velocity on the x-face at xf[i] of cell
    (i, j, k); V on the y-face at yf[j]; W[k, j, i] on the z-face at zf[k],
    k = 0..nz (W = 0 on both walls).  Shapes: U, V (nz, ny, nx); W (nz+1, ny, nx).
    The face fluxes are circulations of the potential around the face edges,
    so every cell's outward flux sums to zero up to rounding.
    """
    xf, yf, zf = (np.asarray(a, dtype=np.float64) for a in (xf, yf, zf))
    nx, ny, nz = xf.size - 1, yf.size - 1, zf.size - 1
    hx, hy, hz = np.diff(xf), np.diff(yf), np.diff(zf)
    coef, kk = _potential_coefficients(kmax, seed)
    # potential components at edge midpoints, on the (x, y, xi) index lattice;
    # xi = k/nz is the computational z coordinate of face k
    ax = _evaluate(coef[0], kk, (nz, ny, nx), (0.0, 0.0, 0.5))   # x-edges (xc, y_j, z_k)
    ay = _evaluate(coef[1], kk, (nz, ny, nx), (0.0, 0.5, 0.0))   # y-edges (x_i, yc, z_k)
    az = _evaluate(coef[2], kk, (nz, ny, nx), (0.5, 0.0, 0.0))   # z-edges (x_i, y_j, zc)
    xi_f = np.arange(nz + 1) / nz
    wall = np.sin(np.pi * xi_f) ** 2
    wall[0] = wall[-1] = 0.0
    xi_c = (np.arange(nz) + 0.5) / nz
    ax = np.concatenate([ax, ax[:1]], axis=0) * wall[:, None, None]
    ay = np.concatenate([ay, ay[:1]], axis=0) * wall[:, None, None]
    az = az * (np.sin(np.pi * xi_c) ** 2)[:, None, None]
    # edge circulations
    gx = ax * hx[None, None, :]            # (nz+1, ny, nx)
    gy = ay * hy[None, :, None]            # (nz+1, ny, nx)
    gz = az * hz[:, None, None]            # (nz, ny, nx)
    # face fluxes (Stokes), x and y periodic
    fx = (np.roll(gz, -1, axis=1) - gz) - (gy[1:] - gy[:-1])
    fy = (gx[1:] - gx[:-1]) - (np.roll(gz, -1, axis=2) - gz)
    fz = (np.roll(gy, -1, axis=2) - gy) - (np.roll(gx, -1, axis=1) - gx)
    U = fx / (hy[None, :, None] * hz[:, None, None])
    V = fy / (hz[:, None, None] * hx[None, None, :])
    W = fz / (hx[None, None, :] * hy[None, :, None])
    W[0] = 0.0
    W[-1] = 0.0
    # rms of the cell-centred velocity, volume weighted
    uc = 0.5 * (U + np.roll(U, -1, axis=2))
    vc = 0.5 * (V + np.roll(V, -1, axis=1))
    wc = 0.5 * (W[1:] + W[:-1])
    vol = hz[:, None, None] * hy[None, :, None] * hx[None, None, :]
    rms = np.sqrt(np.sum((uc * uc + vc * vc + wc * wc) * vol) / np.sum(vol))
    s = urms / rms
    return U * s, V * s, W * s


def coarse_velocity(w, seed=SEED_VELOCITY):
    """Coarse staggered velocity of a workload (faces every M-th dense face)."""
    xf, yf, zf = workload_faces(w)
    mx, my, mz = w.m
    return divergence_free_velocity(xf[::mx], yf[::my], zf[::mz], w.kmax, w.urms, seed)


# ------------------------------------------------------------------------ scalar
def theta_initial(zf, nx, ny, noise=0.02, seed=SEED_THETA):
    """(1 - z_c) plus N(0, noise^2) on the dense cells, shape (nz, ny, nx)."""
    zf = np.asarray(zf, dtype=np.float64)
    zc = 0.5 * (zf[1:] + zf[:-1])
    rng = np.random.default_rng(seed)
    th = rng.standard_normal((zc.size, ny, nx))
    th *= noise
    th += (1.0 - zc)[:, None, None]
    return th


def workload_theta(w, seed=SEED_THETA):
    nx, ny, nz = w.n
    _, _, zf = workload_faces(w)
    return theta_initial(zf, nx, ny, w.noise, seed)


# --------------------------------------------------------------------- time step
def cfl_dt(U, V, W, xf, yf, zf, m, cfl=0.3):
    """Fixed time step dt = cfl / max over coarse cells of
    sum_a max|face velocity on the two a-faces| / (smallest dense width in the cell)."""
    mx, my, mz = m
    hx, hy, hz = np.diff(xf), np.diff(yf), np.diff(zf)
    ncx, ncy, ncz = hx.size // mx, hy.size // my, hz.size // mz
    hxm = hx.reshape(ncx, mx).min(axis=1)
    hym = hy.reshape(ncy, my).min(axis=1)
    hzm = hz.reshape(ncz, mz).min(axis=1)
    au = np.maximum(np.abs(U), np.abs(np.roll(U, -1, axis=2)))
    av = np.maximum(np.abs(V), np.abs(np.roll(V, -1, axis=1)))
    aw = np.maximum(np.abs(W[1:]), np.abs(W[:-1]))
    rate = au / hxm[None, None, :] + av / hym[None, :, None] + aw / hzm[:, None, None]
    return float(cfl / rate.max())


def workload_inputs(w):
    """Everything one run of a workload needs, in FP64 host arrays."""
    xf, yf, zf = workload_faces(w)
    U, V, W = coarse_velocity(w)
    th0 = workload_theta(w)
    dt = cfl_dt(U, V, W, xf, yf, zf, w.m, w.cfl)
    return dict(xf=xf, yf=yf, zf=zf, U=U, V=V, W=W, theta0=th0, dt=dt)
