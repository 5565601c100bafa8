"""Inter-grid steps around the dense scalar step, and the dissipation Nusselt number.

Follows the paper's multiple-resolution time loop (Sec. 3, flow chart Fig. 6):

* upscale integration of the scalar (Sec. 3.3, Eq. 20): the coarse scalar of a
  coarse cell is the average of its dense cells' scalars weighted by their
  volumes (finite-volume cell averages);
* temporal strategy (Sec. 3.4, Eq. 21): the scalar takes M_t steps per coarse
  (momentum) step, and the coarse velocity at the end of sub-step i is the
  linear interpolation in time between the two coarse velocity levels;
* the global dissipation check of Sec. 4.1 (Eq. 23): Nu_T = eps_T (Ra Pr)^(1/2),
  eps_T = kappa <|grad theta|^2>_V.

Readings (each also listed in the design notes):
* Eq. 20 as printed multiplies by the sub-cell widths (with a y index typo) and
  does not divide by anything; since the scalar is a cell average, the coarse
  value is the volume-weighted mean (sum of theta * dense volume over the
  sub-cells, divided by the coarse volume);
* Eq. 21 as printed adds (i/M_t) U^n to U^{n-1}; the reading is the linear
  interpolation (1 - s) U^{n-1} + s U^n with s = i/M_t, i = 1..M_t, which keeps
  the velocity divergence-free (the property the paper states) and gives U^n
  at i = M_t; sub-step i (the step that ends at fraction i/M_t of the coarse
  step) uses the velocity of fraction i/M_t;
* |grad theta|^2 on the staggered grid: each face contributes the squared
  difference quotient across it, times its dual volume (face area times the
  centre-to-centre distance); the plates use the wall value at half a cell
  (Dirichlet) or contribute nothing (adiabatic).  The dual volumes tile the
  domain once per direction, so a linear profile gives its exact gradient.

Test infrastructure only; all arithmetic float64, plain NumPy.
"""
import math

import numpy as np

from .refine import refine_velocity
from .scalar import DIRICHLET, scalar_step


# ------------------------------------------------------------- Eq. 20 (reading)
def integrate_scalar(g, th):
    """Coarse scalar Tc[K, J, I] = sum over the sub-cells of theta * hx hy hz,
    divided by the coarse volume HX HY HZ (Eq. 20, volume-weighted mean)."""
    th = np.asarray(th, dtype=np.float64)
    x, y, z = g.x, g.y, g.z
    weighted = th * g.vol()
    sums = weighted.reshape(z.nc, z.m, y.nc, y.m, x.nc, x.m).sum(axis=(1, 3, 5))
    coarse_vol = z.H[:, None, None] * y.H[None, :, None] * x.H[None, None, :]
    return sums / coarse_vol


# ------------------------------------------------------------- Eq. 21 (reading)
def blend_velocity(U0, V0, W0, U1, V1, W1, i, mt):
    """Coarse velocity at fraction s = i/M_t of the coarse step:
    (1 - s) * level0 + s * level1, for each of the three components (Eq. 21)."""
    if mt < 1 or not 0 <= i <= mt:
        raise ValueError("need 0 <= i <= M_t and M_t >= 1")
    s = i / mt
    return tuple((1.0 - s) * np.asarray(a, dtype=np.float64) + s * np.asarray(b, dtype=np.float64)
                 for a, b in ((U0, U1), (V0, V1), (W0, W1)))


def coarse_step(g, p, n0, mt, th_prev, th_cur, U0, V0, W0, U1, V1, W1):
    """One coarse step of the multiple-resolution loop (Fig. 6) for the scalar:
    for i = 1..M_t, interpolate the coarse velocity to fraction (i-1)/M_t of the
    coarse step (Eq. 21), refine it to the dense grid (Sec. 3.2) and take scalar
    step n0 + i - 1 (Eqs. 6-7, with p.dt the scalar time step, i.e. the coarse
    step over M_t); then integrate the newest scalar to the coarse grid (Eq. 20).
    Sub-step i advances the scalar from time level n0 + i - 1, and the
    advection C(theta^n) of Eqs. 5-7 is taken at level n, so its velocity is the
    one at the start of the sub-step: fractions 0, 1/M_t, ..., (M_t-1)/M_t.
    Returns (theta^{n0+mt-1}, theta^{n0+mt}, Tc)."""
    prev, cur = th_prev, th_cur
    for i in range(1, mt + 1):
        U, V, W = blend_velocity(U0, V0, W0, U1, V1, W1, i - 1, mt)
        u, v, w = refine_velocity(g, U, V, W)
        nxt = scalar_step(g, p, n0 + i - 1, prev, cur, u, v, w)
        prev, cur = cur, nxt
    return prev, cur, integrate_scalar(g, cur)


# ---------------------------------------------------------- Eq. 23 (Sec. 4.1)
def thermal_dissipation(g, p, th):
    """Nu_T = eps_T (Ra Pr)^(1/2) with eps_T = kappa <|grad theta|^2>_V (Eq. 23).

    <.>_V is the volume mean; the squared gradient is summed face by face:
    x faces ((theta_i - theta_{i-1}) / dcx_i)^2 * dcx_i * hy * hz (periodic),
    y faces likewise, z faces ((theta_k - theta_{k-1}) / dcz_k)^2 * dcz_k * hx * hy
    for 0 < k < nz, and at a Dirichlet plate the difference to the wall value
    over half a cell; a side wall (walled x or y) adds nothing.  Returns
    dict(nu_t, gx2, gy2, gz2) with g*2 the volume
    means of the three squared components; sums are exact-rounded (fsum)."""
    th = np.asarray(th, dtype=np.float64)
    x, y, z = g.x, g.y, g.z
    nz = th.shape[0]
    hx = x.h[None, None, :]
    hy = y.h[None, :, None]
    hz = z.h[:, None, None]
    if x.periodic:
        dx = th - np.roll(th, 1, axis=2)                 # x face i: cells i-1, i
        ex = dx * dx / x.dc[None, None, :] * hy * hz
    else:                                                # interior faces 1..nx-1; walls add nothing
        dx = th[:, :, 1:] - th[:, :, :-1]
        ex = dx * dx / x.dc[None, None, 1:-1] * hy * hz
    if y.periodic:
        dy = th - np.roll(th, 1, axis=1)
        ey = dy * dy / y.dc[None, :, None] * hx * hz
    else:
        dy = th[:, 1:, :] - th[:, :-1, :]
        ey = dy * dy / y.dc[None, 1:-1, None] * hx * hz
    area = g.area_xy()
    terms_z = []
    for k in range(1, nz):
        d = th[k] - th[k - 1]
        terms_z.append((d * d / z.dc[k] * area).ravel())
    if p.bc_bot == DIRICHLET:
        d = th[0] - p.t_bot
        terms_z.append((d * d / z.dc[0] * area).ravel())
    if p.bc_top == DIRICHLET:
        d = p.t_top - th[nz - 1]
        terms_z.append((d * d / z.dc[nz] * area).ravel())
    vtot = math.fsum(g.vol().ravel())
    gx2 = math.fsum(ex.ravel()) / vtot
    gy2 = math.fsum(ey.ravel()) / vtot
    gz2 = math.fsum(np.concatenate(terms_z)) / vtot if terms_z else 0.0
    eps_t = p.kappa * (gx2 + gy2 + gz2)
    return dict(nu_t=eps_t * math.sqrt(p.ra * p.pr), gx2=gx2, gy2=gy2, gz2=gz2)
