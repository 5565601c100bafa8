"""Pins of the oracle's inter-grid steps (paper Eqs. 20, 21, Fig. 6) and of the
dissipation Nusselt number (Eq. 23) to closed forms, invariants, special cases
and the independently pinned operators of the scalar step."""
import math

import numpy as np
import pytest

import oracle as O
from oracle.intergrid import blend_velocity, coarse_step, integrate_scalar, thermal_dissipation
from paper_1805_03426_amd import inputs

EPS = np.finfo(np.float64).eps


def _stretched_faces(n, rng, lo=0.0, hi=1.0):
    h = rng.uniform(0.5, 2.0, n)
    f = np.concatenate([[0.0], np.cumsum(h)])
    return lo + (hi - lo) * f / f[-1]


def _grid(nc, m, rng, gamma=1.5, stretch_xy=True):
    ncx, ncy, ncz = nc
    mx, my, mz = m
    xf = _stretched_faces(ncx * mx, rng) if stretch_xy else inputs.uniform_faces(ncx * mx)
    yf = _stretched_faces(ncy * my, rng) if stretch_xy else inputs.uniform_faces(ncy * my)
    zf = inputs.tanh_faces(ncz * mz, gamma)
    return O.Grid(xf, yf, zf, m)


# ------------------------------------------------------------------ Eq. 20
@pytest.mark.parametrize("m", [(2, 2, 2), (3, 2, 4), (2, 3, 1)])
def test_integration_of_linear_fields_is_exact(m):
    """A field linear in x, y and z integrates to its value at the coarse cell
    centre (the mean of a linear function over an interval is its midpoint
    value), on grids stretched in every direction; an unweighted mean of the
    sub-cells fails this on a stretched grid."""
    rng = np.random.default_rng(1)
    g = _grid((5, 4, 6), m, rng)
    a, b, c, d = 0.3, -1.7, 2.2, -0.9
    th = a + b * g.x.c[None, None, :] + c * g.y.c[None, :, None] + d * g.z.c[:, None, None]
    tc = integrate_scalar(g, th)
    XC = 0.5 * (g.x.cf[1:] + g.x.cf[:-1])
    YC = 0.5 * (g.y.cf[1:] + g.y.cf[:-1])
    ZC = 0.5 * (g.z.cf[1:] + g.z.cf[:-1])
    want = a + b * XC[None, None, :] + c * YC[None, :, None] + d * ZC[:, None, None]
    assert np.abs(tc - want).max() < 32 * EPS
    # the conduction profile 1 - z gives 1 - Z at the coarse centres
    tc = integrate_scalar(g, np.broadcast_to(1.0 - g.z.c[:, None, None], g.shape))
    assert np.abs(tc - (1.0 - ZC)[:, None, None]).max() < 8 * EPS
    # plain averaging of the sub-cells differs on this grid
    sh = (g.z.nc, g.z.m, g.y.nc, g.y.m, g.x.nc, g.x.m)
    plain = th.reshape(sh).mean(axis=(1, 3, 5))
    assert np.abs(plain - (a + b * XC[None, None, :] + c * YC[None, :, None] + d * ZC[:, None, None])).max() > 1e-4


def test_integration_conserves_total_scalar():
    """sum(Tc * coarse volume) = sum(theta * dense volume) (the integral of the
    scalar over the domain is unchanged)."""
    rng = np.random.default_rng(2)
    g = _grid((6, 5, 4), (3, 2, 2), rng)
    th = rng.standard_normal(g.shape)
    tc = integrate_scalar(g, th)
    cvol = g.z.H[:, None, None] * g.y.H[None, :, None] * g.x.H[None, None, :]
    lhs = math.fsum((tc * cvol).ravel())
    rhs = math.fsum((th * g.vol()).ravel())
    assert abs(lhs - rhs) < 64 * EPS * math.fsum(np.abs(th * g.vol()).ravel())


def test_integration_m1_is_identity_and_constants_stay():
    rng = np.random.default_rng(3)
    g1 = _grid((4, 3, 5), (1, 1, 1), rng)
    th = rng.standard_normal(g1.shape)
    assert np.abs(integrate_scalar(g1, th) - th).max() < 4 * EPS * np.abs(th).max()
    g = _grid((4, 3, 5), (2, 3, 2), rng)
    tc = integrate_scalar(g, np.full(g.shape, 0.625))
    assert np.abs(tc - 0.625).max() < 8 * EPS


# ------------------------------------------------------------------ Eq. 21
def _levels(g, seed0=11, seed1=12, kmax=2):
    a = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=kmax, seed=seed0)
    b = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=kmax, seed=seed1)
    return a, b


def test_blend_end_levels_and_midpoint_are_exact():
    """i = 0 gives U^{n-1} and i = M_t gives U^n bit for bit; the midpoint of
    M_t = 2 is the exact average (the reading of Eq. 21; the printed form would
    give U^{n-1} + U^n at i = M_t)."""
    g = _grid((6, 5, 6), (2, 2, 2), np.random.default_rng(4), stretch_xy=False)
    (U0, V0, W0), (U1, V1, W1) = _levels(g)
    for mt in (1, 2, 3, 5):
        end = blend_velocity(U0, V0, W0, U1, V1, W1, mt, mt)
        start = blend_velocity(U0, V0, W0, U1, V1, W1, 0, mt)
        for a, b in zip(end, (U1, V1, W1)):
            assert np.array_equal(a, b)
        for a, b in zip(start, (U0, V0, W0)):
            assert np.array_equal(a, b)
    mid = blend_velocity(U0, V0, W0, U1, V1, W1, 1, 2)
    for a, b0, b1 in zip(mid, (U0, V0, W0), (U1, V1, W1)):
        assert np.array_equal(a, (b0 + b1) / 2)
    with pytest.raises(ValueError):
        blend_velocity(U0, V0, W0, U1, V1, W1, 3, 2)


@pytest.mark.parametrize("mt", [2, 3])
def test_blended_velocity_stays_divergence_free_and_linear(mt):
    """Every intermediate coarse velocity refines to a divergence-free dense
    field (the property stated with Eq. 21), and the refined field is the same
    linear combination of the two refined levels (the refinement is linear)."""
    g = _grid((8, 7, 6), (2, 3, 2), np.random.default_rng(5), stretch_xy=False)
    (U0, V0, W0), (U1, V1, W1) = _levels(g)
    d0 = O.refine_velocity(g, U0, V0, W0)
    d1 = O.refine_velocity(g, U1, V1, W1)
    for i in range(1, mt + 1):
        s = i / mt
        u, v, w = O.refine_velocity(g, *blend_velocity(U0, V0, W0, U1, V1, W1, i, mt))
        div, tot = O.divergence(g, u, v, w)
        assert np.max(np.abs(div) / tot) < 64 * EPS
        for a, b0, b1 in zip((u, v, w), d0, d1):
            assert np.abs(a - ((1 - s) * b0 + s * b1)).max() < 1e-14 * max(np.abs(b0).max(), 1.0)


def test_coarse_step_with_steady_velocity_is_the_rollout():
    """With U^{n-1} = U^n every sub-step sees the same refined velocity, so M_t
    sub-steps from n0 = 0 are the plain rollout of M_t steps (pinned on its
    own), and Tc is its integration; continuing from n0 = M_t with the ring
    (theta^{n-1}, theta^n) matches a 2 M_t-step rollout, averaging step included."""
    g = _grid((6, 5, 5), (2, 2, 2), np.random.default_rng(6), stretch_xy=False)
    U, V, W = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=2, seed=13)
    p = O.ScalarParams.from_ra_pr(1e5, 1.0, 2e-3, n_avg=5)
    th0 = inputs.theta_initial(g.z.faces, g.x.n, g.y.n, seed=2)
    mt = 3
    prev, cur, tc = coarse_step(g, p, 0, mt, th0, th0, U, V, W, U, V, W)
    u, v, w = O.refine_velocity(g, U, V, W)
    levels = O.rollout(g, p, th0, u, v, w, 2 * mt, keep=True)
    # (1 - s) U + s U equals U up to rounding for s = i/3
    tol = 1e-14
    assert np.abs(cur - levels[mt]).max() < tol and np.abs(prev - levels[mt - 1]).max() < tol
    assert np.abs(tc - integrate_scalar(g, levels[mt])).max() < tol
    prev, cur, _ = coarse_step(g, p, mt, mt, prev, cur, U, V, W, U, V, W)
    assert np.abs(cur - levels[2 * mt]).max() < tol and np.abs(prev - levels[2 * mt - 1]).max() < tol
    # M_t = 1 from U to rest: the single sub-step starts at the old level and uses U^{n-1}
    zero = (np.zeros_like(U), np.zeros_like(V), np.zeros_like(W))
    _, cur, _ = coarse_step(g, p, 0, 1, th0, th0, U, V, W, *zero)
    assert np.array_equal(cur, levels[1])


def test_coarse_step_sub_steps_use_the_velocity_at_their_start():
    """Sub-step i of M_t = 3 is scalar step n0 + i - 1 on the refinement of the
    coarse velocity at fraction (i - 1)/3: the steps taken by hand from the
    blended levels 0, 1/3, 2/3 agree to the last bit."""
    g = _grid((6, 5, 5), (2, 2, 2), np.random.default_rng(8), stretch_xy=False)
    (U0, V0, W0), (U1, V1, W1) = _levels(g)
    p = O.ScalarParams.from_ra_pr(1e5, 1.0, 2e-3, n_avg=0)
    th0 = inputs.theta_initial(g.z.faces, g.x.n, g.y.n, seed=2)
    prev, cur, _ = coarse_step(g, p, 0, 3, th0, th0, U0, V0, W0, U1, V1, W1)
    a = b = th0
    for i in range(3):
        uvw = O.refine_velocity(g, *blend_velocity(U0, V0, W0, U1, V1, W1, i, 3))
        a, b = b, O.scalar_step(g, p, i, a, b, *uvw)
    assert np.array_equal(cur, b) and np.array_equal(prev, a)


def test_coarse_step_is_second_order_in_time():
    """With a velocity linear in time over the coarse step and no diffusion
    (kappa ~ 1e-10, adiabatic walls), the leapfrog of Eq. 6 is second order when
    each sub-step advects with the velocity at its own start level: halving the
    sub-step (M_t = 4, 8, 16, 32 against M_t = 256) divides the error by 4.
    Taking the velocity one sub-step later (fraction i/M_t) makes it first
    order (ratio 2, and 18 times the error at M_t = 4), which this pin rejects."""
    n = 16
    g = O.Grid(inputs.uniform_faces(n), inputs.uniform_faces(n), inputs.uniform_faces(n), (1, 1, 1))
    lv0 = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=1, urms=0.2, seed=11)
    lv1 = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=1, urms=0.2, seed=12)
    th0 = (np.cos(2 * np.pi * g.x.c)[None, None, :] * np.cos(2 * np.pi * g.y.c)[None, :, None]
           * np.cos(np.pi * g.z.c)[:, None, None])
    T = 0.2
    res = {}
    for mt in (4, 8, 16, 32, 256):
        p = O.ScalarParams.from_ra_pr(1e20, 1.0, T / mt, n_avg=0, bc_bot="adiabatic", bc_top="adiabatic")
        res[mt] = coarse_step(g, p, 0, mt, th0, th0, *lv0, *lv1)[1]
    err = [np.sqrt(np.mean((res[m] - res[256]) ** 2)) for m in (4, 8, 16, 32)]
    for a, b in zip(err[:-1], err[1:]):
        assert 3.5 < a / b < 4.5, err


def test_coarse_step_keeps_conduction_and_constants():
    """At rest the conduction profile is a fixed point, and Tc = 1 - Z; with a
    time-varying divergence-free velocity a uniform scalar with matching
    adiabatic walls stays uniform (free stream), which needs every
    intermediate velocity to be divergence-free."""
    g = _grid((6, 5, 6), (2, 2, 3), np.random.default_rng(7), stretch_xy=False)
    p = O.ScalarParams.from_ra_pr(1e6, 4.38, 1e-3, n_avg=4)
    zero = (np.zeros((g.z.nc, g.y.nc, g.x.nc)),) * 2 + (np.zeros((g.z.nc + 1, g.y.nc, g.x.nc)),)
    cond = np.broadcast_to(1.0 - g.z.c[:, None, None], g.shape).copy()
    prev, cur, tc = coarse_step(g, p, 0, 4, cond, cond, *zero, *zero)
    assert np.abs(cur - cond).max() < 1e-14
    ZC = 0.5 * (g.z.cf[1:] + g.z.cf[:-1])
    assert np.abs(tc - (1.0 - ZC)[:, None, None]).max() < 1e-14
    (U0, V0, W0), (U1, V1, W1) = _levels(g)
    pa = O.ScalarParams.from_ra_pr(1e6, 4.38, 1e-3, n_avg=4, bc_bot="adiabatic", bc_top="adiabatic")
    const = np.full(g.shape, 0.375)
    prev, cur, tc = coarse_step(g, pa, 0, 3, const, const, U0, V0, W0, U1, V1, W1)
    assert np.abs(cur - 0.375).max() < 1e-13
    assert np.abs(tc - 0.375).max() < 1e-13


# ------------------------------------------------------------------ Eq. 23
@pytest.mark.parametrize("gamma", [0.0, 1.5, 2.5])
def test_dissipation_of_conduction_is_one(gamma):
    """theta = 1 - z (conduction between plates at 1 and 0) has |grad theta| = 1,
    so Nu_T = 1 on any z grid, with no x or y part."""
    g = _grid((5, 4, 8), (2, 2, 2), np.random.default_rng(8), gamma=gamma)
    p = O.ScalarParams.from_ra_pr(1e8, 4.38, 1e-3)
    th = np.broadcast_to(1.0 - g.z.c[:, None, None], g.shape).copy()
    d = thermal_dissipation(g, p, th)
    assert abs(d["nu_t"] - 1.0) < 32 * EPS
    assert d["gx2"] == 0.0 and d["gy2"] == 0.0


def test_dissipation_of_a_fourier_mode():
    """cos(2 pi k x) on a uniform periodic grid: the mean squared difference
    quotient is 2 sin^2(pi k / N) / h^2 (closed form); same in y."""
    n, k = 24, 5
    g = O.Grid(inputs.uniform_faces(n), inputs.uniform_faces(n), inputs.tanh_faces(6, 0.0), (1, 1, 1))
    p = O.ScalarParams.from_ra_pr(1.0, 1.0, 1e-3, bc_bot="adiabatic", bc_top="adiabatic")
    h = 1.0 / n
    want = 2.0 * math.sin(math.pi * k / n) ** 2 / h ** 2
    thx = np.broadcast_to(np.cos(2 * math.pi * k * g.x.c)[None, None, :], g.shape).copy()
    d = thermal_dissipation(g, p, thx)
    assert abs(d["gx2"] - want) < 1e-12 * want and d["gy2"] == 0.0 and d["gz2"] == 0.0
    thy = np.broadcast_to(np.cos(2 * math.pi * k * g.y.c)[None, :, None], g.shape).copy()
    d = thermal_dissipation(g, p, thy)
    assert abs(d["gy2"] - want) < 1e-12 * want and d["gx2"] == 0.0
    assert abs(d["nu_t"] - want) < 1e-12 * want      # kappa (Ra Pr)^(1/2) = 1


@pytest.mark.parametrize("bc", [("dirichlet", "dirichlet"), ("adiabatic", "dirichlet"), ("adiabatic", "adiabatic")])
def test_dissipation_summation_by_parts(bc):
    """The face sum of squared gradients equals -sum theta L theta V plus the
    plate terms A (T_bot Nu_bot - T_top Nu_top), with L the step's horizontal and
    vertical diffusion operators and Nu the plate fluxes of the Nusselt
    diagnostics (discrete Green identity; all three pinned on their own)."""
    rng = np.random.default_rng(9)
    g = _grid((5, 4, 7), (2, 3, 2), rng, gamma=2.0)
    p = O.ScalarParams.from_ra_pr(1e7, 2.0, 1e-3, t_bot=1.3, t_top=-0.2, bc_bot=bc[0], bc_top=bc[1])
    th = rng.standard_normal(g.shape)
    vol = g.vol()
    sub, diag, sup, bz = O.z_matrix(g, 1.0, p)
    lz0 = th - (diag[:, None, None] * th)
    lz0[1:] -= sub[1:, None, None] * th[:-1]
    lz0[:-1] -= sup[:-1, None, None] * th[1:]
    lth = O.lap_h(g, th) + lz0 + bz[:, None, None]
    _, nu = O.nusselt(g, p, th, np.zeros((g.z.n + 1, g.y.n, g.x.n)))
    atot = math.fsum(g.area_xy().ravel())
    rhs = -math.fsum((th * lth * vol).ravel()) + atot * (p.t_bot * nu["nu_bot"] - p.t_top * nu["nu_top"])
    d = thermal_dissipation(g, p, th)
    lhs = (d["gx2"] + d["gy2"] + d["gz2"]) * math.fsum(vol.ravel())
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert abs(d["nu_t"] - p.kappa * math.sqrt(p.ra * p.pr) * (d["gx2"] + d["gy2"] + d["gz2"])) < 1e-15 * d["nu_t"]
