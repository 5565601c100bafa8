"""GPU parity of the inter-grid entry points (Eqs. 20, 21, Fig. 6) and of the
dissipation Nusselt number (Eq. 23) against the oracle, through the C ABI.
Tolerances as for the step: 1e-12 (FP64), 1e-5 (FP32 tier)."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle.intergrid import blend_velocity, coarse_step, integrate_scalar, thermal_dissipation
from paper_1805_03426_amd import inputs
from paper_1805_03426_amd.configs import WORKLOADS
from tests.test_gpu_parity import FP32_TOL, FP64_TOL, Case, dev, host, rel_l2, rel_max

pytestmark = pytest.mark.gpu


def _second_level(case, seed=21):
    g = case.g
    return inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, 2, 0.2, seed)


# ------------------------------------------------------------------ Eq. 20
@pytest.mark.parametrize("nc,m,prec", [((9, 7, 5), (2, 2, 2), "fp64"), ((100, 4, 3), (3, 2, 4), "fp64"),
                                       ((7, 6, 5), (1, 1, 1), "fp64"), ((9, 7, 5), (3, 3, 2), "fp32"),
                                       ((130, 3, 3), (2, 1, 3), "fp32")])
def test_integrate_parity(nc, m, prec):
    """Ragged rows (a workgroup covers 256/mx coarse cells), M = 1, stretched x."""
    print("case integrate", nc, m, prec, flush=True)
    case = Case(nc, m, 1.5, kmax=1, precision=prec, stretch_x=True, random_velocity=True, dt=1e-4)
    rng = np.random.default_rng(5)
    th = case.th0 + 0.3 * rng.standard_normal(case.th0.shape)
    want = integrate_scalar(case.g, th)
    with case.ctx() as ctx:
        got = host(ctx.integrate_scalar(case.d(th)))
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    assert rel_max(got, want) <= tol


def test_integrate_conduction_is_exact():
    case = Case((8, 6, 7), (2, 3, 2), 2.0, kmax=1, random_velocity=True)
    th = np.broadcast_to(1.0 - case.g.z.c[:, None, None], case.g.shape).copy()
    ZC = 0.5 * (case.g.z.cf[1:] + case.g.z.cf[:-1])
    with case.ctx() as ctx:
        got = host(ctx.integrate_scalar(case.d(th)))
    assert np.abs(got - (1.0 - ZC)[:, None, None]).max() < 1e-15


# ------------------------------------------------------------------ Eq. 23
@pytest.mark.parametrize("prec,bc", [("fp64", ("dirichlet", "dirichlet")), ("fp64", ("adiabatic", "dirichlet")),
                                     ("fp32", ("dirichlet", "dirichlet"))])
def test_dissipation_parity(prec, bc):
    print("case dissipation", prec, bc, flush=True)
    case = Case((9, 7, 6), (2, 3, 2), 1.5, kmax=1, precision=prec, bc=bc, stretch_x=True, random_velocity=True, dt=1e-4)
    rng = np.random.default_rng(6)
    th = case.th0 + 0.1 * rng.standard_normal(case.th0.shape)
    if prec == "fp32":
        th = th.astype(np.float32).astype(np.float64)   # the oracle sees the stored values
    want = thermal_dissipation(case.g, case.p, th)
    with case.ctx() as ctx:
        _, got = ctx.thermal_dissipation(case.d(th))
    tol = FP64_TOL if prec == "fp64" else 1e-12   # sums are FP64 in both tiers
    for k in ("nu_t", "gx2", "gy2", "gz2"):
        assert abs(got[k] - want[k]) <= tol * abs(want["nu_t"]), (k, got[k], want[k])


@pytest.mark.parametrize("prec,nc", [("fp64", (640, 80, 120)), ("fp32", (70, 17, 40)), ("fp64", (1, 1, 9))])
def test_dissipation_parity_tiles(prec, nc):
    """Nu_T over several tiles of 64 columns by 8 rows, ragged in x and y, and
    over level ranges of 11 (load batches of 4, 4 and 3 levels) and of 1, and
    on a single column (its own x and y neighbour)."""
    print("case dissipation tiles", prec, nc, flush=True)
    case = Case(nc, (1, 1, 1), 1.5, kmax=1, precision=prec, random_velocity=True, dt=1e-5)
    rng = np.random.default_rng(7)
    th = case.th0 + 0.1 * rng.standard_normal(case.th0.shape)
    if prec == "fp32":
        th = th.astype(np.float32).astype(np.float64)
    want = thermal_dissipation(case.g, case.p, th)
    with case.ctx() as ctx:
        _, got = ctx.thermal_dissipation(case.d(th))
    for k in ("nu_t", "gx2", "gy2", "gz2"):
        assert abs(got[k] - want[k]) <= 1e-12 * abs(want["nu_t"]), (k, got[k], want[k])


def test_dissipation_of_conduction_is_one():
    case = Case((8, 6, 9), (2, 2, 2), 2.5, kmax=1, random_velocity=True)
    th = np.broadcast_to(1.0 - case.g.z.c[:, None, None], case.g.shape).copy()
    with case.ctx() as ctx:
        _, got = ctx.thermal_dissipation(case.d(th))
    assert abs(got["nu_t"] - 1.0) < 1e-14 and got["gx2"] == 0.0 and got["gy2"] == 0.0


# ------------------------------------------------------------------ Eq. 21
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_time_interpolated_refinement_parity(prec):
    print("case refine in time", prec, flush=True)
    case = Case((8, 7, 6), (2, 3, 2), 1.5, kmax=2, precision=prec)
    U1, V1, W1 = _second_level(case)
    mt = 3
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    with case.ctx() as ctx:
        lv0 = [case.d(a) for a in (case.U, case.V, case.W)]
        lv1 = [case.d(a) for a in (U1, V1, W1)]
        for i in range(mt + 1):
            got = ctx.interpolate_velocity_time(*lv0, *lv1, i, mt)
            want = O.refine_velocity(case.g, *blend_velocity(case.U, case.V, case.W, U1, V1, W1, i, mt))
            for a, b in zip(got, want):
                assert rel_max(host(a), b) <= tol
            dv = host(ctx.divergence(*got))
            assert dv[1] < (64 * np.finfo(np.float64).eps if prec == "fp64" else 1e-5)
        # the end levels are the plain refinements, bit for bit
        end = ctx.interpolate_velocity_time(*lv0, *lv1, mt, mt)
        ref = ctx.interpolate_velocity(*lv1)
        start = ctx.interpolate_velocity_time(*lv0, *lv1, 0, mt)
        ref0 = ctx.interpolate_velocity(*lv0)
        for a, b in zip(end + start, ref + ref0):
            assert torch.equal(a, b)


# ------------------------------------------------------------------ Fig. 6
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_coarse_step_parity(prec):
    """Two coarse steps of M_t = 3 (the second from n0 = 3 through an averaging
    step), the ring indices and the integrated scalar, against the oracle."""
    print("case coarse step", prec, flush=True)
    case = Case((8, 7, 6), (2, 2, 2), 1.5, ra=1e5, kmax=2, n_avg=5, precision=prec)
    U1, V1, W1 = _second_level(case)
    U2, V2, W2 = _second_level(case, seed=22)
    mt = 3
    p1, c1, tc1 = coarse_step(case.g, case.p, 0, mt, case.th0, case.th0, case.U, case.V, case.W, U1, V1, W1)
    p2, c2, tc2 = coarse_step(case.g, case.p, mt, mt, p1, c1, U1, V1, W1, U2, V2, W2)
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    with case.ctx() as ctx:
        ring = [case.d(case.th0), ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell)]
        uvw = (ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_w))
        tc = ctx.empty(ctx.shape_coarse)
        lv = [[case.d(a) for a in q] for q in ((case.U, case.V, case.W), (U1, V1, W1), (U2, V2, W2))]
        prev, cur = ctx.coarse_step(0, mt, *lv[0], *lv[1], uvw, ring, 0, 0, tc)
        assert prev != cur
        assert rel_l2(host(ring[cur]), c1) <= tol and rel_l2(host(ring[prev]), p1) <= tol
        assert rel_max(host(tc), tc1) <= tol
        prev, cur = ctx.coarse_step(mt, mt, *lv[1], *lv[2], uvw, ring, prev, cur, tc)
        assert rel_l2(host(ring[cur]), c2) <= tol and rel_l2(host(ring[prev]), p2) <= tol
        assert rel_max(host(tc), tc2) <= tol
        # the last refined velocity is the one of the last sub-step: fraction
        # (M_t - 1) / M_t between the two levels
        want = O.refine_velocity(case.g, *blend_velocity(U1, V1, W1, U2, V2, W2, mt - 1, mt))
        for a, b in zip(uvw, want):
            assert rel_max(host(a), b) <= tol


def test_coarse_step_rejects_bad_rings():
    from paper_1805_03426_amd._lib import MRError
    case = Case((6, 5, 5), (2, 2, 2), 1.0, kmax=1, random_velocity=True)
    with case.ctx() as ctx:
        a = ctx.empty(ctx.shape_cell)
        uvw = (ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_w))
        lv = [case.d(x) for x in (case.U, case.V, case.W)]
        with pytest.raises(MRError):
            ctx.coarse_step(0, 2, *lv, *lv, uvw, [a, a, ctx.empty(ctx.shape_cell)], 0, 0)
        ring = [a, ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell)]
        with pytest.raises(MRError):
            ctx.coarse_step(4, 2, *lv, *lv, uvw, ring, 1, 1)       # n0 > 0 needs two levels
        with pytest.raises(MRError):
            ctx.coarse_step(0, 0, *lv, *lv, uvw, ring, 0, 0)       # mt >= 1


# ------------------------------------------------------------------ full size
def test_full_size_rb256_intergrid():
    """256^3 (M = 2, tanh z): integration and Nu_T of the generator's scalar
    against the oracle, and the time-interpolated refinement on sampled faces."""
    print("case rb256 intergrid full size", flush=True)
    w = WORKLOADS["rb256-m2-fp64"]
    d = inputs.workload_inputs(w)
    g = O.Grid(d["xf"], d["yf"], d["zf"], w.m)
    p = O.ScalarParams.from_ra_pr(w.ra, w.pr, d["dt"], n_avg=w.n_avg)
    from paper_1805_03426_amd.context import Context
    with Context(d["xf"], d["yf"], d["zf"], w.m, w.ra, w.pr, d["dt"], n_avg=w.n_avg) as ctx:
        th = dev(d["theta0"])
        assert rel_max(host(ctx.integrate_scalar(th)), integrate_scalar(g, d["theta0"])) <= FP64_TOL
        _, got = ctx.thermal_dissipation(th)
        want = thermal_dissipation(g, p, d["theta0"])
        for k in ("nu_t", "gx2", "gy2", "gz2"):
            assert abs(got[k] - want[k]) <= FP64_TOL * want["nu_t"], k
        print("rb256 Nu_T %.6f (oracle %.6f)" % (got["nu_t"], want["nu_t"]), flush=True)


def test_full_size_rb256_coarse_step():
    """One coarse step of M_t = 4 scalar steps at 256^3 in the benchmark's
    launch configuration (the second coarse level is the first reversed in z,
    with zero wall planes): the native loop against the oracle's."""
    print("case rb256 coarse step full size", flush=True)
    w = WORKLOADS["rb256-m2-fp64"]
    d = inputs.workload_inputs(w)
    g = O.Grid(d["xf"], d["yf"], d["zf"], w.m)
    p = O.ScalarParams.from_ra_pr(w.ra, w.pr, d["dt"], n_avg=w.n_avg)
    U0, V0, W0 = d["U"], d["V"], d["W"]
    U1, V1, W1 = (np.ascontiguousarray(a[::-1]) for a in (U0, V0, W0))
    W1[0] = W1[-1] = 0.0
    mt = 4
    prev_o, cur_o, tc_o = coarse_step(g, p, 0, mt, d["theta0"], d["theta0"], U0, V0, W0, U1, V1, W1)
    from paper_1805_03426_amd.context import Context
    with Context(d["xf"], d["yf"], d["zf"], w.m, w.ra, w.pr, d["dt"], n_avg=w.n_avg) as ctx:
        uvw = (ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_w))
        ring = [dev(d["theta0"]), ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell)]
        tc = ctx.empty(ctx.shape_coarse)
        pi, ci = ctx.coarse_step(0, mt, *(dev(a) for a in (U0, V0, W0, U1, V1, W1)), uvw, ring, 0, 0, tc)
        assert rel_l2(host(ring[ci]), cur_o) <= FP64_TOL
        assert rel_max(host(ring[ci]), cur_o) <= FP64_TOL
        assert rel_l2(host(ring[pi]), prev_o) <= FP64_TOL
        assert rel_max(host(tc), tc_o) <= FP64_TOL
