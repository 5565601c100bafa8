"""GPU parity of the three-kernel refinement path (stage z, then y, then x,
the intermediates in device memory) on periodic sides, and of the transposed
refinement on the same grids, against the oracle (Sec. 3.2, Fig. 5a,
Eqs. 12-19; Sec. 3.4, Eq. 21).

The library takes this path when the single fused kernel does not apply: a z
refinement factor above 4, or a tile of coarse cells whose stage fields do
not fit the fused kernel's 64 KB LDS budget (for example M = (1, 16, 2) in
FP64).  Tolerances: element-wise relative max <= 1e-12 in FP64, <= 1e-5 in
FP32 (the oracle sees the FP32-rounded coarse input), and the normalised
divergence of every result within the rounding bound below."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.intergrid import blend_velocity
from paper_1805_03426_amd import inputs
from tests.test_gpu_parity import FP32_TOL, FP64_TOL, Case, host, rel_max

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps

# (coarse cells, refinement factors, z stretching): M_z = 5 and 6, and an
# x tile of 64 dense columns with 16 dense rows per coarse row, which exceeds
# the fused kernel's LDS budget in FP64 (two x tiles, the second ragged)
STAGE_CASES = [((5, 4, 4), (2, 2, 5), 1.5), ((4, 3, 3), (3, 2, 6), 2.0), ((70, 3, 3), (1, 16, 2), 1.0)]


def div_bound(m, eps):
    """Bound on max |net flux| / sum |face flux| of a refined cell: every march
    chains up to M - 1 dependent updates along its axis, each adding rounding
    of the order of eps relative to the cell's face fluxes, so the bound grows
    with the factors (the oracle itself reaches 55-61 eps at M = (3, 2, 6) and
    (1, 16, 2)); 64 eps for the small factors of the workloads."""
    return max(64.0, 8.0 * sum(m)) * eps


def _fields(case, prec):
    """Divergence-free coarse field, cast to the tier (the oracle sees the
    stored values)."""
    U, V, W = case.U, case.V, case.W
    if prec == "fp32":
        U, V, W = (a.astype(np.float32).astype(np.float64) for a in (U, V, W))
    return U, V, W


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nc,m,gamma", STAGE_CASES)
def test_stage_refine_parity_periodic(nc, m, gamma, prec):
    print("case stage refine", nc, m, prec, flush=True)
    case = Case(nc, m, gamma, kmax=1, precision=prec, stretch_x=True)
    U, V, W = _fields(case, prec)
    want = O.refine_velocity(case.g, U, V, W)
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    with case.ctx() as ctx:
        got = ctx.interpolate_velocity(case.d(U), case.d(V), case.d(W))
        for a, b in zip(got, want):
            assert rel_max(host(a), b) <= tol
        dv = host(ctx.divergence(*got))
    eps = EPS64 if prec == "fp64" else np.finfo(np.float32).eps
    assert dv[1] < div_bound(m, eps), dv[1] / eps


@pytest.mark.parametrize("nc,m,gamma", STAGE_CASES)
def test_stage_refine_in_time_parity(nc, m, gamma):
    """The time-blended coarse loads of stage z (Eq. 21 read as the linear
    interpolation between two coarse levels) at i = 1 of M_t = 3, and the end
    points i = 0 and i = M_t, which must equal the plain refinement of each
    level bit for bit."""
    print("case stage refine in time", nc, m, flush=True)
    case = Case(nc, m, gamma, kmax=1, stretch_x=True)
    g = case.g
    U1, V1, W1 = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, 1, 0.2, 23)
    lv0 = (case.U, case.V, case.W)
    lv1 = (U1, V1, W1)
    want = O.refine_velocity(g, *blend_velocity(*lv0, *lv1, 1, 3))
    with case.ctx() as ctx:
        d0 = [case.d(a) for a in lv0]
        d1 = [case.d(a) for a in lv1]
        got = ctx.interpolate_velocity_time(*d0, *d1, 1, 3)
        for a, b in zip(got, want):
            assert rel_max(host(a), b) <= FP64_TOL
        dv = host(ctx.divergence(*got))
        assert dv[1] < div_bound(m, EPS64), dv[1] / EPS64
        for i, lv in ((0, d0), (3, d1)):
            end = ctx.interpolate_velocity_time(*d0, *d1, i, 3)
            plain = ctx.interpolate_velocity(*lv)
            for a, b in zip(end, plain):
                assert torch.equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nc,m,gamma", STAGE_CASES)
def test_stage_refine_transpose_parity(nc, m, gamma, prec):
    """The transposed refinement on the same grids against the oracle's
    transpose, and <P x, y> = <x, P^T y> through the library in FP64."""
    print("case stage transpose", nc, m, prec, flush=True)
    case = Case(nc, m, gamma, kmax=1, precision=prec, stretch_x=True)
    g = case.g
    rng = np.random.default_rng(31)
    dense = ((g.z.n, g.y.n, g.x.n), (g.z.n, g.y.n, g.x.n), (g.z.n + 1, g.y.n, g.x.n))
    ys = [rng.standard_normal(s) for s in dense]
    if prec == "fp32":
        ys = [y.astype(np.float32).astype(np.float64) for y in ys]
    want = O.refine_velocity_transpose(g, *ys)
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    with case.ctx() as ctx:
        PTy = [host(t) for t in ctx.interpolate_velocity_backward(*[case.d(y) for y in ys])]
        for a, b in zip(PTy, want):
            assert rel_max(a, b) <= tol
        if prec == "fp64":
            xs = [rng.standard_normal(s) for s in (case.U.shape, case.V.shape, case.W.shape)]
            Px = [host(t) for t in ctx.interpolate_velocity(*[case.d(x) for x in xs])]
            lhs = sum(np.vdot(a, b) for a, b in zip(Px, ys))
            rhs = sum(np.vdot(a, b) for a, b in zip(xs, PTy))
            assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
