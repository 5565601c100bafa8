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


@pytest.mark.parametrize("prec,nc", [("fp64", (700, 3, 4)), ("fp32", (1400, 3, 3)), ("fp64", (40, 7, 5))])
def test_transpose_wide_and_narrow_rows(prec, nc):
    """The transposed refinement's x stage takes a whole dense row per level in
    LDS for rows of up to 1024 columns (here 80); rows of 1400 (FP64) and 2800
    (FP32) columns go through the two-kernel form.  Both against the oracle's
    transpose."""
    print("case transpose rows", prec, nc, flush=True)
    case = Case(nc, (2, 2, 2), 1.5, kmax=1, precision=prec, random_velocity=True, dt=1e-6)
    g = case.g
    rng = np.random.default_rng(32)
    dense = ((g.z.n, g.y.n, g.x.n), (g.z.n, g.y.n, g.x.n), (g.z.n + 1, g.y.n, g.x.n))
    ys = [rng.standard_normal(s) for s in dense]
    if prec == "fp32":
        ys = [y.astype(np.float32).astype(np.float64) for y in ys]
    want = O.refine_velocity_transpose(g, *ys)
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    with case.ctx() as ctx:
        got = [host(t) for t in ctx.interpolate_velocity_backward(*[case.d(y) for y in ys])]
    for a, b in zip(got, want):
        assert rel_max(a, b) <= tol


@pytest.mark.parametrize("side_y,m", [("periodic", (2, 2, 2)), ("walls", (2, 3, 2)), ("periodic", (3, 1, 1)),
                                      ("walls", (1, 2, 3))])
def test_transpose_row_and_layer_ranges(side_y, m):
    """The fused y and z stages of the transposed refinement split the coarse
    rows into ranges of up to 32 and the coarse layers into ranges of up to
    16, each with two halo rows or layers on either side: 70 coarse rows and 40
    coarse layers cross several range boundaries, on periodic and walled y
    (one-sided stencils reach two rows), against the oracle's transpose."""
    print("case transpose ranges", side_y, m, flush=True)
    from paper_1805_03426_amd.context import Context
    nc = (5, 70, 40)
    n = [a * b for a, b in zip(nc, m)]
    xf, yf, zf = inputs.uniform_faces(n[0]), inputs.uniform_faces(n[1]), inputs.tanh_faces(n[2], 1.5)
    walls = side_y == "walls"
    g = O.Grid(xf, yf, zf, m, periodic=(True, not walls, False))
    rng = np.random.default_rng(33)
    ny_faces = n[1] + (1 if walls else 0)   # the oracle keeps the high wall face of a walled axis
    ys = [rng.standard_normal((n[2], n[1], n[0])), rng.standard_normal((n[2], ny_faces, n[0])),
          rng.standard_normal((n[2] + 1, n[1], n[0]))]
    if walls:
        ys[1][:, 0, :] = 0.0
        ys[1][:, -1, :] = 0.0
    want = O.refine_velocity_transpose(g, *ys)
    if walls:
        ys[1] = ys[1][:, :-1, :]   # the library keeps the low wall face only
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    with Context(xf, yf, zf, m, 1e6, 4.38, 1e-5, side_y=side_y) as ctx:
        gU, gV, gW = [host(t) for t in ctx.interpolate_velocity_backward(*[dev(y) for y in ys])]
    assert rel_max(gU, want[0]) <= FP64_TOL
    assert rel_max(gW, want[2]) <= FP64_TOL
    if walls:
        # the low wall face is taken as zero by the forward map: zero gradient
        assert np.all(gV[:, 0] == 0)
        assert rel_max(gV[:, 1:], want[1][:, 1:-1]) <= FP64_TOL
    else:
        assert rel_max(gV, want[1]) <= FP64_TOL
