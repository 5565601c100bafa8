"""The refinement and its transpose over a matrix of refinement factors and
side conditions, against the oracle (FP64, element-wise), with the time-blended
form and an adjoint check: every factor from 1 to 5 on each axis (M_z up to 4
in the fused kernel, 5 through the three stage kernels), periodic or walled x
and y, coarse sizes that leave ragged tiles."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.intergrid import blend_velocity
from tests.test_gpu_parity import FP64_TOL, host, rel_max
from tests.test_gpu_walls import WallCase

pytestmark = pytest.mark.gpu

FACTORS = [(1, 1, 1), (2, 1, 1), (1, 2, 3), (3, 3, 3), (2, 2, 4), (4, 1, 2), (1, 3, 5), (5, 2, 1)]
SIDES = [(False, False), (True, False), (False, True), (True, True)]


@pytest.mark.parametrize("walls", SIDES)
@pytest.mark.parametrize("m", FACTORS)
def test_refine_matrix(m, walls):
    print("case refine matrix", m, walls, flush=True)
    c = WallCase((7, 5, 4), m, walls, dt=1e-4)
    U, V, W = c.coarse_velocity()
    U1, V1, W1 = c.coarse_velocity(scale=0.3)
    Ul, Vl = c.to_lib(U, V)
    U1l, V1l = c.to_lib(U1, V1)
    rng = np.random.default_rng(11)
    with c.ctx() as ctx:
        got = [host(t) for t in ctx.interpolate_velocity(c.d(Ul), c.d(Vl), c.d(W))]
        gu, gv = c.to_oracle(got[0], got[1])
        want = O.refine_velocity(c.g, U, V, W)
        for a, b in zip((gu, gv, got[2]), want):
            assert rel_max(a, b) <= FP64_TOL
        # the random coarse field is not divergence-free: the check's largest
        # |net flux| and |net flux| / sum |flux| against the oracle's
        dv = host(ctx.divergence(*(c.d(x) for x in got)))
        div, tot = O.refine.divergence(c.g, *want)
        rel = np.abs(div)[tot > 0] / tot[tot > 0]
        assert abs(dv[0] - np.abs(div).max()) <= 1e-12 * np.abs(div).max()
        assert abs(dv[1] - rel.max()) <= 1e-12 * rel.max()
        # the time-blended coarse loads, at a fraction inside the coarse step
        i, mt = 2, 3
        got_t = [host(t) for t in ctx.interpolate_velocity_time(c.d(Ul), c.d(Vl), c.d(W), c.d(U1l), c.d(V1l),
                                                                 c.d(W1), i, mt)]
        gu, gv = c.to_oracle(got_t[0], got_t[1])
        want_t = O.refine_velocity(c.g, *blend_velocity(U, V, W, U1, V1, W1, i, mt))
        for a, b in zip((gu, gv, got_t[2]), want_t):
            assert rel_max(a, b) <= FP64_TOL
        # transposed refinement: against the oracle's transpose, and <P x, y> = <x, P^T y>
        yu, yv, yw = (rng.standard_normal(t.shape) for t in got)
        if walls[0]:
            yu[:, :, 0] = 0.0
        if walls[1]:
            yv[:, 0] = 0.0
        gU, gV, gW = (host(t) for t in ctx.interpolate_velocity_backward(c.d(yu), c.d(yv), c.d(yw)))
    yuo, yvo = c.to_oracle(yu, yv)
    wU, wV, wW = O.refine_velocity_transpose(c.g, yuo, yvo, yw)
    # a walled axis: the wall faces are not inputs of the refinement
    assert (rel_max(gU[:, :, 1:], wU[:, :, 1:-1]) if walls[0] else rel_max(gU, wU)) <= FP64_TOL
    assert (rel_max(gV[:, 1:], wV[:, 1:-1]) if walls[1] else rel_max(gV, wV)) <= FP64_TOL
    assert rel_max(gW, wW) <= FP64_TOL
    lhs = sum(float(np.sum(a * b)) for a, b in zip(got, (yu, yv, yw)))
    rhs = sum(float(np.sum(a * b)) for a, b in zip((Ul, Vl, W), (gU, gV, gW)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
