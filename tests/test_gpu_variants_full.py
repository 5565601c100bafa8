"""The variants of the step at the full 128^3 -> 256^3 workload, in the launch
configuration the benchmark times them in: the whole field against the oracle
for the start-up, a leapfrog and an averaging step (side walls also through
the refinement)."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_1805_03426_amd import inputs
from paper_1805_03426_amd.configs import WORKLOADS
from tests.test_gpu_parity import FP64_TOL, dev, host, rel_l2, rel_max

pytestmark = pytest.mark.gpu


def _three_steps(ctx, g, p, d, uvw_oracle, uvw_dev):
    """Steps 0, 1 and 49 (the averaging step) from the oracle's own levels."""
    th0 = d["theta0"]
    out = ctx.empty(ctx.shape_cell)
    t1 = O.scalar_step(g, p, 0, th0, th0, *uvw_oracle)
    ctx.scalar_step(0, dev(th0), dev(th0), out, *uvw_dev)
    assert rel_l2(host(out), t1) <= FP64_TOL
    assert rel_max(host(out), t1) <= FP64_TOL
    t2 = O.scalar_step(g, p, 1, th0, t1, *uvw_oracle)
    ctx.scalar_step(1, dev(th0), dev(t1), out, *uvw_dev)
    assert rel_l2(host(out), t2) <= FP64_TOL
    t50 = O.scalar_step(g, p, 49, t1, t2, *uvw_oracle)
    ctx.scalar_step(49, dev(t1), dev(t2), out, *uvw_dev)
    assert rel_l2(host(out), t50) <= FP64_TOL


@pytest.mark.parametrize("variant", [dict(z_explicit=0.5), dict(face_order=4)])
def test_rb256_variant_steps(variant):
    print("case rb256 full size", variant, flush=True)
    from paper_1805_03426_amd.context import Context
    w = WORKLOADS["rb256-m2-fp64"]
    d = inputs.workload_inputs(w)
    g = O.Grid(d["xf"], d["yf"], d["zf"], w.m)
    p = dataclasses.replace(O.ScalarParams.from_ra_pr(w.ra, w.pr, d["dt"], n_avg=w.n_avg), **variant)
    uvw = O.refine_velocity(g, d["U"], d["V"], d["W"])
    with Context(d["xf"], d["yf"], d["zf"], w.m, w.ra, w.pr, d["dt"], n_avg=w.n_avg, **variant) as ctx:
        du = ctx.interpolate_velocity(dev(d["U"]), dev(d["V"]), dev(d["W"]))
        _three_steps(ctx, g, p, d, uvw, du)


def test_rb256_side_walls():
    """Adiabatic no-slip walls in x and y: the generator's coarse velocity with
    its low wall faces zeroed (the library's layout keeps n faces; the oracle's
    adds the zero high wall face).  Zeroing the wall faces of a periodic field
    leaves the coarse cells at the walls with a net flux, so the refined field
    is not divergence-free there; the step is defined for any face velocity."""
    print("case rb256 full size, side walls", flush=True)
    from paper_1805_03426_amd.context import Context
    w = WORKLOADS["rb256-m2-fp64"]
    d = inputs.workload_inputs(w)
    U, V = d["U"].copy(), d["V"].copy()
    U[:, :, 0] = 0.0
    V[:, 0, :] = 0.0
    Uo = np.concatenate([U, np.zeros(U.shape[:2] + (1,))], axis=2)
    Vo = np.concatenate([V, np.zeros((V.shape[0], 1, V.shape[2]))], axis=1)
    g = O.Grid(d["xf"], d["yf"], d["zf"], w.m, periodic=(False, False, False))
    p = O.ScalarParams.from_ra_pr(w.ra, w.pr, d["dt"], n_avg=w.n_avg)
    u, v, ww = O.refine_velocity(g, Uo, Vo, d["W"])
    with Context(d["xf"], d["yf"], d["zf"], w.m, w.ra, w.pr, d["dt"], n_avg=w.n_avg, side_x="walls",
                 side_y="walls") as ctx:
        du = ctx.interpolate_velocity(dev(U), dev(V), dev(d["W"]))
        gu, gv, gw = (host(t) for t in du)
        assert rel_max(gu, u[:, :, :-1]) <= FP64_TOL
        assert rel_max(gv, v[:, :-1]) <= FP64_TOL
        assert rel_max(gw, ww) <= FP64_TOL
        assert np.all(gu[:, :, 0] == 0) and np.all(gv[:, 0] == 0)
        _three_steps(ctx, g, p, d, (u, v, ww), du)


def test_rb256_fp32_steps():
    """The FP32 tier at the full 256^3 size in the launch configuration the
    benchmark times (8 chunks of 32 levels, one-row patches, two levels of
    prefetch): refinement and the start-up, leapfrog and averaging steps on
    the whole field against the FP64 oracle, within the FP32 per-step bar."""
    print("case rb256 full size fp32", flush=True)
    import torch
    from paper_1805_03426_amd.context import Context
    from tests.test_gpu_parity import FP32_FLUCT_TOL, FP32_INCR_TOL, FP32_TOL, fp32_fine_errors
    w = WORKLOADS["rb256-m2-fp64"]
    d = inputs.workload_inputs(w)
    g = O.Grid(d["xf"], d["yf"], d["zf"], w.m)
    p = O.ScalarParams.from_ra_pr(w.ra, w.pr, d["dt"], n_avg=w.n_avg)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float32)
    as32 = lambda a: a.astype(np.float32).astype(np.float64)     # the values the GPU holds
    uvw = O.refine_velocity(g, as32(d["U"]), as32(d["V"]), as32(d["W"]))
    th0 = as32(d["theta0"])
    with Context(d["xf"], d["yf"], d["zf"], w.m, w.ra, w.pr, d["dt"], n_avg=w.n_avg, precision="fp32") as ctx:
        du = ctx.interpolate_velocity(f32(d["U"]), f32(d["V"]), f32(d["W"]))
        for a, b in zip(du, uvw):
            assert rel_l2(host(a), b) <= FP32_TOL
        out = ctx.empty(ctx.shape_cell)
        zc = g.z.c

        def check(got, want, cur):
            assert rel_l2(got, want) <= FP32_TOL
            ef, ei = fp32_fine_errors(got, want, cur, cur, zc)
            print("fp32 rb256 step: fluctuation %.2e, increment %.2e" % (ef, ei), flush=True)
            assert ef <= FP32_FLUCT_TOL and ei <= FP32_INCR_TOL

        t1 = O.scalar_step(g, p, 0, th0, th0, *uvw)
        ctx.scalar_step(0, f32(th0), f32(th0), out, *du)
        check(host(out), t1, th0)
        t1 = as32(t1)
        t2 = O.scalar_step(g, p, 1, th0, t1, *uvw)
        ctx.scalar_step(1, f32(th0), f32(t1), out, *du)
        check(host(out), t2, t1)
        t50 = O.scalar_step(g, p, 49, th0, t1, *uvw)
        ctx.scalar_step(49, f32(th0), f32(t1), out, *du)
        check(host(out), t50, t1)
