"""GPU parity of the column-sweep step sequences (mr_scalar_steps, and
mr_scalar_step on columns taller than the line solver's) against the oracle
(Eqs. 5-7 with the z diffusion implicit), through the C ABI.

Each sweep kernel finishes the previous step's implicit solve while it
eliminates its own in the other z direction, so a sequence of count steps
runs count + 1 kernels; a sequence of one step is a sweep and a back
substitution.  The tile shape follows N_x (the first of each precision's
shapes whose width divides it, else the one with the fewest idle lanes: FP64
256 x 4, 192 x 4, 128 x 8, 64 x 16; FP32 128 x 8, 192 x 4, 256 x 4, 64 x 16),
walked in bands of 4 (FP64) and 8 (FP32) x tiles.  Cases cover every shape,
ragged tiles (x and y not multiples of the tile, a single column), several x
tiles and a last band of one tile (x of 1100), one to three z levels, every
step type, both directions of the last back substitution (odd and even
counts), tall columns of 700 and 1024 levels, the coarse step of the temporal
strategy, and the FP32 tier.  Tolerances as for the fused step: 1e-12 (FP64),
1e-5 per step (FP32) with the fluctuation and increment bounds."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.intergrid import coarse_step
from paper_1805_03426_amd import _lib, inputs
from tests.test_gpu_parity import (FP32_FLUCT_TOL, FP32_INCR_TOL, FP32_TOL, FP64_TOL, Case, fp32_fine_errors,
                                   host, rel_l2, rel_max)

pytestmark = pytest.mark.gpu


def _ctx(case, method="sweep"):
    from paper_1805_03426_amd.context import Context
    return Context(case.xf, case.yf, case.zf, case.m, case.ra, case.pr, case.dt, n_avg=case.n_avg,
                   bc_bot=case.bc[0], bc_top=case.bc[1], precision=case.precision, step_method=method)


def _oracle_levels(case, uvw, n0, count, prev, cur):
    out = []
    for q in range(count):
        nxt = O.scalar_step(case.g, case.p, n0 + q, prev, cur, *uvw)
        out.append(nxt)
        prev, cur = cur, nxt
    return out


SIZES = [((5, 3, 7), (3, 1, 2), 1.0),     # x of 15 (one ragged tile), y of 3 (one ragged tile)
         ((33, 5, 4), (2, 2, 2), 1.5),    # x of 66: a second tile of 2 columns; y of 10
         ((1, 1, 1), (1, 1, 1), 0.0),     # a single cell: its own neighbour on every side
         ((4, 9, 2), (2, 1, 1), 0.5),     # two levels, y of 9 (tiles of 8 and 1 rows)
         ((3, 4, 3), (2, 2, 1), 2.0),     # three levels
         ((70, 17, 12), (1, 1, 2), 2.0),  # y of 17: five FP64, three FP32 row tiles; 24 levels
         ((550, 2, 2), (2, 1, 1), 1.0),   # x of 1100: 6 FP64 tiles of 192 (bands of 4 and 2), 9 FP32 of 128 (8 and 1)
         ((96, 3, 3), (2, 2, 1), 1.0),    # x of 192: tiles of 192 x 4 in both precisions
         ((160, 10, 3), (2, 2, 1), 1.0)]  # x of 320: tiles of 64 x 16 in both, y of 20 (16 and 4 rows)


def _dt(nc, m):
    """The explicit x diffusion bound at 320 columns and more on the unit
    width is close to or below the advective step: take a small step there."""
    return 1e-5 if nc[0] * m[0] > 300 else None


@pytest.mark.parametrize("nc,m,gamma", SIZES)
@pytest.mark.parametrize("n0,count", [(0, 1), (0, 2), (0, 5), (3, 4)])
def test_sweep_sequence_parity(nc, m, gamma, n0, count):
    """A sequence of count steps from n0 (start-up at n0 = 0; the averaging
    step at n = 5 with N_p = 3 inside the (3, 4) sequence) against the
    oracle's steps from the same two levels, every output level compared."""
    print("case sweep sequence", nc, m, n0, count, flush=True)
    case = Case(nc, m, gamma, kmax=1, n_avg=3, random_velocity=True, dt=_dt(nc, m))
    uvw = O.refine_velocity(case.g, case.U, case.V, case.W)
    rng = np.random.default_rng(4)
    prev = case.th0 + 0.05 * rng.standard_normal(case.th0.shape) if n0 > 0 else case.th0
    cur = case.th0
    want = _oracle_levels(case, uvw, n0, count, prev, cur)
    with _ctx(case) as ctx:
        du = [case.d(a) for a in uvw]
        # a ring of three buffers (each output differs from the two levels
        # before it); only the last three levels survive
        ring = [ctx.empty(ctx.shape_cell) for _ in range(3)]
        outs = [ring[q % 3] for q in range(count)]
        ctx.scalar_steps(n0, case.d(prev), case.d(cur), outs, *du)
        torch.cuda.synchronize()
        for q in range(max(0, count - 3), count):
            assert rel_max(host(outs[q]), want[q]) <= FP64_TOL, q


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nc,m,gamma", SIZES[:2] + SIZES[-3:])
def test_reverse_sweeps_match_line_reverse_steps(nc, m, gamma, prec):
    """Reverse-step sequences through the column sweeps (mr_scalar_steps_backward)
    against the line solver's reverse steps one at a time, every output:
    the last step of a rollout (no mu^{n0+1}), sequences with mu^{n0+1}
    across the averaging steps (N_p = 3), and a single step down to mu^0.
    FP64 within 1e-12, FP32 within 1e-5 relative L2."""
    print("case reverse sweeps", nc, m, prec, flush=True)
    case = Case(nc, m, gamma, kmax=1, n_avg=3, random_velocity=True, precision=prec, dt=_dt(nc, m))
    uvw = O.refine_velocity(case.g, case.U, case.V, case.W)
    rng = np.random.default_rng(8)
    mus = [rng.standard_normal(case.th0.shape) for _ in range(2)]
    for n0, count, has_next in ((6, 6, False), (5, 4, True), (1, 1, True)):
        want = []
        with _ctx(case, "line") as ctx:
            du = [case.d(a) for a in uvw]
            nxt = case.d(mus[0]) if has_next else None
            cur = case.d(mus[1])
            for q in range(count):
                out = ctx.empty(ctx.shape_cell)
                ctx.scalar_step_backward(n0 - q, nxt, cur, None, out, *du)
                want.append(host(out))
                nxt, cur = cur, out
        with _ctx(case, "sweep") as ctx:
            du = [case.d(a) for a in uvw]
            ring = [ctx.empty(ctx.shape_cell) for _ in range(3)]
            outs = [ring[q % 3] for q in range(count)]
            ctx.scalar_steps_backward(n0, case.d(mus[0]) if has_next else None, case.d(mus[1]), outs, *du)
            torch.cuda.synchronize()
            for q in range(max(0, count - 3), count):
                got = host(outs[q])
                if prec == "fp64":
                    assert rel_max(got, want[q]) <= FP64_TOL, (n0, q)
                else:
                    assert rel_l2(got, want[q]) <= FP32_TOL, (n0, q)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sweep_tiles_bit_identical(prec):
    """Every tile shape gives the same bits: each column's arithmetic does not
    depend on which lanes, rows or workgroups hold its neighbours (x of 200 and
    y of 37 are ragged for every shape; 9 steps from n = 0 through an averaging
    step)."""
    print("case sweep tiles", prec, flush=True)
    case = Case((100, 37, 12), (2, 1, 2), 1.5, kmax=1, n_avg=4, random_velocity=True, precision=prec, dt=1e-5)
    uvw = O.refine_velocity(case.g, case.U, case.V, case.W)
    from paper_1805_03426_amd.context import Context
    results = {}
    for tile in ((1, 2, 3, 4) if prec == "fp64" else (2, 3, 4)):
        with Context(case.xf, case.yf, case.zf, case.m, case.ra, case.pr, case.dt, n_avg=case.n_avg,
                     precision=prec, step_method="sweep", sweep_tile=tile) as ctx:
            du = [case.d(a) for a in uvw]
            ring = [ctx.empty(ctx.shape_cell) for _ in range(3)]
            outs = [ring[q % 3] for q in range(9)]
            ctx.scalar_steps(0, None, case.d(case.th0), outs, *du)
            torch.cuda.synchronize()
            results[tile] = [host(outs[q]) for q in (6, 7, 8)]
    first = results[min(results)]
    for tile, got in results.items():
        for a, b in zip(got, first):
            assert np.array_equal(a, b), tile


@pytest.mark.parametrize("nc,m,gamma", SIZES[:2] + SIZES[-4:])
def test_sweep_single_steps_fp32(nc, m, gamma):
    """FP32 tier through the column sweeps, step by step from the oracle's own
    levels (cast): the per-step bar and the fluctuation and increment bounds."""
    print("case sweep fp32", nc, m, flush=True)
    case = Case(nc, m, gamma, kmax=1, n_avg=3, random_velocity=True, precision="fp32", dt=_dt(nc, m))
    as32 = lambda a: a.astype(np.float32).astype(np.float64)
    uvw = O.refine_velocity(case.g, *(as32(a) for a in (case.U, case.V, case.W)))
    prev = cur = as32(case.th0)
    worst = [0.0, 0.0, 0.0]
    with _ctx(case) as ctx:
        du = [case.d(a) for a in uvw]
        out = ctx.empty(ctx.shape_cell)
        for n in range(6):
            want = O.scalar_step(case.g, case.p, n, prev, cur, *uvw)
            ctx.scalar_steps(n, case.d(prev), case.d(cur), [out], *du)
            got = host(out)
            e = rel_l2(got, want)
            ef, ei = fp32_fine_errors(got, want, cur, cur, case.g.z.c)
            worst = [max(a, b) for a, b in zip(worst, (e, ef, ei))]
            assert e <= FP32_TOL and ef <= FP32_FLUCT_TOL and ei <= FP32_INCR_TOL, (n, e, ef, ei)
            prev, cur = cur, as32(want)
    print("fp32 sweep step errors: theta %.2e, fluctuation %.2e, increment %.2e" % tuple(worst), flush=True)


def test_sweep_sequence_fp32_matches_line_solver_to_rounding():
    """A ten-step FP32 sequence through the column sweeps and through the line
    solver, both against the oracle's FP64 run: each within 1e-5 relative L2."""
    print("case sweep fp32 sequence", flush=True)
    case = Case((33, 12, 10), (2, 2, 2), 1.5, kmax=2, n_avg=4, precision="fp32")
    as32 = lambda a: a.astype(np.float32).astype(np.float64)
    uvw = O.refine_velocity(case.g, *(as32(a) for a in (case.U, case.V, case.W)))
    th0 = as32(case.th0)
    want = _oracle_levels(case, uvw, 0, 10, th0, th0)[-1]
    for method in ("sweep", "line"):
        with _ctx(case, method) as ctx:
            du = [case.d(a) for a in uvw]
            ring = [ctx.empty(ctx.shape_cell) for _ in range(3)]
            outs = [ring[q % 3] for q in range(10)]
            ctx.scalar_steps(0, None, case.d(th0), outs, *du)
            e = rel_l2(host(outs[-1]), want)
            print("fp32 10-step sequence (%s): %.2e" % (method, e), flush=True)
            assert e <= FP32_TOL


@pytest.mark.parametrize("nz,gamma", [(700, 2.0), (1024, 2.5)])
def test_tall_columns_fp64(nz, gamma):
    """Columns beyond the line solver's 640 levels (1024: the paper's dense
    mesh height, Sec. 4.4) on a small x-y footprint: single steps and a
    sequence, FP64, against the oracle; a reverse step with a direct loss
    gradient (lam_add) has no sweep form and is refused."""
    print("case tall columns", nz, flush=True)
    case = Case((3, 5, nz // 2), (3, 1, 2), gamma, kmax=1, n_avg=3, random_velocity=True, dt=2e-4)
    uvw = O.refine_velocity(case.g, case.U, case.V, case.W)
    want = _oracle_levels(case, uvw, 0, 4, case.th0, case.th0)
    with _ctx(case, "auto") as ctx:
        du = ctx.interpolate_velocity(case.d(case.U), case.d(case.V), case.d(case.W))
        for a, b in zip(du, uvw):
            assert rel_max(host(a), b) <= FP64_TOL
        out = ctx.empty(ctx.shape_cell)
        ctx.scalar_step(0, None, case.d(case.th0), out, *du)
        assert rel_max(host(out), want[0]) <= FP64_TOL
        ctx.scalar_step(2, case.d(want[0]), case.d(want[1]), out, *du)
        assert rel_max(host(out), want[2]) <= FP64_TOL
        ring = [ctx.empty(ctx.shape_cell) for _ in range(3)]
        outs = [ring[q % 3] for q in range(4)]
        ctx.scalar_steps(0, None, case.d(case.th0), outs, *du)
        assert rel_max(host(outs[3]), want[3]) <= FP64_TOL
        with pytest.raises(_lib.MRError) as e:
            ctx.scalar_step_backward(3, ring[1], ring[2], out, ring[0], *du)   # lam_add = out, into ring[0]
        assert e.value.status == _lib.MR_ESHAPE


@pytest.mark.parametrize("nz,ckpt", [(700, 2), (1024, 3)])
def test_tall_columns_adjoint_fp64(nz, ckpt):
    """The checkpointed rollout's gradients on columns beyond the line solver
    (the seed solve, the reverse steps and the start-up step's reverse as
    column sweeps) against the oracle's discrete adjoint (FP64, 5 steps)."""
    print("case tall columns adjoint", nz, flush=True)
    from paper_1805_03426_amd.autograd import rollout
    case = Case((3, 5, nz // 2), (3, 1, 2), 2.0, kmax=1, n_avg=3, ra=1e4, dt=2e-4)
    target = inputs.theta_initial(case.zf, case.g.x.n, case.g.y.n, seed=3)
    _, w0, wU, wV, wW = O.rollout_loss_grad(case.g, case.p, case.th0, case.U, case.V, case.W, 5, target)
    with _ctx(case, "auto") as ctx:
        assert ctx.step_method == "sweep"
        th = case.d(case.th0).requires_grad_(True)
        U, V, W = (case.d(a).requires_grad_(True) for a in (case.U, case.V, case.W))
        out = rollout(ctx, th, U, V, W, 5, ckpt)
        torch.autograd.backward(out, out.detach() - case.d(target))
        got = [host(t.grad) for t in (th, U, V, W)]
    for a, b in zip(got, (w0, wU, wV, wW)):
        assert rel_max(a, b) <= 1e-11


def test_coarse_step_through_sweeps():
    """The temporal strategy's coarse step (M_t = 3 sub-steps on the velocity
    refined in time, then the integration) through the column sweeps, against
    the oracle's coarse step, twice in a row (FP64)."""
    print("case coarse step sweeps", flush=True)
    case = Case((9, 7, 5), (2, 2, 2), 1.5, kmax=1, n_avg=4)
    g = case.g
    U1, V1, W1 = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, 1, 0.2, 22)
    lv0, lv1 = (case.U, case.V, case.W), (U1, V1, W1)
    p0, c0 = case.th0, case.th0
    wants = []
    for n0 in (0, 3):
        p0, c0, tc = coarse_step(g, case.p, n0, 3, p0, c0, *lv0, *lv1)
        wants.append((p0, c0, tc))
    with _ctx(case) as ctx:
        d0, d1 = [case.d(a) for a in lv0], [case.d(a) for a in lv1]
        uvw = (ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_w))
        ring = [case.d(case.th0), ctx.empty(ctx.shape_cell), ctx.empty(ctx.shape_cell)]
        tcd = ctx.empty(ctx.shape_coarse)
        p, c = 0, 0
        for (wp, wc, wt), n0 in zip(wants, (0, 3)):
            p, c = ctx.coarse_step(n0, 3, *d0, *d1, uvw, ring, p, c, tcd)
            assert rel_max(host(ring[c]), wc) <= FP64_TOL
            assert rel_max(host(ring[p]), wp) <= FP64_TOL
            assert rel_max(host(tcd), wt) <= FP64_TOL
