"""Stopping and resuming a run through the on-disk state: a run that saves
(theta^{n-1}, theta^n, n), ends its context and resumes in a new one computes
the same bits as a run that never stopped, on the line solver and on the
column sweeps, in both precisions (10 steps in two sequences of 5, the
resumed run crossing the start-up and an averaging step)."""
import pytest
import torch

from tests.test_gpu_parity import Case

pytestmark = pytest.mark.gpu


def _run(case, method, seqs, th0, u, v, w, state=None):
    """Step sequences (n0, count) in one context; returns the final levels."""
    from paper_1805_03426_amd.context import Context
    with Context(case.xf, case.yf, case.zf, case.m, case.ra, case.pr, case.dt, n_avg=case.n_avg,
                 precision=case.precision, step_method=method) as ctx:
        prev, cur = state if state is not None else (None, th0)
        for n0, count in seqs:
            ring = [ctx.empty(ctx.shape_cell) for _ in range(3)]
            outs = [ring[q % 3] for q in range(count)]
            ctx.scalar_steps(n0, prev, cur, outs, u, v, w)
            prev, cur = (outs[-2] if count > 1 else cur), outs[-1]
        torch.cuda.synchronize()
        return ctx, prev.clone(), cur.clone()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["line", "sweep"])
def test_resumed_run_is_bit_identical(tmp_path, prec, method):
    print("case checkpoint resume", prec, method, flush=True)
    from paper_1805_03426_amd import checkpoint
    from paper_1805_03426_amd.context import Context
    case = Case((10, 8, 6), (2, 2, 2), 1.5, kmax=2, n_avg=4, precision=prec)
    with Context(case.xf, case.yf, case.zf, case.m, case.ra, case.pr, case.dt, n_avg=case.n_avg,
                 precision=prec) as c0:
        u, v, w = c0.interpolate_velocity(case.d(case.U), case.d(case.V), case.d(case.W))
    th0 = case.d(case.th0)
    _, want_prev, want = _run(case, method, [(0, 5), (5, 5)], th0, u, v, w)
    ctx, p5, c5 = _run(case, method, [(0, 5)], th0, u, v, w)
    path = str(tmp_path / "state.safetensors")
    # the context is closed; save needs only its sizes and parameters
    checkpoint.save(path, ctx, 5, p5, c5)
    del p5, c5
    from paper_1805_03426_amd.context import Context as C2
    with C2(case.xf, case.yf, case.zf, case.m, case.ra, case.pr, case.dt, n_avg=case.n_avg, precision=prec,
            step_method=method) as ctx2:
        n, p, c = checkpoint.load(path, ctx2)
    assert n == 5
    _, got_prev, got = _run(case, method, [(5, 5)], th0, u, v, w, state=(p, c))
    assert torch.equal(got, want) and torch.equal(got_prev, want_prev)
