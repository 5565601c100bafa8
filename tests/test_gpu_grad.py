"""GPU parity of the velocity gradient of a range of steps
(mr_velocity_grad) against the oracle's transpose of the advective term with
respect to the dense face velocities (Eqs. 5-7: the central face values times
the difference of the adjoint across the face), summed over the steps with
each step's weight tau, through the C ABI.

The kernel walks tiles of 64 columns by 16 rows and z segments of 8 (FP32)
or 4 (FP64) levels: the cases cover several x and y tiles with ragged ends,
ragged last segments, a single tile row, every step kind, periodic and walled
sides (non-uniform y), and the accumulation into existing gradients.
Tolerances: element-wise relative max 1e-12 (FP64), 1e-5 (FP32, the oracle
sees the FP32-rounded inputs)."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.scalar import _advection_velocity_transpose
from paper_1805_03426_amd import inputs
from tests.test_gpu_parity import FP64_TOL, host, rel_max
from tests.test_gpu_walls import WallCase, oracle_to_lib

pytestmark = pytest.mark.gpu

CASES = [((70, 35, 13), (False, False)), ((70, 35, 13), (True, True)), ((20, 17, 9), (True, False)),
         ((3, 5, 21), (False, True))]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,walls", CASES)
def test_velocity_grad_parity(n, walls, prec):
    print("case velocity gradient", n, walls, prec, flush=True)
    c = WallCase(n, (1, 1, 1), walls, precision=prec, n_avg=3)
    rng = np.random.default_rng(12)
    steps = list(range(10))          # start-up, leapfrog and averaging (n = 2, 5, 8) steps
    cast = (lambda a: a.astype(np.float32).astype(np.float64)) if prec == "fp32" else (lambda a: a)
    ths = [cast(inputs.theta_initial(c.zf, c.g.x.n, c.g.y.n, noise=0.2, seed=20 + s)) for s in steps]
    mus = [cast(rng.standard_normal(ths[0].shape)) for _ in steps]
    want = [0.0, 0.0, 0.0]
    for s, th, mu in zip(steps, ths, mus):
        tau = O.step_kind(s, c.n_avg, c.dt)[0]
        for q, gq in enumerate(_advection_velocity_transpose(c.g, mu, th, 2)):
            want[q] = want[q] + tau * gq
    gu_o, gv_o, gw_o = want
    if walls[0]:
        gu_o = oracle_to_lib(gu_o, 2)
    if walls[1]:
        gv_o = oracle_to_lib(gv_o, 1)
    start = [cast(rng.standard_normal(a.shape)) for a in (gu_o, gv_o, gw_o)]
    with c.ctx() as ctx:
        g = [c.d(a) for a in start]
        ctx.velocity_grad(steps, [c.d(t) for t in ths], [c.d(m) for m in mus], *g)
        torch.cuda.synchronize()
        got = [host(a) - b for a, b in zip(g, start)]
    tol = FP64_TOL if prec == "fp64" else 1e-5
    for a, b in zip(got, (gu_o, gv_o, gw_o)):
        assert rel_max(a, b) <= tol, rel_max(a, b)
    if walls[0]:
        assert np.abs(got[0][:, :, 0]).max() <= 1e-14 * np.abs(gu_o).max()
    if walls[1]:
        assert np.abs(got[1][:, 0, :]).max() <= 1e-14 * np.abs(gv_o).max()
