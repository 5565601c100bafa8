"""The windowed oracle used for large-grid sampled parity equals the
full-field oracle at the sampled columns (CPU)."""
import numpy as np

import oracle as O
from paper_1805_03426_amd import inputs
from paper_1805_03426_amd.configs import WORKLOADS
from tests import sampling as S


def test_windowed_oracle_matches_full_field():
    w = WORKLOADS["rb64-m2-fp64"]
    d = inputs.workload_inputs(w)
    nx, ny, nz = w.n
    mx, my, mz = w.m
    g = O.Grid(d["xf"], d["yf"], d["zf"], w.m)
    p = O.ScalarParams.from_ra_pr(w.ra, w.pr, d["dt"], n_avg=3)
    uvw = O.refine_velocity(g, d["U"], d["V"], d["W"])
    th0 = d["theta0"]
    th1 = inputs.theta_initial(d["zf"], nx, ny, seed=9)
    full = {n: O.scalar_step(g, p, n, th0, th1, *uvw) for n in (0, 1, 2)}
    for (i, j) in S.sample_columns(nx, ny, mx, my, 6, seed=5):
        win, origin = S.refine_window(d["U"], d["V"], d["W"], w.m, d["zf"], nx, ny, i // mx, j // my)
        for a, b in zip(S.dense_column(win, origin, i, j), (uvw[0][:, j, i], uvw[1][:, j, i], uvw[2][:, j, i])):
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(b).max())
        for n in (0, 1, 2):
            col = S.step_column(th0, th1, win, origin, d["zf"], nx, ny, w.m, p, n, i, j)
            np.testing.assert_allclose(col, full[n][:, j, i], rtol=1e-13, atol=1e-14)
