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


def test_reverse_step_chain_is_the_discrete_adjoint():
    """Seeding with Z^-T (theta_N - target) and chaining the reverse step from
    n = N-1 down to 0 gives the oracle rollout's dL/dtheta^0, and the summed
    velocity gradients, refined back, its coarse gradients (every step type)."""
    g = O.Grid(inputs.uniform_faces(10), inputs.uniform_faces(10), inputs.tanh_faces(7, 1.5), (2, 2, 1))
    U, V, W = inputs.divergence_free_velocity(g.x.cf, g.y.cf, g.z.cf, kmax=2, seed=1)
    th0 = inputs.theta_initial(g.z.faces, g.x.n, g.y.n, noise=0.1, seed=2)
    tgt = inputs.theta_initial(g.z.faces, g.x.n, g.y.n, noise=0.1, seed=3)
    p = O.ScalarParams.from_ra_pr(1e4, 4.38, dt=0.02, n_avg=3)
    N = 7
    _, w0, wU, wV, wW = O.rollout_loss_grad(g, p, th0, U, V, W, N, tgt)
    u, v, w = O.refine_velocity(g, U, V, W)
    th = O.rollout(g, p, th0, u, v, w, N, keep=True)
    mu = {N - 1: S.seed(g, p, N - 1, th[N] - tgt)}
    gsum = [np.zeros_like(a) for a in (u, v, w)]
    for n in range(N - 1, -1, -1):
        out, grads = S.reverse_step(g, p, n, mu.get(n + 1), mu[n], th[n], u, v, w)
        for acc, d in zip(gsum, grads):
            acc += d
        if n >= 1:
            mu[n - 1] = out
    np.testing.assert_allclose(out, w0, rtol=0, atol=1e-12 * np.abs(w0).max())
    for a, b in zip(O.refine_velocity_transpose(g, *gsum), (wU, wV, wW)):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(b).max())


def test_windowed_reverse_step_matches_full_field():
    """backward_column on 3x3 windows equals the whole-field reverse step at
    sampled columns, the periodic seam included, for every step type."""
    w = WORKLOADS["rb64-m2-fp64"]
    d = inputs.workload_inputs(w)
    nx, ny, nz = w.n
    mx, my, mz = w.m
    g = O.Grid(d["xf"], d["yf"], d["zf"], w.m)
    p = O.ScalarParams.from_ra_pr(w.ra, w.pr, d["dt"], n_avg=3)
    uvw = O.refine_velocity(g, d["U"], d["V"], d["W"])
    rng = np.random.default_rng(7)
    mu_a, mu_b, th = (rng.standard_normal((nz, ny, nx)) for _ in range(3))
    cols = S.sample_columns(nx, ny, mx, my, 6, seed=5)
    for n, nxt in ((0, mu_a), (1, mu_a), (2, mu_a), (5, None)):
        full, fgrads = S.reverse_step(g, p, n, nxt, mu_b, th, *uvw)
        for (i, j) in cols:
            win, origin = S.refine_window(d["U"], d["V"], d["W"], w.m, d["zf"], nx, ny, i // mx, j // my)
            xs, ys = np.arange(i - 1, i + 2) % nx, np.arange(j - 1, j + 2) % ny
            cut = lambda a: None if a is None else a[:, ys][:, :, xs]
            col, cgrads = S.backward_column(cut(nxt), cut(mu_b), cut(th), win, origin, d["zf"], nx, ny, p, n, i, j)
            np.testing.assert_allclose(col, full[:, j, i], rtol=0, atol=1e-13 * np.abs(full).max())
            for a, b in zip(cgrads, fgrads):
                np.testing.assert_allclose(a, b[:, j, i], rtol=0, atol=1e-13 * np.abs(b).max())
