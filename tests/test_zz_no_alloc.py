"""The allocation-free Nusselt entry point (mr_nusselt_noalloc) through the C
ABI: the same profile and summary as mr_nusselt (Eq. 22), bit for bit, on two
calls in a row, the second on a smaller grid (fewer faces and horizontal
parts, so it reads fewer partials than the first call left behind), in both
precisions; and MR_ESHAPE beyond its 1024-face limit."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_03426_amd import _lib
from tests.test_gpu_parity import Case, host

pytestmark = pytest.mark.gpu


def _noalloc(ctx, theta, w, prof):
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return _lib.lib().mr_nusselt_noalloc(ctx._ctx, ctypes.c_void_p(theta.data_ptr()),
                                         ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(prof.data_ptr()), s)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nusselt_noalloc_matches_nusselt(prec):
    print("case nusselt noalloc", prec, flush=True)
    rng = np.random.default_rng(17)
    for nc, m in (((48, 40, 24), (2, 2, 3)), ((10, 6, 8), (2, 2, 2))):   # the second call is smaller
        case = Case(nc, m, 1.5, kmax=1, precision=prec, random_velocity=True, dt=1e-4)
        th = case.th0 + 0.05 * rng.standard_normal(case.th0.shape)
        w = 0.2 * rng.standard_normal((case.g.z.n + 1,) + case.g.shape[1:])
        w[0] = w[-1] = 0.0
        if prec == "fp32":
            th = th.astype(np.float32).astype(np.float64)
            w = w.astype(np.float32).astype(np.float64)
        want, summ = O.nusselt(case.g, case.p, th, w)
        with case.ctx() as ctx:
            dth, dw = case.d(th), case.d(w)
            ref, _ = ctx.nusselt(dth, dw, sync=False)
            got = torch.full_like(ref, float("nan"))
            assert _noalloc(ctx, dth, dw, got) == _lib.MR_OK
            torch.cuda.synchronize()
            assert torch.equal(got, ref)
            g = host(got)
            assert np.abs(g[:-5] - want).max() <= 1e-12 * np.abs(want).max()
            for k, key in enumerate(["nu_bot", "nu_top", "nu_vol", "nu_paper", "mean_theta"]):
                assert abs(g[-5 + k] - summ[key]) <= 1e-12 * max(1.0, abs(summ[key])), key


def test_nusselt_noalloc_rejects_more_than_1024_faces():
    print("case nusselt noalloc limit", flush=True)
    case = Case((3, 3, 550), (2, 2, 2), 2.0, kmax=1, random_velocity=True, dt=1e-5)   # 1100 levels
    with case.ctx() as ctx:
        th = ctx.empty(ctx.shape_cell)
        w = ctx.empty(ctx.shape_w)
        prof = torch.empty(ctx.nz + 6, dtype=torch.float64, device="cuda")
        assert _noalloc(ctx, th, w, prof) == _lib.MR_ESHAPE
