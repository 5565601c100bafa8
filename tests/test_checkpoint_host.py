"""On-disk run state (paper_1805_03426_amd/checkpoint.py) on the CPU: a save
and load round trip is exact, and a state written for another grid,
precision or time step is refused."""
import types

import pytest
import torch

from paper_1805_03426_amd import checkpoint


def _ctx(nz=3, ny=4, nx=5, precision="fp64", dt=1e-3):
    dtype = torch.float64 if precision == "fp64" else torch.float32
    desc = types.SimpleNamespace(dt=dt, ra=1e6, pr=4.38, n_avg=50)
    return types.SimpleNamespace(nx=nx, ny=ny, nz=nz, precision=precision, dtype=dtype, shape_cell=(nz, ny, nx),
                                 desc=desc, device=torch.device("cpu"))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_round_trip_is_exact(tmp_path, precision):
    ctx = _ctx(precision=precision)
    g = torch.Generator().manual_seed(3)
    a = torch.randn(ctx.shape_cell, generator=g, dtype=ctx.dtype)
    b = torch.randn(ctx.shape_cell, generator=g, dtype=ctx.dtype)
    path = str(tmp_path / "state.safetensors")
    checkpoint.save(path, ctx, 17, a, b)
    n, pa, pb = checkpoint.load(path, ctx)
    assert n == 17 and torch.equal(pa, a) and torch.equal(pb, b) and pa.dtype == ctx.dtype


def test_start_state_needs_no_previous_level(tmp_path):
    ctx = _ctx()
    b = torch.ones(ctx.shape_cell, dtype=ctx.dtype)
    path = str(tmp_path / "s0.safetensors")
    checkpoint.save(path, ctx, 0, None, b)
    n, pa, pb = checkpoint.load(path, ctx)
    assert n == 0 and torch.equal(pb, b)
    with pytest.raises(ValueError):
        checkpoint.save(path, ctx, 4, None, b)


@pytest.mark.parametrize("other", [dict(dt=2e-3), dict(precision="fp32"), dict(nx=6)])
def test_state_for_another_run_is_refused(tmp_path, other):
    ctx = _ctx()
    t = torch.zeros(ctx.shape_cell, dtype=ctx.dtype)
    path = str(tmp_path / "s.safetensors")
    checkpoint.save(path, ctx, 5, t, t)
    with pytest.raises(ValueError):
        checkpoint.load(path, _ctx(**other))


def test_wrong_shape_or_dtype_refused(tmp_path):
    ctx = _ctx()
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "x"), ctx, 1, torch.zeros(2, 2, dtype=torch.float64),
                        torch.zeros(ctx.shape_cell, dtype=torch.float64))
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "x"), ctx, 1, torch.zeros(ctx.shape_cell, dtype=torch.float32),
                        torch.zeros(ctx.shape_cell, dtype=torch.float32))
