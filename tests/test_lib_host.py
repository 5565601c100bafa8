"""CPU tests of the C-ABI library: it loads, exports every symbol the header
declares, builds the same grid tables as the oracle on the host, and rejects
bad descriptors before touching a GPU.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1805_03426_amd import _lib, inputs
from paper_1805_03426_amd.context import (host_face_weights, host_refinement_table, host_z_face_weights,
                                           host_z_system, make_desc)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrscalar.h")


def test_library_exports_every_declared_symbol():
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(mr_[a-z_0-9]+)\s*\(", text))
    assert declared, "no declarations parsed"
    L = _lib.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(_lib.EXPORTS)


def test_status_strings():
    assert _lib.status_string(0) == "ok"
    assert "invalid" in _lib.status_string(-1)


def _desc(nc=(6, 5, 7), m=(2, 3, 2), gamma=1.5, **kw):
    xf = inputs.uniform_faces(nc[0] * m[0])
    yf = inputs.uniform_faces(nc[1] * m[1])
    zf = inputs.tanh_faces(nc[2] * m[2], gamma)
    args = dict(ra=1e6, pr=4.38, dt=1e-3)
    args.update(kw)
    return make_desc(xf, yf, zf, m, **args), (xf, yf, zf)


@pytest.mark.parametrize("m", [(2, 2, 2), (3, 2, 4), (1, 3, 1)])
def test_host_refinement_tables_match_oracle(m):
    (d, keep), (xf, yf, zf) = _desc(m=m, gamma=2.0)
    g = O.Grid(xf, yf, zf, m)
    for axis, ax in enumerate((g.x, g.y, g.z)):
        R, s = host_refinement_table(d, axis)
        for I in range(ax.nc):
            np.testing.assert_allclose(R[I], O.r_matrix(ax, I), rtol=0, atol=1e-14)
            if ax.m > 1:
                assert s[I] == O.stencil_start(ax, I)


@pytest.mark.parametrize("m", [(2, 3, 2), (3, 2, 2)])
def test_host_refinement_tables_with_side_walls(m):
    """Walled x and y: one-sided stencils at the first and last coarse cells."""
    nc = (5, 4, 4)
    xf, yf, zf = (inputs.uniform_faces(c * q) for c, q in zip(nc, m))
    zf = inputs.tanh_faces(nc[2] * m[2], 1.5)
    d, keep = make_desc(xf, yf, zf, m, ra=1e4, pr=1.0, dt=1e-5, side_x="walls", side_y="walls")
    g = O.Grid(xf, yf, zf, m, periodic=(False, False, False))
    for axis, ax in enumerate((g.x, g.y)):
        R, s = host_refinement_table(d, axis)
        for I in range(ax.nc):
            np.testing.assert_allclose(R[I], O.r_matrix(ax, I), rtol=0, atol=1e-14)
            assert s[I] == O.stencil_start(ax, I)
    assert host_refinement_table(d, 0)[1][0] == 0 and host_refinement_table(d, 0)[1][-1] == nc[0] - 3


def test_host_refinement_stretched_x():
    rng = np.random.default_rng(3)
    hx = rng.uniform(0.5, 2.0, 12)
    xf = np.concatenate([[0], np.cumsum(hx)]) / hx.sum()
    yf = inputs.uniform_faces(8)
    zf = inputs.tanh_faces(12, 1.0)
    d, keep = make_desc(xf, yf, zf, (3, 2, 2), ra=1e4, pr=1.0, dt=1e-4)
    g = O.Grid(xf, yf, zf, (3, 2, 2))
    R, _ = host_refinement_table(d, 0)
    for I in range(4):
        np.testing.assert_allclose(R[I], O.r_matrix(g.x, I), atol=1e-14)


@pytest.mark.parametrize("bc", [("dirichlet", "dirichlet"), ("adiabatic", "dirichlet"),
                                ("dirichlet", "adiabatic")])
def test_host_z_system_matches_oracle(bc):
    (d, keep), (xf, yf, zf) = _desc(gamma=2.5, n_avg=4, bc_bot=bc[0], bc_top=bc[1], t_bot=0.8, t_top=0.1)
    g = O.Grid(xf, yf, zf, (2, 3, 2))
    p = O.ScalarParams.from_ra_pr(1e6, 4.38, dt=1e-3, n_avg=4, bc_bot=bc[0], bc_top=bc[1], t_bot=0.8,
                                  t_top=0.1)
    for n in (0, 1, 3, 7):
        sub, diag, sup, bz, tau = host_z_system(d, n)
        want_tau = O.step_kind(n, 4, 1e-3)[0]
        assert tau == want_tau
        osub, odiag, osup, obz = O.z_matrix(g, tau * p.kappa, p)
        np.testing.assert_allclose(sub, osub, rtol=1e-14, atol=0)
        np.testing.assert_allclose(diag, odiag, rtol=1e-14, atol=0)
        np.testing.assert_allclose(sup, osup, rtol=1e-14, atol=0)
        np.testing.assert_allclose(bz, obz, rtol=1e-14, atol=0)


@pytest.mark.parametrize("wz", [0.5, 0.3])
def test_host_z_system_with_explicit_share(wz):
    """The solved system keeps the implicit share (1 - w) of the z diffusion;
    the wall source b_z is unchanged."""
    (d, keep), (xf, yf, zf) = _desc(gamma=2.5, n_avg=4, t_bot=0.8, t_top=0.1)
    d.z_explicit = wz
    g = O.Grid(xf, yf, zf, (2, 3, 2))
    p = O.ScalarParams.from_ra_pr(1e6, 4.38, dt=1e-3, n_avg=4, t_bot=0.8, t_top=0.1, z_explicit=wz)
    for n in (0, 1, 3):
        sub, diag, sup, bz, tau = host_z_system(d, n)
        osub, odiag, osup, obz = O.z_matrix(g, tau * p.kappa * (1.0 - wz), p)
        for a, b in ((sub, osub), (diag, odiag), (sup, osup), (bz, obz)):
            np.testing.assert_allclose(a, b, rtol=1e-14, atol=0)


@pytest.mark.parametrize("nz,gamma", [(1, 0.0), (2, 1.0), (3, 1.0), (12, 2.5), (40, 1.5)])
def test_host_z_face_weights_match_oracle(nz, gamma):
    """The library builds its z weights from the derivative of the interpolated
    primitive (Lagrange basis); the oracle solves the cell-mean system."""
    (d, keep), (xf, yf, zf) = _desc(nc=(6, 5, nz), m=(2, 3, 1), gamma=gamma, face_order=4)
    got = host_z_face_weights(d)
    g = O.Grid(xf, yf, zf, (2, 3, 1))
    cells, wts = O.scalar.face_weights(g.z, 4)
    want = np.zeros((nz + 1, 4))
    for f in range(nz + 1):
        for s in range(4):
            if wts[f, s] != 0.0:
                want[f, cells[f, s] - (f - 2)] += wts[f, s]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("order", [0, 2, 4])
def test_face_order_accepted(order):
    (d, keep), _ = _desc(face_order=order)
    host_z_system(d, 0)


def _random_faces(rng, n):
    h = rng.uniform(0.6, 1.5, n)
    return np.concatenate([[0.0], np.cumsum(h)]) / h.sum()


@pytest.mark.parametrize("walls,n", [((False, False), (12, 15)), ((False, False), (1, 2)), ((False, False), (3, 2)),
                                     ((True, True), (12, 15)), ((True, True), (3, 4)), ((True, False), (5, 1)),
                                     ((False, True), (2, 6))])
def test_host_face_weights_xy_match_oracle(walls, n):
    """Fourth-order face weights of stretched x and y axes, periodic (wrapped,
    also on axes shorter than the stencil) and walled, against the oracle's
    moment solve; the z axis through the same call equals mr_host_z_face_weights."""
    rng = np.random.default_rng(5)
    nx, ny = n
    xf = inputs.tanh_faces(nx, 1.5) if walls[0] else _random_faces(rng, nx)
    yf = _random_faces(rng, ny)
    zf = inputs.tanh_faces(8, 1.5)
    d, keep = make_desc(xf, yf, zf, (1, 1, 2), ra=1e6, pr=4.38, dt=1e-5, face_order=4,
                        side_x="walls" if walls[0] else "periodic", side_y="walls" if walls[1] else "periodic")
    g = O.Grid(xf, yf, zf, (1, 1, 2), periodic=(not walls[0], not walls[1], False))
    for axis, ax in ((0, g.x), (1, g.y)):
        got = host_face_weights(d, axis)
        cells, wts = O.scalar.face_weights(ax, 4)
        assert got.shape == (ax.n + 1, 4)
        # the oracle packs a walled stencil from slot 0 and names its cells; the
        # library's slot s is cell f-2+s (wrapped on a periodic axis)
        want = np.zeros((ax.n + 1, 4))
        for f in range(wts.shape[0]):
            for s_ in range(4):
                if wts[f, s_] != 0.0:
                    slot = s_ if ax.periodic else cells[f, s_] - (f - 2)
                    if ax.periodic:
                        assert cells[f, s_] == (f - 2 + s_) % ax.n
                    want[f, slot] += wts[f, s_]
        if ax.periodic:
            want[ax.n] = want[0]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(host_face_weights(d, 2), host_z_face_weights(d))
    buf = np.zeros(64)
    for axis in (-1, 3):
        assert _lib.lib().mr_host_face_weights(ctypes.byref(d), axis,
                                               buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == _lib.MR_EINVAL


def test_face_order4_takes_stretched_x_and_y():
    rng = np.random.default_rng(3)
    yf = _random_faces(rng, 15)
    xf = inputs.tanh_faces(12, 1.5)
    for order in (2, 4):
        d, keep = make_desc(xf, yf, inputs.tanh_faces(14, 1.5), (2, 3, 2), ra=1e6, pr=4.38, dt=1e-3,
                            face_order=order, side_x="walls")
        host_z_system(d, 0)


def _init_status(**over):
    """mr_init status for a descriptor with one field changed (checked on the
    host before any HIP call)."""
    (d, keep), _ = _desc()
    for k, v in over.items():
        setattr(d, k, v)
    ctx = ctypes.c_void_p()
    return _lib.lib().mr_init(ctypes.byref(d), ctypes.byref(ctx))


@pytest.mark.parametrize("field,value", [
    ("mx", 0), ("ncz", 0), ("ncx", 2), ("dt", 0.0), ("dt", -1.0), ("ra", 0.0), ("pr", -2.0),
    ("bc_bot", 7), ("precision", 5), ("n_avg", -1), ("dt", float("nan")), ("side_x", 2), ("side_y", -1),
    ("z_explicit", -0.1), ("z_explicit", 0.6), ("z_explicit", float("nan")), ("face_order", 3),
    ("face_order", -4),
])
def test_init_rejects_bad_descriptor(field, value):
    assert _init_status(**{field: value}) == _lib.MR_EINVAL


def test_init_rejects_non_monotone_faces():
    (d, keep), (xf, yf, zf) = _desc()
    zbad = zf.copy()
    zbad[3], zbad[4] = zbad[4], zbad[3]
    d2, keep2 = make_desc(xf, yf, zbad, (2, 3, 2), ra=1e6, pr=4.38, dt=1e-3)
    ctx = ctypes.c_void_p()
    assert _lib.lib().mr_init(ctypes.byref(d2), ctypes.byref(ctx)) == _lib.MR_EINVAL
    assert not ctx.value


def test_init_rejects_large_diffusion_number():
    """2 dt kappa (4/hx^2 + 4/hy^2) > 1 is refused (explicit x/y diffusion)."""
    xf = inputs.uniform_faces(64)
    d, keep = make_desc(xf, xf, inputs.uniform_faces(8), (2, 2, 2), ra=1.0, pr=1.0, dt=1e-3)
    ctx = ctypes.c_void_p()
    assert _lib.lib().mr_init(ctypes.byref(d), ctypes.byref(ctx)) == _lib.MR_EINVAL


@pytest.mark.parametrize("kw", [dict(side_x="walls"), dict(step_method="line"), dict(z_explicit=0.5),
                                dict(face_order=4)])
def test_init_rejects_too_many_z_levels(kw):
    """More z levels than the line solver's 16 chunks x 40 levels is MR_ESHAPE
    unless the column sweeps apply (periodic uniform x and y, the plain method)
    and the line solver is not asked for."""
    xf = inputs.uniform_faces(8)
    d, keep = make_desc(xf, xf, inputs.uniform_faces(642), (2, 2, 2), ra=1e6, pr=1.0, dt=1e-5, **kw)
    ctx = ctypes.c_void_p()
    assert _lib.lib().mr_init(ctypes.byref(d), ctypes.byref(ctx)) == _lib.MR_ESHAPE
    with pytest.raises(_lib.MRError) as e:
        host_z_system(d, 0)
    assert e.value.status == _lib.MR_ESHAPE


def test_tall_columns_accepted_for_column_sweeps():
    """1024 z levels on periodic uniform x and y with the plain method: the
    descriptor is valid (column sweeps), in both precisions and step methods
    "auto" and "sweep"."""
    xf = inputs.uniform_faces(8)
    for prec in ("fp64", "fp32"):
        for method in ("auto", "sweep"):
            d, keep = make_desc(xf, xf, inputs.tanh_faces(1024, 2.0), (2, 2, 2), ra=1e6, pr=1.0, dt=1e-5,
                                precision=prec, step_method=method)
            sub, diag, sup, bz, tau = host_z_system(d, 0)
            assert diag.shape == (1024,) and tau == 1e-5


@pytest.mark.parametrize("kw", [dict(side_y="walls"), dict(z_explicit=0.25), dict(face_order=4),
                                dict(stretch=True)])
def test_column_sweeps_refused_where_they_do_not_apply(kw):
    """step_method "sweep" needs periodic uniform x and y and the plain method (MR_EINVAL)."""
    kw = dict(kw)
    xf = inputs.uniform_faces(12)
    if kw.pop("stretch", False):
        xf = np.concatenate([[0.0], np.cumsum(np.linspace(1.0, 2.0, 12))])
        xf /= xf[-1]
    d, keep = make_desc(xf, inputs.uniform_faces(12), inputs.uniform_faces(8), (2, 2, 2), ra=1e6, pr=1.0,
                        dt=1e-5, step_method="sweep", **kw)
    with pytest.raises(_lib.MRError) as e:
        host_z_system(d, 0)
    assert e.value.status == _lib.MR_EINVAL


def test_unknown_step_method_rejected():
    assert _init_status(step_method=3) == _lib.MR_EINVAL
    assert _init_status(step_method=-1) == _lib.MR_EINVAL


def test_sweep_tile_validated():
    """The column sweeps' tile is 0 (chosen from nx) or one of four shapes;
    256 x 4 (1) exists in FP64 only."""
    assert _init_status(sweep_tile=5) == _lib.MR_EINVAL
    assert _init_status(sweep_tile=-1) == _lib.MR_EINVAL
    assert _init_status(sweep_tile=1, precision=_lib.MR_FP32) == _lib.MR_EINVAL


def test_null_arguments_rejected():
    L = _lib.lib()
    assert L.mr_init(None, None) == _lib.MR_EINVAL
    assert L.mr_destroy(None) == _lib.MR_OK
    assert L.mr_scalar_step(None, 0, None, None, None, None, None, None, None) == _lib.MR_EINVAL
    assert L.mr_nusselt(None, None, None, None, None, None) == _lib.MR_EINVAL
    assert L.mr_copy_probe(None, None, 16, None) == _lib.MR_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; more than one exits with a message before any GPU work."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_init_rejects_levels_beyond_32bit_byte_offsets():
    """A z level of 24000 x 24000 cells holds 5.76e8 values: 2.3 GB in FP32 is
    addressable with the step's 32-bit byte offsets, 4.6 GB in FP64 is not
    (MR_ESHAPE), although (nz + 1) nx ny stays below 2^31 with one level."""
    f = inputs.uniform_faces(24000)
    zf = inputs.uniform_faces(1)
    d32, keep32 = make_desc(f, f, zf, (1, 1, 1), ra=1.0, pr=1.0, dt=1e-12, precision="fp32")
    host_z_system(d32, 0)
    d64, keep64 = make_desc(f, f, zf, (1, 1, 1), ra=1.0, pr=1.0, dt=1e-12, precision="fp64")
    with pytest.raises(_lib.MRError) as e:
        host_z_system(d64, 0)
    assert e.value.status == _lib.MR_ESHAPE


@pytest.mark.parametrize("ckpt", [0, -3, 2.5])
def test_rollout_rejects_bad_checkpoint_interval(ckpt):
    """The rollout refuses a checkpoint interval that is not a positive integer
    before it touches the context or a GPU."""
    import torch
    from paper_1805_03426_amd.autograd import rollout
    t = torch.zeros((2, 2, 2), dtype=torch.float64)
    with pytest.raises(ValueError):
        rollout(None, t, t, t, t, 3, ckpt)
