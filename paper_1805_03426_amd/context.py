"""Python face of the library: one ``Context`` per grid.

Every method marshals torch tensors (device memory) and the current torch
stream into a C ABI call; all arithmetic runs in the HIP kernels.  Shapes
follow include/mrscalar.h: dense scalar, u, v ``(nz, ny, nx)``, dense w
``(nz+1, ny, nx)``, coarse U, V ``(ncz, ncy, ncx)``, coarse W
``(ncz+1, ncy, ncx)``, x fastest.
"""
import ctypes
from ctypes import byref, c_double, c_int32, c_int64, c_void_p

import numpy as np
import torch

from . import _lib
from ._lib import MRError, check, lib, mr_desc, mr_nu

_BC = {"dirichlet": _lib.MR_DIRICHLET, "adiabatic": _lib.MR_ADIABATIC}
_PREC = {"fp64": _lib.MR_FP64, "fp32": _lib.MR_FP32}
_SIDE = {"periodic": _lib.MR_PERIODIC, "walls": _lib.MR_WALLS}
_METHOD = {"auto": 0, "line": 1, "sweep": 2}


def make_desc(xf, yf, zf, m, ra, pr, dt, n_avg=50, t_bot=1.0, t_top=0.0, bc_bot="dirichlet",
              bc_top="dirichlet", precision="fp64", side_x="periodic", side_y="periodic",
              z_explicit=0.0, face_order=2, step_method="auto", sweep_tile=0):
    """Build an ``mr_desc``; returns (desc, keepalive) -- keep the second alive
    while the descriptor is in use (it owns the face arrays).  side_x / side_y:
    "periodic" or "walls" (adiabatic no-slip side walls); z_explicit: share w of
    the z diffusion taken explicit on the lagged level (0 to 1/2); face_order:
    2 (mean of the two cells) or 4 (fourth-order face values, any widths);
    step_method: "auto", "line" (fused line solver) or "sweep" (column sweeps);
    sweep_tile: 0 (chosen from nx) or 1..4 (256 x 4, 192 x 4, 128 x 8, 64 x 16)."""
    faces = [np.ascontiguousarray(np.asarray(f, dtype=np.float64)) for f in (xf, yf, zf)]
    mx, my, mz = (int(a) for a in m)
    n = [f.size - 1 for f in faces]
    for ni, mi in zip(n, (mx, my, mz)):
        if mi < 1 or ni % mi:
            raise ValueError("dense cells (%d) must be a multiple of the refinement factor (%d)" % (ni, mi))
    d = mr_desc()
    d.ncx, d.ncy, d.ncz = n[0] // mx, n[1] // my, n[2] // mz
    d.mx, d.my, d.mz = mx, my, mz
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(c_double))
    d.xf, d.yf, d.zf = ptr(faces[0]), ptr(faces[1]), ptr(faces[2])
    d.bc_bot, d.bc_top = _BC[bc_bot], _BC[bc_top]
    d.t_bot, d.t_top = float(t_bot), float(t_top)
    d.ra, d.pr, d.dt = float(ra), float(pr), float(dt)
    d.n_avg = int(n_avg)
    d.precision = _PREC[precision]
    d.side_x, d.side_y = _SIDE[side_x], _SIDE[side_y]
    d.z_explicit = float(z_explicit)
    d.face_order = int(face_order)
    d.step_method = _METHOD[step_method]
    d.sweep_tile = int(sweep_tile)
    return d, faces


def host_refinement_table(desc, axis):
    """R tables (nc, m, 3) and stencil starts of one axis, built on the host by
    the library (no GPU involved)."""
    nc = [desc.ncx, desc.ncy, desc.ncz][axis]
    m = [desc.mx, desc.my, desc.mz][axis]
    R = np.zeros((nc, m, 3))
    s = np.zeros(nc, dtype=np.int32)
    check(lib().mr_host_refinement_table(byref(desc), axis,
                                         R.ctypes.data_as(ctypes.POINTER(c_double)),
                                         s.ctypes.data_as(ctypes.POINTER(c_int32))),
          "mr_host_refinement_table")
    return R, s


def host_z_system(desc, n):
    """(sub, diag, sup, bz, tau) of the implicit z system of step n (host only)."""
    nz = desc.ncz * desc.mz
    arrs = [np.zeros(nz) for _ in range(4)]
    tau = c_double()
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(c_double))
    check(lib().mr_host_z_system(byref(desc), n, *[P(a) for a in arrs], byref(tau)), "mr_host_z_system")
    return (*arrs, tau.value)


def host_z_face_weights(desc):
    """(nz+1, 4) fourth-order face weights of the z axis, face f's for the cells
    f-2..f+1, as the step uses them with face_order 4 (host only)."""
    nz = desc.ncz * desc.mz
    w = np.zeros((nz + 1, 4))
    check(lib().mr_host_z_face_weights(byref(desc), w.ctypes.data_as(ctypes.POINTER(c_double))),
          "mr_host_z_face_weights")
    return w


def host_face_weights(desc, axis):
    """(n+1, 4) fourth-order face weights of one axis (0 = x, 1 = y, 2 = z),
    face f's for the cells f-2..f+1 (wrapped on a periodic axis), as the step
    uses them with face_order 4 (host only)."""
    n = (desc.ncx * desc.mx, desc.ncy * desc.my, desc.ncz * desc.mz)[axis]
    w = np.zeros((n + 1, 4))
    check(lib().mr_host_face_weights(byref(desc), axis, w.ctypes.data_as(ctypes.POINTER(c_double))),
          "mr_host_face_weights")
    return w


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """Grid tables on the current GPU plus typed entry points.

    Arguments as for ``make_desc``: dense face coordinates xf, yf, zf,
    refinement factors m = (mx, my, mz), Ra, Pr, the fixed time step dt, the
    averaging period n_avg (Eq. 7), the wall conditions and values of the
    scalar, the storage precision ("fp64" or "fp32"), the x and y sides
    ("periodic" or "walls"), the explicit share z_explicit of the z diffusion
    (0 to 1/2), the face order of the advection (2 or 4) and the step method
    ("auto", "line" or "sweep")."""

    def __init__(self, xf, yf, zf, m, ra, pr, dt, n_avg=50, t_bot=1.0, t_top=0.0,
                 bc_bot="dirichlet", bc_top="dirichlet", precision="fp64", side_x="periodic",
                 side_y="periodic", z_explicit=0.0, face_order=2, step_method="auto", sweep_tile=0):
        if not torch.cuda.is_available():
            raise RuntimeError("the multiple-resolution library needs a HIP GPU")
        desc, keep = make_desc(xf, yf, zf, m, ra, pr, dt, n_avg, t_bot, t_top, bc_bot, bc_top, precision,
                               side_x, side_y, z_explicit, face_order, step_method, sweep_tile)
        self.desc, self._keep = desc, keep
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._ctx = c_void_p()
        check(lib().mr_init(byref(desc), byref(self._ctx)), "mr_init")
        self.nx, self.ny, self.nz = desc.ncx * desc.mx, desc.ncy * desc.my, desc.ncz * desc.mz
        self.ncx, self.ncy, self.ncz = desc.ncx, desc.ncy, desc.ncz
        self.m = (desc.mx, desc.my, desc.mz)
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.n_avg = n_avg
        self.dt = dt

    # ------------------------------------------------------------ helpers
    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().mr_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def shape_cell(self):
        return (self.nz, self.ny, self.nx)

    @property
    def shape_w(self):
        return (self.nz + 1, self.ny, self.nx)

    @property
    def shape_coarse(self):
        return (self.ncz, self.ncy, self.ncx)

    @property
    def shape_coarse_w(self):
        return (self.ncz + 1, self.ncy, self.ncx)

    def empty(self, shape):
        return torch.empty(shape, dtype=self.dtype, device=self.device)

    def _ptr(self, t, shape, name, dtype=None):
        if t is None:
            return None
        dtype = dtype or self.dtype
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise ValueError("%s must be a GPU tensor" % name)
        if t.dtype != dtype:
            raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        return c_void_p(t.data_ptr())

    # ------------------------------------------------------------ refinement
    def interpolate_velocity(self, U, V, W, out=None):
        """Coarse (U, V, W) -> dense (u, v, w) (divergence-free refinement)."""
        if out is None:
            out = (self.empty(self.shape_cell), self.empty(self.shape_cell), self.empty(self.shape_w))
        u, v, w = out
        args = [self._ptr(U, self.shape_coarse, "U"), self._ptr(V, self.shape_coarse, "V"),
                self._ptr(W, self.shape_coarse_w, "W"), self._ptr(u, self.shape_cell, "u"),
                self._ptr(v, self.shape_cell, "v"), self._ptr(w, self.shape_w, "w")]
        check(lib().mr_interpolate_velocity(self._ctx, *args, _stream()), "mr_interpolate_velocity", self._ctx)
        return u, v, w

    def interpolate_velocity_backward(self, gu, gv, gw, out=None):
        """Transpose of the refinement: dense face adjoints -> coarse face adjoints."""
        if out is None:
            out = (self.empty(self.shape_coarse), self.empty(self.shape_coarse),
                   self.empty(self.shape_coarse_w))
        gU, gV, gW = out
        args = [self._ptr(gu, self.shape_cell, "gu"), self._ptr(gv, self.shape_cell, "gv"),
                self._ptr(gw, self.shape_w, "gw"), self._ptr(gU, self.shape_coarse, "gU"),
                self._ptr(gV, self.shape_coarse, "gV"), self._ptr(gW, self.shape_coarse_w, "gW")]
        check(lib().mr_interpolate_velocity_backward(self._ctx, *args, _stream()),
              "mr_interpolate_velocity_backward", self._ctx)
        return gU, gV, gW

    def interpolate_velocity_time(self, U0, V0, W0, U1, V1, W1, i, mt, out=None):
        """Dense velocity at fraction i/mt of a coarse step: the refinement of
        (1 - i/mt) (U0, V0, W0) + (i/mt) (U1, V1, W1)."""
        if out is None:
            out = (self.empty(self.shape_cell), self.empty(self.shape_cell), self.empty(self.shape_w))
        u, v, w = out
        cs, cw = self.shape_coarse, self.shape_coarse_w
        args = [self._ptr(U0, cs, "U0"), self._ptr(V0, cs, "V0"), self._ptr(W0, cw, "W0"),
                self._ptr(U1, cs, "U1"), self._ptr(V1, cs, "V1"), self._ptr(W1, cw, "W1"),
                c_int64(i), c_int64(mt), self._ptr(u, self.shape_cell, "u"),
                self._ptr(v, self.shape_cell, "v"), self._ptr(w, self.shape_w, "w")]
        check(lib().mr_interpolate_velocity_time(self._ctx, *args, _stream()),
              "mr_interpolate_velocity_time", self._ctx)
        return u, v, w

    def integrate_scalar(self, theta, out=None):
        """Coarse scalar: volume-weighted mean of theta over each coarse cell."""
        if out is None:
            out = self.empty(self.shape_coarse)
        check(lib().mr_integrate_scalar(self._ctx, self._ptr(theta, self.shape_cell, "theta"),
                                        self._ptr(out, self.shape_coarse, "out"), _stream()),
              "mr_integrate_scalar", self._ctx)
        return out

    def coarse_step(self, n0, mt, U0, V0, W0, U1, V1, W1, uvw, ring, prev, cur, theta_c=None):
        """One coarse step (mt scalar steps on the time-interpolated, refined
        velocity, then the integration of the newest scalar into theta_c).
        ``ring`` holds three scalar buffers; ring[cur] is theta^{n0}, ring[prev]
        theta^{n0-1}.  Returns the new (prev, cur) indices."""
        if len(ring) != 3:
            raise ValueError("ring must hold three scalar buffers")
        cs, cw = self.shape_coarse, self.shape_coarse_w
        u, v, w = uvw
        rp = (c_void_p * 3)(*[self._ptr(t, self.shape_cell, "ring[%d]" % q).value for q, t in enumerate(ring)])
        p, c = c_int32(prev), c_int32(cur)
        args = [self._ptr(U0, cs, "U0"), self._ptr(V0, cs, "V0"), self._ptr(W0, cw, "W0"),
                self._ptr(U1, cs, "U1"), self._ptr(V1, cs, "V1"), self._ptr(W1, cw, "W1"),
                self._ptr(u, self.shape_cell, "u"), self._ptr(v, self.shape_cell, "v"),
                self._ptr(w, self.shape_w, "w"), rp, byref(p), byref(c),
                self._ptr(theta_c, cs, "theta_c")]
        check(lib().mr_coarse_step(self._ctx, c_int64(n0), c_int32(mt), *args, _stream()),
              "mr_coarse_step", self._ctx)
        return p.value, c.value

    def divergence(self, u, v, w, out=None):
        """Device tensor [max |net flux|, max |net flux| / sum |face flux|] (float64)."""
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=self.device)
        args = [self._ptr(u, self.shape_cell, "u"), self._ptr(v, self.shape_cell, "v"),
                self._ptr(w, self.shape_w, "w"), self._ptr(out, (2,), "out", torch.float64)]
        check(lib().mr_divergence(self._ctx, *args, _stream()), "mr_divergence", self._ctx)
        return out

    # ------------------------------------------------------------ step
    def scalar_step(self, n, th_prev, th_cur, out, u, v, w):
        """theta^{n+1} into ``out`` (must differ from th_prev and th_cur)."""
        args = [self._ptr(th_prev, self.shape_cell, "th_prev") if n > 0 else None,
                self._ptr(th_cur, self.shape_cell, "th_cur"), self._ptr(out, self.shape_cell, "out"),
                self._ptr(u, self.shape_cell, "u"), self._ptr(v, self.shape_cell, "v"),
                self._ptr(w, self.shape_w, "w")]
        check(lib().mr_scalar_step(self._ctx, c_int64(n), *args, _stream()), "mr_scalar_step", self._ctx)
        return out

    def scalar_steps(self, n0, th_prev, th_cur, outs, u, v, w):
        """Steps n0 .. n0+len(outs)-1: outs[q] receives theta^{n0+q+1} (each
        output must differ from the two levels before it)."""
        k = len(outs)
        if k < 1:
            raise ValueError("outs must hold at least one buffer")
        op = (c_void_p * k)(*[self._ptr(t, self.shape_cell, "outs[%d]" % q).value for q, t in enumerate(outs)])
        args = [self._ptr(th_prev, self.shape_cell, "th_prev") if n0 > 0 else None,
                self._ptr(th_cur, self.shape_cell, "th_cur"), op,
                self._ptr(u, self.shape_cell, "u"), self._ptr(v, self.shape_cell, "v"),
                self._ptr(w, self.shape_w, "w")]
        check(lib().mr_scalar_steps(self._ctx, c_int64(n0), c_int32(k), *args, _stream()), "mr_scalar_steps",
              self._ctx)
        return outs

    def scalar_steps_backward(self, n0, mu_next, mu_cur, outs, u, v, w):
        """Reverse steps n0 .. n0-len(outs)+1 (all >= 1): outs[q] receives
        mu^{n0-q-1} (each output must differ from the two levels before it);
        mu_next = mu^{n0+1} or None."""
        k = len(outs)
        if k < 1:
            raise ValueError("outs must hold at least one buffer")
        op = (c_void_p * k)(*[self._ptr(t, self.shape_cell, "outs[%d]" % q).value for q, t in enumerate(outs)])
        args = [self._ptr(mu_next, self.shape_cell, "mu_next") if mu_next is not None else None,
                self._ptr(mu_cur, self.shape_cell, "mu_cur"), op,
                self._ptr(u, self.shape_cell, "u"), self._ptr(v, self.shape_cell, "v"),
                self._ptr(w, self.shape_w, "w")]
        check(lib().mr_scalar_steps_backward(self._ctx, c_int64(n0), c_int32(k), *args, _stream()),
              "mr_scalar_steps_backward", self._ctx)
        return outs

    @property
    def step_method(self):
        """The method step sequences run with: "line" or "sweep"."""
        m = c_int32()
        check(lib().mr_get_step_method(self._ctx, byref(m)), "mr_get_step_method", self._ctx)
        return "sweep" if m.value == 2 else "line"

    def step_runner(self, ring, u, v, w):
        """Prepared repeated stepping on fixed buffers: checks the buffers once
        and caches their pointers and the current stream, so each step is one
        library call.  ``ring`` is a list of scalar buffers; run.step(n, a, b, c)
        computes ring[c] from ring[a] (level n-1) and ring[b] (level n)."""
        return _StepRunner(self, ring, u, v, w)

    def adjoint_seed(self, n, lam, out):
        """mu^n = (I - tau_n kappa Lz)^-T lam."""
        check(lib().mr_adjoint_seed(self._ctx, c_int64(n), self._ptr(lam, self.shape_cell, "lam"),
                                    self._ptr(out, self.shape_cell, "out"), _stream()),
              "mr_adjoint_seed", self._ctx)
        return out

    def scalar_step_backward(self, n, mu_next, mu_cur, lam_add, out, u, v, w):
        """Fused reverse step: out = mu^{n-1} (n >= 1) or dL/dtheta^0 (n = 0)."""
        args = [self._ptr(mu_next, self.shape_cell, "mu_next"), self._ptr(mu_cur, self.shape_cell, "mu_cur"),
                self._ptr(lam_add, self.shape_cell, "lam_add"), self._ptr(out, self.shape_cell, "out"),
                self._ptr(u, self.shape_cell, "u"), self._ptr(v, self.shape_cell, "v"),
                self._ptr(w, self.shape_w, "w")]
        check(lib().mr_scalar_step_backward(self._ctx, c_int64(n), *args, _stream()),
              "mr_scalar_step_backward", self._ctx)
        return out

    def velocity_grad(self, steps, thetas, mus, gu, gv, gw):
        """g_u, g_v, g_w += velocity gradient of the given steps (at most 16 per call)."""
        k = len(steps)
        if not (1 <= k <= 16) or len(thetas) != k or len(mus) != k:
            raise ValueError("velocity_grad takes 1..16 steps with matching thetas and mus")
        st = (c_int64 * k)(*steps)
        th = (c_void_p * k)(*[self._ptr(t, self.shape_cell, "theta").value for t in thetas])
        mu = (c_void_p * k)(*[self._ptr(t, self.shape_cell, "mu").value for t in mus])
        check(lib().mr_velocity_grad(self._ctx, k, st, th, mu, self._ptr(gu, self.shape_cell, "gu"),
                                     self._ptr(gv, self.shape_cell, "gv"), self._ptr(gw, self.shape_w, "gw"),
                                     _stream()), "mr_velocity_grad", self._ctx)

    # ------------------------------------------------------------ diagnostics
    def nusselt(self, theta, w, profile=None, sync=True):
        """Nu profile on the nz+1 dense z faces plus summary (device tensor of nz+6
        doubles); with sync=True also returns the summary as a dict."""
        if profile is None:
            profile = torch.empty(self.nz + 6, dtype=torch.float64, device=self.device)
        out = mr_nu() if sync else None
        st = lib().mr_nusselt(self._ctx, self._ptr(theta, self.shape_cell, "theta"),
                              self._ptr(w, self.shape_w, "w"),
                              self._ptr(profile, (self.nz + 6,), "profile", torch.float64),
                              byref(out) if sync else None, _stream())
        check(st, "mr_nusselt", self._ctx)
        if not sync:
            return profile, None
        return profile, dict(nu_bot=out.nu_bot, nu_top=out.nu_top, nu_vol=out.nu_vol,
                             nu_paper=out.nu_paper, mean_theta=out.mean_theta)


    def thermal_dissipation(self, theta, out=None, sync=True):
        """Device tensor {Nu_T, <theta_x^2>, <theta_y^2>, <theta_z^2>} (float64);
        with sync=True also returns them as a dict."""
        if out is None:
            out = torch.empty(4, dtype=torch.float64, device=self.device)
        host = (c_double * 4)() if sync else None
        st = lib().mr_thermal_dissipation(self._ctx, self._ptr(theta, self.shape_cell, "theta"),
                                          self._ptr(out, (4,), "out", torch.float64), host, _stream())
        check(st, "mr_thermal_dissipation", self._ctx)
        if not sync:
            return out, None
        return out, dict(nu_t=host[0], gx2=host[1], gy2=host[2], gz2=host[3])


class _StepRunner:
    def __init__(self, ctx, ring, u, v, w):
        self._ctx = ctx
        self._ring = list(ring)   # keep the tensors alive
        self._p = [ctx._ptr(t, ctx.shape_cell, "ring[%d]" % q) for q, t in enumerate(ring)]
        self._uvw = (ctx._ptr(u, ctx.shape_cell, "u"), ctx._ptr(v, ctx.shape_cell, "v"),
                     ctx._ptr(w, ctx.shape_w, "w"))
        self._keep = (u, v, w)
        self._stream = _stream()
        self._fn = lib().mr_scalar_step

    def step(self, n, a, b, c):
        if c == a or c == b:
            raise ValueError("the output buffer must differ from the inputs")
        st = self._fn(self._ctx._ctx, n, self._p[a], self._p[b], self._p[c], *self._uvw, self._stream)
        if st:
            check(st, "mr_scalar_step", self._ctx._ctx)

    def steps(self, n0, a, b, outs):
        """Steps n0 .. n0+len(outs)-1 from ring[a] (level n0-1) and ring[b]
        (level n0); step n0+q writes ring[outs[q]]."""
        k = len(outs)
        op = (c_void_p * k)(*[self._p[q].value for q in outs])
        st = lib().mr_scalar_steps(self._ctx._ctx, n0, k, self._p[a], self._p[b], op, *self._uvw, self._stream)
        if st:
            check(st, "mr_scalar_steps", self._ctx._ctx)


def copy_probe(src, dst):
    """Device copy with the library's streaming kernel (bandwidth reference)."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < n:
        raise ValueError("destination too small")
    check(lib().mr_copy_probe(c_void_p(src.data_ptr()), c_void_p(dst.data_ptr()), n, _stream()),
          "mr_copy_probe")
