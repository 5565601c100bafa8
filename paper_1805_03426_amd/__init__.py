"""MI355X (gfx950) library for the dense-grid scalar step of the
multiple-resolution finite-volume scheme (Chong, Ding & Xia): divergence-free
coarse-to-dense velocity refinement (also interpolated in time), central-flux
advection (second or fourth order) with implicit or partly explicit z
diffusion in the Euler-leapfrog integrator, periodic or walled sides, the
dense-to-coarse integration, the native coarse step of the temporal strategy,
Nusselt and dissipation diagnostics and the discrete adjoint, all as
hand-written HIP kernels behind a C ABI (include/mrscalar.h).  PyTorch
supplies device memory and streams only.
"""
from ._lib import MRError  # noqa: F401


def __getattr__(name):
    if name in ("Context", "copy_probe", "make_desc", "host_refinement_table", "host_z_system",
                "host_z_face_weights"):
        from . import context
        return getattr(context, name)
    if name in ("rollout", "ScalarRollout"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
