"""ctypes view of the C ABI in include/mrscalar.h (argument marshalling only).

The shared library libmrscalar.so is built in-tree by
``python -m paper_1805_03426_amd.build``; loading fails loudly if it is
missing -- there is no fallback implementation.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_void_p, c_char_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmrscalar.so")

MR_OK, MR_EINVAL, MR_ESHAPE, MR_EHIP, MR_ENOMEM, MR_ENONFINITE = 0, -1, -2, -3, -4, -5
MR_FP64, MR_FP32 = 0, 1
MR_DIRICHLET, MR_ADIABATIC = 0, 1
MR_PERIODIC, MR_WALLS = 0, 1

# every symbol the header declares
EXPORTS = [
    "mr_init", "mr_destroy", "mr_interpolate_velocity", "mr_interpolate_velocity_backward",
    "mr_divergence", "mr_scalar_step", "mr_adjoint_seed", "mr_scalar_step_backward",
    "mr_velocity_grad", "mr_nusselt", "mr_copy_probe", "mr_host_refinement_table",
    "mr_host_z_system", "mr_get_dims", "mr_status_string", "mr_last_hip_error",
    "mr_thermal_dissipation", "mr_interpolate_velocity_time", "mr_integrate_scalar",
    "mr_coarse_step", "mr_host_z_face_weights", "mr_host_face_weights", "mr_scalar_steps",
    "mr_scalar_steps_backward", "mr_get_step_method",
    "mr_nusselt_noalloc",
]


class mr_desc(ctypes.Structure):
    _fields_ = [
        ("ncx", c_int32), ("ncy", c_int32), ("ncz", c_int32),
        ("mx", c_int32), ("my", c_int32), ("mz", c_int32),
        ("xf", POINTER(c_double)), ("yf", POINTER(c_double)), ("zf", POINTER(c_double)),
        ("bc_bot", c_int32), ("bc_top", c_int32),
        ("t_bot", c_double), ("t_top", c_double),
        ("ra", c_double), ("pr", c_double),
        ("dt", c_double),
        ("n_avg", c_int32),
        ("precision", c_int32),
        ("side_x", c_int32), ("side_y", c_int32),
        ("z_explicit", c_double),
        ("face_order", c_int32),
        ("step_method", c_int32),
        ("sweep_tile", c_int32),
    ]


class mr_nu(ctypes.Structure):
    _fields_ = [("nu_bot", c_double), ("nu_top", c_double), ("nu_vol", c_double),
                ("nu_paper", c_double), ("mean_theta", c_double)]


class MRError(RuntimeError):
    """A non-zero status from the library."""

    def __init__(self, status, where="", hip_error=0):
        self.status = status
        self.hip_error = hip_error
        msg = "%s failed: %s (status %d)" % (where, status_string(status), status)
        if hip_error:
            msg += ", hipError %d" % hip_error
        super().__init__(msg)


_lib = None


def lib():
    """Load libmrscalar.so once and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmrscalar.so is not built: run `python -m paper_1805_03426_amd.build` "
                          "(expected at %s)" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "mr_init": (c_int, [POINTER(mr_desc), POINTER(c_void_p)]),
        "mr_destroy": (c_int, [P]),
        "mr_interpolate_velocity": (c_int, [P, P, P, P, P, P, P, P]),
        "mr_interpolate_velocity_backward": (c_int, [P, P, P, P, P, P, P, P]),
        "mr_divergence": (c_int, [P, P, P, P, P, P]),
        "mr_scalar_step": (c_int, [P, c_int64, P, P, P, P, P, P, P]),
        "mr_scalar_steps": (c_int, [P, c_int64, c_int32, P, P, POINTER(c_void_p), P, P, P, P]),
        "mr_scalar_steps_backward": (c_int, [P, c_int64, c_int32, P, P, POINTER(c_void_p), P, P, P, P]),
        "mr_adjoint_seed": (c_int, [P, c_int64, P, P, P]),
        "mr_scalar_step_backward": (c_int, [P, c_int64, P, P, P, P, P, P, P, P]),
        "mr_velocity_grad": (c_int, [P, c_int32, POINTER(c_int64), POINTER(c_void_p),
                                     POINTER(c_void_p), P, P, P, P]),
        "mr_nusselt": (c_int, [P, P, P, P, POINTER(mr_nu), P]),
        "mr_nusselt_noalloc": (c_int, [P, P, P, P, P]),
        "mr_copy_probe": (c_int, [P, P, c_int64, P]),
        "mr_thermal_dissipation": (c_int, [P, P, P, POINTER(c_double), P]),
        "mr_interpolate_velocity_time": (c_int, [P, P, P, P, P, P, P, c_int64, c_int64, P, P, P, P]),
        "mr_integrate_scalar": (c_int, [P, P, P, P]),
        "mr_coarse_step": (c_int, [P, c_int64, c_int32, P, P, P, P, P, P, P, P, P, POINTER(c_void_p),
                                   POINTER(c_int32), POINTER(c_int32), P, P]),
        "mr_host_refinement_table": (c_int, [POINTER(mr_desc), c_int32, POINTER(c_double),
                                             POINTER(c_int32)]),
        "mr_host_z_system": (c_int, [POINTER(mr_desc), c_int64, POINTER(c_double),
                                     POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                     POINTER(c_double)]),
        "mr_host_z_face_weights": (c_int, [POINTER(mr_desc), POINTER(c_double)]),
        "mr_host_face_weights": (c_int, [POINTER(mr_desc), c_int32, POINTER(c_double)]),
        "mr_get_dims": (c_int, [P, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                POINTER(c_int32)]),
        "mr_get_step_method": (c_int, [P, POINTER(c_int32)]),
        "mr_status_string": (c_char_p, [c_int]),
        "mr_last_hip_error": (c_int, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def status_string(status):
    try:
        return lib().mr_status_string(status).decode()
    except ImportError:
        return "status %d" % status


def check(status, where, ctx=None):
    if status != MR_OK:
        hip = lib().mr_last_hip_error(ctx) if ctx else 0
        raise MRError(status, where, hip)
