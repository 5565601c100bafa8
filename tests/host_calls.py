"""Host-side entry points of the library exercised in a child process (the
sanitizer test runs it against an ASan/UBSan build of the host code): the
descriptor checks, the refinement tables, the z systems and the fourth-order
z weights for every option, and the error paths of mr_init.  Needs no GPU.

usage: python tests/host_calls.py <library path>"""
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1805_03426_amd import _lib, inputs  # noqa: E402

_lib.LIB_PATH = sys.argv[1]

from paper_1805_03426_amd.context import (host_refinement_table, host_z_face_weights,  # noqa: E402
                                          host_z_system, make_desc)


def main():
    xf = inputs.uniform_faces(24)
    zf = inputs.tanh_faces(30, 2.0)
    cases = (dict(), dict(side_x="walls", side_y="walls"), dict(face_order=4), dict(z_explicit=0.5),
             dict(precision="fp32"), dict(bc_bot="adiabatic"), dict(step_method="sweep", sweep_tile=3))
    for kw in cases:
        d, keep = make_desc(xf, xf, zf, (2, 3, 2), 1e6, 1.0, 1e-5, **kw)
        for ax in range(3):
            host_refinement_table(d, ax)
        for n in (0, 1, 2, 49):
            host_z_system(d, n)
        host_z_face_weights(d)
    # tall columns (no line-solver chunks) and a single coarse cell per axis
    d, keep = make_desc(inputs.uniform_faces(8), inputs.uniform_faces(8), inputs.tanh_faces(1024, 2.0),
                        (2, 2, 2), 1e6, 1.0, 1e-5)
    host_z_system(d, 0)
    d, keep = make_desc([0.0, 1.0], [0.0, 1.0], [0.0, 0.5, 1.0], (1, 1, 1), 1e6, 1.0, 1e-5)
    host_z_system(d, 0)
    # mr_init's argument checks (all before any HIP call)
    L = _lib.lib()
    ctx = ctypes.c_void_p()
    bad = dict(step_method=5, sweep_tile=9, face_order=3, z_explicit=0.9, n_avg=-1, dt=-1.0)
    for field, value in bad.items():
        d, keep = make_desc(xf, xf, zf, (2, 3, 2), 1e6, 1.0, 1e-5)
        setattr(d, field, value)
        assert L.mr_init(ctypes.byref(d), ctypes.byref(ctx)) == _lib.MR_EINVAL, field
    assert L.mr_init(None, ctypes.byref(ctx)) == _lib.MR_EINVAL
    print("host calls ok", flush=True)


if __name__ == "__main__":
    main()
