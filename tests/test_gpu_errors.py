"""Error paths of the diagnostics on the GPU: a NaN or an infinity in the
scalar field reaches the compensated reductions, and the calls that return a
host summary report MR_ENONFINITE instead of a number (the asynchronous form
leaves the non-finite values in the device output)."""
import math

import numpy as np
import pytest
import torch

from paper_1805_03426_amd import _lib
from tests.test_gpu_parity import Case, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_nonfinite_scalar_is_reported(bad, prec):
    print("case non-finite", bad, prec, flush=True)
    case = Case((6, 5, 8), (2, 2, 2), 1.5, kmax=1, precision=prec, random_velocity=True, dt=1e-4)
    th = case.th0.copy()
    th[3, 4, 5] = bad
    w = np.zeros((case.g.z.n + 1,) + case.g.shape[1:])
    with case.ctx() as ctx:
        dth, dw = case.d(th), case.d(w)
        with pytest.raises(_lib.MRError) as e:
            ctx.nusselt(dth, dw)
        assert e.value.status == _lib.MR_ENONFINITE
        with pytest.raises(_lib.MRError) as e:
            ctx.thermal_dissipation(dth)
        assert e.value.status == _lib.MR_ENONFINITE
        # asynchronous forms: no status, the non-finite sums stay on the device
        prof, _ = ctx.nusselt(dth, dw, sync=False)
        diss, _ = ctx.thermal_dissipation(dth, sync=False)
        torch.cuda.synchronize()
        assert not np.all(np.isfinite(host(prof)))
        assert not math.isfinite(host(diss)[0])
        # a finite field after the failure: the context still works
        _, s = ctx.nusselt(case.d(case.th0), dw)
        assert math.isfinite(s["nu_vol"])
