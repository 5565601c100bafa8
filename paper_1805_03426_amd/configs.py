"""Named synthetic workloads of the multiple-resolution scalar step.

Every workload is a Rayleigh-Benard cell [0,1]^3, periodic in x and y, with
walls at z = 0 (T = 1) and z = 1 (T = 0); the coarse grid is refined by the
factors (mx, my, mz) into the dense scalar grid (paper Sec. 3.1).  The dense z
faces follow a tanh law with clustering parameter ``gamma`` (0 = uniform),
which puts every M-th dense face on the coarse grid, as the paper's grid design
requires.  Ra and Pr set the diffusivity kappa = (Ra Pr)^(-1/2) of the heat
equation (Eq. 2).

The names say what each workload is: dense size, refinement factor and
storage precision.
"""
from dataclasses import dataclass, field


@dataclass(frozen=True)
class Workload:
    name: str
    nc: tuple            # coarse cells (ncx, ncy, ncz)
    m: tuple             # refinement factors (mx, my, mz)
    gamma: float         # tanh clustering of the z faces (0 = uniform)
    ra: float
    pr: float
    steps: int
    kmax: int            # largest wavenumber of the synthetic vector potential
    precision: str       # "fp64" | "fp32"
    nu_every: int = 0    # Nusselt diagnostics every this many steps (0 = never)
    ckpt_every: int = 0  # adjoint checkpoint interval (0 = no adjoint)
    n_avg: int = 50      # averaging step period N_p (paper Sec. 2.2)
    cfl: float = 0.3
    urms: float = 0.2
    noise: float = 0.02

    @property
    def n(self):
        return tuple(c * m for c, m in zip(self.nc, self.m))

    @property
    def cells(self):
        nx, ny, nz = self.n
        return nx * ny * nz


WORKLOADS = {w.name: w for w in [
    # 32^3 -> 64^3, uniform, Ra 1e6: small enough for the oracle in seconds.
    Workload("rb64-m2-fp64", (32, 32, 32), (2, 2, 2), 0.0, 1e6, 4.38, 10, 8, "fp64"),
    # 128^3 -> 256^3, tanh 1.5, Ra 1e8: the FP64 throughput workload.
    Workload("rb256-m2-fp64", (128, 128, 128), (2, 2, 2), 1.5, 1e8, 4.38, 100, 32, "fp64",
             nu_every=10),
    # 192^3 -> 576^3, tanh 2.0, Ra 1e8, Pr 100: the FP32 precision tier.
    Workload("rb576-m3-fp32", (192, 192, 192), (3, 3, 3), 2.0, 1e8, 100.0, 200, 32, "fp32"),
    # 128^3 -> 256^3 adjoint, FP32, 20 steps, checkpoint every 5.
    Workload("rb256-m2-adjoint-fp32", (128, 128, 128), (2, 2, 2), 1.5, 1e8, 4.38, 20, 32, "fp32",
             ckpt_every=5),
    # 512x512x256 -> 1024x1024x512, tanh 2.5, Ra 1e9, Pr 7, FP32, forward + adjoint.
    Workload("rb1024x1024x512-m2-fp32", (512, 512, 256), (2, 2, 2), 2.5, 1e9, 7.0, 50, 32, "fp32",
             ckpt_every=10),
    # The same grid and inputs in FP64, with the Nusselt diagnostics every 10
    # steps: the largest workload that fits one GPU, in the paper's precision.
    Workload("rb1024x1024x512-m2-fp64", (512, 512, 256), (2, 2, 2), 2.5, 1e9, 7.0, 50, 32, "fp64",
             nu_every=10, ckpt_every=10),
]}
