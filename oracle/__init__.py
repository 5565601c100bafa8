"""Plain FP64 CPU oracle of the multiple-resolution dense-grid scalar step.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the HIP library is checked against.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the product path
never does, and it shares no code with the HIP library (it never imports the
package ``paper_1805_03426_amd`` and the library never reads anything here).
Inputs reach it as plain NumPy arrays.

What it computes (Chong, Ding & Xia, "Multiple-resolution scheme in
finite-volume code for active or passive scalar turbulence"):

* ``grid``     -- dense and coarse geometry (Sec. 3.1, "Grid design");
* ``refine``   -- the mass-conserving quadratic split R = A_s A^-1
                  (Eqs. 12-19), the stepwise divergence-free refinement of the
                  coarse staggered velocity (Sec. 3.2, Fig. 5a), its discrete
                  divergence, and the transpose of the refinement;
* ``scalar``   -- finite-volume advection and diffusion of the scalar
                  (Eqs. 2, 5), the Euler-leapfrog step with the averaging step
                  every N_p steps (Eqs. 6, 7) with z-diffusion implicit, the
                  Nusselt diagnostics (Eq. 22), and the discrete adjoint of a
                  step and of a whole rollout;
* ``intergrid`` -- the volume-weighted dense-to-coarse integration of the
                  scalar (Eq. 20), the linear-in-time coarse velocity of the
                  temporal strategy (Eq. 21), one coarse step of the
                  multiple-resolution loop (Fig. 6), and the dissipation
                  Nusselt number Nu_T (Eq. 23).

Pins (tests marked ``not gpu``) tie every function to closed forms, invariants
and brute force; see each function's docstring for the passage it follows.
All arithmetic is float64.
"""
from .grid import Axis, Grid
from .refine import (r_matrix, stencil_start, refine_velocity, refine_velocity_transpose,
                     divergence, split)
from .scalar import (ScalarParams, step_kind, z_matrix, thomas, advection, lap_h, scalar_step,
                     nusselt, step_vjp, rollout, rollout_loss_grad)
from .intergrid import integrate_scalar, blend_velocity, coarse_step, thermal_dissipation

__all__ = ["Axis", "Grid", "r_matrix", "stencil_start", "refine_velocity",
           "refine_velocity_transpose", "divergence", "split", "ScalarParams", "step_kind",
           "z_matrix", "thomas", "advection", "lap_h", "scalar_step", "nusselt", "step_vjp",
           "rollout", "rollout_loss_grad", "integrate_scalar", "blend_velocity", "coarse_step",
           "thermal_dissipation"]
