/*
 * mrscalar.h -- C ABI of the MI355X (gfx950) library for the dense-grid scalar
 * step of the multiple-resolution finite-volume scheme (Chong, Ding & Xia,
 * "Multiple-resolution scheme in finite-volume code for active or passive
 * scalar turbulence").
 *
 * The scalar (temperature) lives on a dense grid, the velocity on a coarse
 * grid whose faces are every M-th dense face (paper Sec. 3.1).  The library:
 *   - refines the coarse staggered velocity onto the dense faces so that every
 *     dense cell keeps zero net flux (Sec. 3.2, Eqs. 12-19);
 *   - advances the cell-averaged scalar with finite-volume central advection
 *     (Eqs. 2 and 5) in the Euler-leapfrog integrator with the averaging step
 *     every N_p steps (Eqs. 6 and 7), x/y diffusion explicit on level n-1 and
 *     z diffusion implicit on level n+1 (one tridiagonal solve per (x, y) line);
 *   - reports the heat-flux Nusselt profile (Eq. 22), the mean scalar and the
 *     dissipation Nusselt number Nu_T (Eq. 23);
 *   - runs the inter-grid steps of the multiple-resolution loop: the coarse
 *     velocity interpolated in time (Eq. 21), the dense-to-coarse integration
 *     of the scalar (Eq. 20), and whole coarse steps of M_t scalar steps;
 *   - provides the discrete adjoint of the step and of the refinement.
 *
 * Conventions
 *   Domain: x and y periodic, walls at z = zf[0] and z = zf[nz].
 *   Arrays are C-contiguous with x fastest, indexed [z][y][x]:
 *     dense scalar theta, u (x-faces), v (y-faces):  [nz][ny][nx]
 *     dense w (z-faces, both walls included):        [nz+1][ny][nx]
 *     coarse U, V:                                   [ncz][ncy][ncx]
 *     coarse W (both walls included):                [ncz+1][ncy][ncx]
 *   Face index i of u is the face at xf[i], between cells i-1 and i (cell -1
 *   is the periodic image of cell nx-1); likewise v at yf[j] and w at zf[k].
 *   Element type of every field pointer: double for MR_FP64 contexts, float
 *   for MR_FP32 contexts.  Reductions (Nusselt, divergence) are always double.
 *   Field pointers are device pointers owned by the caller, naturally aligned,
 *   and must not alias unless a function says so.
 *
 * Streams: every call enqueues its kernels on the given hipStream_t (passed as
 * void*, NULL = the null stream) and returns without waiting, except
 * mr_nusselt with a non-NULL host_out, which waits for that stream.
 * A context must not be used from two host threads at once, and calls on one
 * context must not overlap on different streams: the context's work buffers
 * (reduction partials, the sweeps' elimination fields, the blended coarse
 * velocity and the refinement intermediates) are shared by its calls.
 *
 * Errors: every function returns an int status (mr_status).  Arguments are
 * checked on the host before anything is launched; a failed HIP call returns
 * MR_EHIP and its hipError_t is kept for mr_last_hip_error.  Nothing aborts.
 */
#ifndef MRSCALAR_H
#define MRSCALAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mr_ctx mr_ctx;

typedef enum {
  MR_OK = 0,
  MR_EINVAL = -1,      /* invalid argument or descriptor */
  MR_ESHAPE = -2,      /* sizes the kernels cannot handle */
  MR_EHIP = -3,        /* a HIP runtime call failed */
  MR_ENOMEM = -4,      /* device allocation failed */
  MR_ENONFINITE = -5   /* a reduction met NaN or Inf */
} mr_status;

typedef enum { MR_FP64 = 0, MR_FP32 = 1 } mr_precision;
typedef enum { MR_DIRICHLET = 0, MR_ADIABATIC = 1 } mr_wall_bc;
/* Side conditions in x and y: periodic, or adiabatic no-slip walls at both
 * ends (the paper's cube, Sec. 4).  On a walled axis the face arrays keep
 * their shape: face i of u still lies at xf[i], so u[..., 0] is the low wall
 * and the high wall (xf[nx]) is not stored; the library treats both wall
 * faces as zero velocity and zero diffusive flux, whatever the array holds at
 * face 0, writes zero there, and reports zero gradient for it. */
typedef enum { MR_PERIODIC = 0, MR_WALLS = 1 } mr_side;

/* Problem description (host memory; copied by mr_init). */
typedef struct {
  int32_t ncx, ncy, ncz;   /* coarse cells per axis (>= 3 where the refinement factor > 1) */
  int32_t mx, my, mz;      /* refinement factors M_x, M_y, M_z (>= 1), Sec. 3.1 */
  const double* xf;        /* nx+1 dense x faces, strictly increasing; period xf[nx]-xf[0] (or walls) */
  const double* yf;        /* ny+1 dense y faces, strictly increasing; period yf[ny]-yf[0] (or walls) */
  const double* zf;        /* nz+1 dense z faces, strictly increasing; walls at both ends */
  int32_t bc_bot, bc_top;  /* scalar condition on each wall (mr_wall_bc) */
  double t_bot, t_top;     /* wall values for MR_DIRICHLET */
  double ra, pr;           /* diffusivity kappa = (Ra Pr)^(-1/2) (Eq. 2); Nu uses (Ra Pr)^(1/2) */
  double dt;               /* fixed time step (> 0) */
  int32_t n_avg;           /* averaging period N_p of Eq. 7 (0 = never) */
  int32_t precision;       /* mr_precision of every field buffer */
  int32_t side_x, side_y;  /* mr_side of the x and y axes (0 = periodic) */
  double z_explicit;       /* w in [0, 1/2]: share of the z diffusion taken explicit on the
                              lagged level (0 = fully implicit, 1/2 = Crank-Nicolson across
                              the step's time span; a reading of Sec. 2.2's implicit z) */
  int32_t face_order;      /* face value of the advected scalar: 2 (or 0) = mean of the two cells,
                              4 = fourth order (Sec. 2.2; the polynomial whose means over the
                              two cells on each side of the face equal their values, only the
                              cells that exist next to a wall; on any widths in x, y and z:
                              per-face weight tables, mr_host_face_weights) */
  int32_t step_method;     /* how step sequences run: 0 = chosen by the library, 1 = the fused
                              line solver (one kernel per step), 2 = column sweeps (see
                              mr_scalar_steps; x and y periodic with uniform widths, z_explicit 0,
                              face order 2 only) */
  int32_t sweep_tile;      /* tile of the column sweeps: 0 = chosen from nx by the library,
                              1 = 256 x 4 columns (FP64 only), 2 = 192 x 4, 3 = 128 x 8,
                              4 = 64 x 16; results are the same for every tile (MR_EINVAL
                              otherwise) */
} mr_desc;

/* Nusselt summary of one scalar field (Eq. 22, instantaneous). */
typedef struct {
  double nu_bot;      /* bottom plate: -<(theta_0 - T_bot)/(hz_0/2)> */
  double nu_top;      /* top plate: -<(T_top - theta_{nz-1})/(hz_{nz-1}/2)> */
  double nu_vol;      /* sum_k h_k Nu_k, h_k the distance between the cell centres around face k */
  double nu_paper;    /* mean of Nu_k over the nz-1 interior faces */
  double mean_theta;  /* volume-weighted mean scalar */
} mr_nu;

/* ---------------------------------------------------------------- setup */

/* Validate the descriptor, build the grid tables on the host (refinement
 * matrices R = A_s A^-1 per coarse cell and axis, Eq. 19; tridiagonal factors
 * of the implicit z diffusion for the three step types) and upload them to the
 * current HIP device.  R depends on the grid only and is computed once
 * (Sec. 3.2).  Fails with MR_EINVAL on: a non-positive or inconsistent size,
 * refinement factor < 1, fewer than 3 coarse cells on an axis with factor > 1,
 * non-increasing faces, dt <= 0, Ra*Pr <= 0, an unknown wall condition or
 * precision, an explicit x/y diffusion number
 * 2 dt kappa (4/hx_min^2 + 4/hy_min^2) above 1, or column sweeps asked for
 * where they do not apply.  Fails with MR_ESHAPE on sizes
 * the kernels cannot address: an axis of more than 2^20 dense cells,
 * (N_z + 1) N_x N_y above 2^31 - 1 values, one z level (N_x N_y values of the
 * context's precision) above 2^32 - 1 bytes, or more than 640 z levels (the
 * line solver's 16 chunks of at most 40 levels) unless column sweeps apply
 * (x and y periodic with uniform widths, z_explicit 0, face order 2) and the
 * line solver is not asked for: such columns are stepped by column sweeps (see
 * mr_scalar_steps), and mr_adjoint_seed and mr_scalar_step_backward return
 * MR_ESHAPE for them.  *out is set only on success. */
int mr_init(const mr_desc* desc, mr_ctx** out);

/* Free the context and its device tables.  NULL is accepted. */
int mr_destroy(mr_ctx* ctx);

/* --------------------------------------------------------- refinement (Sec. 3.2) */

/* Coarse (U, V, W) -> dense (u, v, w).  Stages z, then y, then x: split the
 * outer coarse face velocities with R (Eq. 19), then march each inner face
 * from zero net outward flux of the sub-cell below it (Fig. 5a).  Every dense
 * cell's net flux is the coarse cell's divergence for the last sub-cell of
 * each coarse cell and zero (to rounding) for the others.  Inputs are not
 * modified; outputs must not alias inputs. */
int mr_interpolate_velocity(mr_ctx* ctx, const void* U, const void* V, const void* W,
                            void* u, void* v, void* w, void* stream);

/* Transpose of mr_interpolate_velocity: (gu, gv, gw) on the dense faces ->
 * (gU, gV, gW) on the coarse faces, overwriting gU, gV, gW.  Every coarse face
 * array is covered, the wall W planes included. */
int mr_interpolate_velocity_backward(mr_ctx* ctx, const void* gu, const void* gv, const void* gw,
                                     void* gU, void* gV, void* gW, void* stream);

/* Discrete divergence check (Sec. 3.2 reports ~1e-17 in double precision).
 * Writes to device memory dev_out[0] = max over dense cells of |net outward
 * volume flux|, dev_out[1] = max over cells of |net flux| / (sum of |face
 * fluxes| of the cell) (0 for a cell with no flux).  Always computed in double. */
int mr_divergence(mr_ctx* ctx, const void* u, const void* v, const void* w,
                  double* dev_out, void* stream);

/* ------------------------------------------------------------ scalar step */

/* theta^{n+1} from theta^{n-1} and theta^n (Eqs. 6-7, z diffusion implicit):
 *   (I - (1-w) tau kappa Lz0) theta^{n+1} = a_p theta^{n-1} + a_c theta^n
 *        + tau [C_u(theta^n) + kappa Lh(theta^lag) + w kappa Lz0(theta^lag) + kappa b_z]
 * with C_u the central-flux advection (face value = mean of the two cells, no
 * flux through the walls), Lh the x/y diffusion, Lz0 the z diffusion without
 * the wall values, b_z the Dirichlet wall source, w = desc->z_explicit,
 * and per step type
 *   n = 0 (start-up):          tau = dt,     a_p = 0,   a_c = 1,   lag = n
 *   (n+1) mod N_p = 0, n >= 1: tau = 1.5 dt, a_p = 1/2, a_c = 1/2, lag = n-1
 *   otherwise (leapfrog):      tau = 2 dt,   a_p = 1,   a_c = 0,   lag = n-1.
 * th_prev is not read at n = 0 (may be NULL).  th_next must not alias th_prev or
 * th_cur: callers rotate three buffers.  The tridiagonal elimination runs in
 * double for both precisions.  One fused line-solver kernel, or with
 * step_method 2 (and on columns taller than 640 levels) one column sweep and
 * its back substitution (see mr_scalar_steps). */
int mr_scalar_step(mr_ctx* ctx, int64_t n, const void* th_prev, const void* th_cur, void* th_next,
                   const void* u, const void* v, const void* w, void* stream);

/* Steps n0 .. n0+count-1 in one call: outs[q] (device, count pointers in a
 * host array) receives theta^{n0+q+1}.  th_prev = theta^{n0-1} (not read at
 * n0 = 0, may be NULL), th_cur = theta^{n0}.  Every output must differ from
 * the two levels before it (outs[0] from th_cur and th_prev, outs[1] from
 * outs[0] and th_cur, outs[q] from outs[q-1] and outs[q-2]): a ring of three
 * buffers satisfies this.  Results equal count calls of mr_scalar_step to
 * rounding.
 * With step_method 2, and with step_method 0 on grids whose sweep tiles keep
 * the GPU full (at least 16 wavefronts per CU, rounds of tiles at least 3/4
 * full: 576 x 576 and 1024 x 1024 columns, not 256 x 256) or columns too tall
 * for the line solver (x and y periodic with uniform widths and the plain
 * method in both cases), the steps run as column sweeps: each kernel back-substitutes the previous step's implicit solve
 * while it eliminates its own in the other z direction, so a cell moves
 * 7 values per step instead of the 6 of one fused step but no column is held
 * whole on chip.  These sweeps use two elimination fields of the context
 * (nz*ny*nx values each), allocated on first use and kept until mr_destroy;
 * MR_EHIP (hipErrorOutOfMemory) if that allocation fails.  In the FP32 tier
 * the elimination runs in double and its values are stored in float. */
int mr_scalar_steps(mr_ctx* ctx, int64_t n0, int32_t count, const void* th_prev, const void* th_cur,
                    void* const* outs, const void* u, const void* v, const void* w, void* stream);

/* ------------------------------------------------------------ adjoint */

/* mu^n = (I - tau_n kappa Lz)^-T lam: the transposed implicit solve of step n.
 * Seeds the reverse sweep with lam = dL/dtheta^{n+1}.  mu_out must not alias lam.
 * On columns taller than the line solver's, a solve column by column (its
 * elimination values pass through mu_out). */
int mr_adjoint_seed(mr_ctx* ctx, int64_t n, const void* lam, void* mu_out, void* stream);

/* One fused reverse step.  With mu^m = (I - tau_m kappa Lz)^-T dL/dtheta^{m+1}:
 *   lam^n = [mu_next != NULL] (a_p(n+1) mu^{n+1} + tau_{n+1} kappa Lh^T mu^{n+1})
 *         + a_c(n) mu^n + tau_n C_u^T mu^n + [lam_add != NULL] lam_add
 * is the complete dL/dtheta^n (lam_add: any direct loss gradient on theta^n).
 * n >= 1: out = mu^{n-1} = (I - tau_{n-1} kappa Lz)^-T lam^n.
 * n == 0: out = dL/dtheta^0 = lam^0 + tau_0 kappa Lh^T mu^0 (the start-up step
 *         reads theta^0 for its diffusion too).
 * out must not alias the inputs.  Velocity gradients are accumulated
 * separately by mr_velocity_grad.  On columns taller than the line solver's
 * the step runs as a column sweep (n >= 1: a sweep and a back substitution;
 * n = 0: one pass with no solve); lam_add is then refused (MR_ESHAPE). */
int mr_scalar_step_backward(mr_ctx* ctx, int64_t n, const void* mu_next, const void* mu_cur,
                            const void* lam_add, void* out,
                            const void* u, const void* v, const void* w, void* stream);

/* Reverse steps n0, n0-1, .., n0-count+1 (Eqs. 5-7 transposed, the same mu
 * form as mr_scalar_step_backward, without lam_add), all with n >= 1, in one
 * call: outs[q] (device, count pointers in a host array) receives
 * mu^{n0-q-1}, what mr_scalar_step_backward returns for step n0-q.
 * mu_next = mu^{n0+1} (NULL when there is no step n0+1), mu_cur = mu^{n0}.
 * Every output must differ from the two levels before it (outs[0] from
 * mu_cur and mu_next, outs[1] from outs[0] and mu_cur, outs[q] from outs[q-1]
 * and outs[q-2]).  Results equal count calls of mr_scalar_step_backward to
 * rounding.  Where the context runs step sequences as column sweeps
 * (mr_get_step_method 2) the reverse steps run as column sweeps too: each
 * kernel back-substitutes the previous reverse step's transposed solve while
 * it eliminates its own the other way (7 values per cell and step), with the
 * same two elimination fields; columns taller than the line solver's are then
 * accepted.  The reverse step n = 0 (the start-up step's, whose output is the
 * adjoint of theta^0 itself) is not part of a sequence: call
 * mr_scalar_step_backward for it.  MR_EINVAL for count < 1, n0-count+1 < 1,
 * NULL pointers or an output equal to one of the two levels before it;
 * MR_ESHAPE for tall columns on the line-solver path. */
int mr_scalar_steps_backward(mr_ctx* ctx, int64_t n0, int32_t count, const void* mu_next,
                             const void* mu_cur, void* const* outs, const void* u, const void* v,
                             const void* w, void* stream);

/* Accumulate the dense face-velocity gradient of `count` steps (count <= 16):
 *   g_f += sum_s tau_{n_s} A_f (theta_L + theta_R)/2 (mu_R/V_R - mu_L/V_L)
 * on every dense face f with cells L and R (zero on the z walls), where
 * theta = thetas[s] = theta^{n_s} and mu = mus[s] = mu^{n_s}.  steps, thetas
 * and mus are host arrays (thetas/mus hold device pointers).  gu, gv, gw are
 * read and written (+=). */
int mr_velocity_grad(mr_ctx* ctx, int32_t count, const int64_t* steps,
                     const void* const* thetas, const void* const* mus,
                     void* gu, void* gv, void* gw, void* stream);

/* ------------------------------------------------------------ diagnostics */

/* Heat-flux Nusselt number on every dense z face (Eq. 22):
 *   Nu_k = (Ra Pr)^(1/2) <w_k (theta_{k-1} + theta_k)/2> - <(theta_k - theta_{k-1})/dc_k>
 * with <.> the area-weighted x/y mean and dc_k the centre distance (half a
 * cell at the plates, where the wall value replaces the missing cell).
 * dev_profile (device, nz+6 doubles) receives Nu_0..Nu_nz followed by
 * nu_bot, nu_top, nu_vol, nu_paper, mean_theta.  Sums are compensated
 * (double-double) with a fixed reduction order, so results are bitwise
 * reproducible.  If host_out is not NULL the summary is also copied there
 * (the call then waits for the stream) and MR_ENONFINITE is returned when any
 * value is NaN or Inf. */
int mr_nusselt(mr_ctx* ctx, const void* theta, const void* w, double* dev_profile,
               mr_nu* host_out, void* stream);

/* mr_nusselt for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results (bit for bit) as mr_nusselt with host_out NULL, with
 * the reduction partials in a fixed device array of the library (3.15 MB per
 * GPU, set up by mr_init on its device and held until the process ends)
 * instead of the context's lazily allocated buffer.  Allocates nothing.
 * Limit: nz <= 1024 (MR_ESHAPE beyond).  Every call on one GPU shares that
 * array, so calls that overlap on one GPU (other streams, other threads, other
 * contexts of the same device) race and must be serialised by the caller;
 * each call rewrites every partial it reads, so nothing needs clearing between
 * calls.  Asynchronous on the stream; no host summary (read dev_profile's last
 * five values). */
int mr_nusselt_noalloc(mr_ctx* ctx, const void* theta, const void* w, double* dev_profile,
                       void* stream);

/* Dissipation Nusselt number (Sec. 4.1, Eq. 23): Nu_T = eps_T (Ra Pr)^(1/2) with
 * eps_T = kappa <|grad theta|^2>_V, the volume mean of the squared gradient
 * summed face by face: each face adds its squared difference quotient times
 * its dual volume (face area times the centre distance across it); a
 * Dirichlet plate uses the wall value at half a cell, an adiabatic plate adds
 * nothing.  dev_out (device, 4 doubles) receives {Nu_T, <theta_x^2>,
 * <theta_y^2>, <theta_z^2>} (volume means of the three squared components).
 * Compensated sums in a fixed order.  host_out (4 doubles or NULL) as for
 * mr_nusselt: the call then waits and reports MR_ENONFINITE for NaN/Inf. */
int mr_thermal_dissipation(mr_ctx* ctx, const void* theta, double* dev_out, double* host_out,
                           void* stream);

/* ------------------------------------------------- inter-grid steps (Secs. 3.3-3.4) */

/* Coarse velocity at fraction s = i/mt of a coarse step, refined to the dense
 * faces (temporal strategy, Sec. 3.4, Eq. 21, read as the linear interpolation
 * between the two coarse levels): refines (1 - s)(U0, V0, W0) + s (U1, V1, W1)
 * as mr_interpolate_velocity does, the blend formed first in a coarse buffer
 * of the context (none at s = 0 or 1).  0 <= i <= mt, mt >= 1; i = mt gives exactly the refinement of
 * (U1, V1, W1), i = 0 that of (U0, V0, W0).  Two divergence-free levels give a
 * divergence-free result (to rounding).  Outputs must not alias inputs. */
int mr_interpolate_velocity_time(mr_ctx* ctx, const void* U0, const void* V0, const void* W0,
                                 const void* U1, const void* V1, const void* W1, int64_t i,
                                 int64_t mt, void* u, void* v, void* w, void* stream);

/* Upscale integration of the scalar (Sec. 3.3, Eq. 20, read as the
 * volume-weighted mean of the cell averages): theta_c[K][J][I] = (sum over the
 * mx*my*mz sub-cells of theta * hx*hy*hz) / (coarse cell volume).
 * theta [nz][ny][nx] -> theta_c [ncz][ncy][ncx], the context's element type;
 * sums in double.  theta_c must not alias theta. */
int mr_integrate_scalar(mr_ctx* ctx, const void* theta, void* theta_c, void* stream);

/* One coarse step of the multiple-resolution loop for the scalar (Fig. 6):
 * for i = 1..mt, refine the coarse velocity at fraction (i-1)/mt into (u, v, w)
 * (as mr_interpolate_velocity_time: the velocity at the start of sub-step i,
 * the time level whose scalar the step advects, Eqs. 5-7) and take scalar
 * step n0 + i - 1 (as
 * mr_scalar_step; the context's dt is the scalar step, i.e. the coarse step
 * divided by mt); then, if theta_c is not NULL, integrate the newest scalar
 * into theta_c (as mr_integrate_scalar).
 * ring: host array of three distinct device scalar buffers.  On entry
 * ring[*cur] holds theta^{n0} and, for n0 > 0, ring[*prev] holds theta^{n0-1}
 * (at n0 = 0, *prev is ignored and may equal *cur).  On return *prev and *cur
 * index theta^{n0+mt-1} and theta^{n0+mt}.  u, v, w are dense velocity
 * buffers the call overwrites.  n0 >= 0, mt >= 1.  All work is enqueued on
 * the stream; nothing is allocated beyond the context's refinement buffers. */
int mr_coarse_step(mr_ctx* ctx, int64_t n0, int32_t mt, const void* U0, const void* V0,
                   const void* W0, const void* U1, const void* V1, const void* W1, void* u, void* v,
                   void* w, void* const* ring, int32_t* prev, int32_t* cur, void* theta_c,
                   void* stream);

/* ------------------------------------------------------------ utilities */

/* Plain device copy of nbytes (multiple of 16, 16-byte aligned pointers) with
 * the library's own streaming kernel: the bandwidth reference for profiles. */
int mr_copy_probe(const void* src, void* dst, int64_t nbytes, void* stream);

/* Host-only inspection of the tables mr_init would build (no GPU needed).
 * axis 0/1/2 = x/y/z: R_out receives nc*m*3 doubles (R of every coarse cell,
 * row-major [cell][sub][stencil]) and start_out nc int32 (first stencil cell,
 * may be -1 on a periodic axis).  Either pointer may be NULL. */
int mr_host_refinement_table(const mr_desc* desc, int32_t axis, double* R_out, int32_t* start_out);

/* Host-only: the tridiagonal (sub, diag, sup) of I - (1-w) tau_n kappa Lz0 and
 * the wall source b_z (each nz doubles, any may be NULL) used by step n, and
 * *tau_out (w = desc->z_explicit). */
int mr_host_z_system(const mr_desc* desc, int64_t n, double* sub, double* diag, double* sup,
                     double* bz, double* tau_out);

/* Host-only: the fourth-order face weights of the z axis (Sec. 2.2) that the
 * step uses with face_order 4: w_out receives (nz+1)*4 doubles, face f's
 * weights for the cells f-2, f-1, f, f+1 (zero for the wall faces and for
 * cells beyond a wall). */
int mr_host_z_face_weights(const mr_desc* desc, double* w_out);

/* Host-only: the fourth-order face weights of one axis (0 = x, 1 = y, 2 = z;
 * Sec. 2.2) that the step and the velocity gradient use with face_order 4:
 * w_out receives (n+1)*4 doubles for the axis's n dense cells, face f's
 * weights for the cells f-2, f-1, f, f+1.  A walled axis (z always) has zero
 * rows for its wall faces and zero weights for cells beyond a wall; on a
 * periodic axis the stencil wraps around (face f is the one between cells f-1
 * and f, face 0 between cell n-1 and cell 0) and row n repeats row 0.
 * MR_EINVAL for another axis. */
int mr_host_face_weights(const mr_desc* desc, int32_t axis, double* w_out);

/* The method mr_scalar_steps uses on this context: 1 = the fused line
 * solver, 2 = column sweeps. */
int mr_get_step_method(const mr_ctx* ctx, int32_t* method);

/* Dense sizes of a context and its precision. */
int mr_get_dims(const mr_ctx* ctx, int32_t* nx, int32_t* ny, int32_t* nz, int32_t* precision);

const char* mr_status_string(int status);
int mr_last_hip_error(const mr_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* MRSCALAR_H */
