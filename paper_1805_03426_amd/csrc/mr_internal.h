// Internal declarations shared by the host API and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "mrscalar.h"

namespace mr {

// Step types of the Euler-leapfrog integrator with periodic averaging.
enum StepKind { KIND_STARTUP = 0, KIND_LEAPFROG = 1, KIND_AVERAGE = 2, NKINDS = 3 };

// Largest number of z chunks (one wavefront each) of the line solver, and the
// chunk lengths the step kernels are instantiated for.
constexpr int kMaxChunks = 16;
constexpr int kChunkLens[] = {32, 36, 40};
constexpr int kWave = 64;
// Column-sweep tile shapes: segments of 64 x columns by rows, one wavefront
// per segment and row.  mr_init picks one per context (mr_ctx::sweep_shape).
struct SweepShape {
  int segs, rows;
};
constexpr int kSweepShapes = 4;
constexpr SweepShape kSweepShape[kSweepShapes] = {{4, 4}, {3, 4}, {2, 8}, {1, 16}};
int sweep_pick_shape(int nx, bool fp64);

// Grid tables of one precision (device pointers into the context's table block).
template <typename T>
struct Geom {
  const T* hx;    // [nx] dense widths
  const T* ihx;   // [nx] 1/hx
  const T* idxc;  // [nx] 1/(xc_i - xc_{i-1}) across face i (periodic)
  const T* hy;
  const T* ihy;
  const T* idyc;
  const T* hz;    // [nz]
  const T* ihz;   // [nz]
  const T* iHX;   // [ncx] 1/coarse width
  const T* iHY;   // [ncy]
  const T* Rx;    // [ncx][mx][3] refinement matrices (Eq. 19)
  const T* Ry;    // [ncy][my][3]
  const T* Rz;    // [ncz][mz][3]
  const int* sx;  // [ncx][3] stencil cells (wrapped)
  const int* sy;  // [ncy][3]
  const int* sz;  // [ncz][3]
  const T* zlo;   // [nch*L] 1 where z level k has an interior face below (0 < k < nz), else 0
  const T* zhi;   // [nch*L] 1 where z level k has an interior face above (k < nz-1), else 0
  // Lz0 (vertical diffusion per unit volume without the Dirichlet wall source):
  // row k = lzl[k] level k-1 + lzd[k] level k + lzh[k] level k+1; its transpose
  // has lztl[k] = lzh[k-1] and lzth[k] = lzl[k+1] off the diagonal.  [nch*L],
  // zero on the padding rows of the line solver.
  const T* lzl;
  const T* lzd;
  const T* lzh;
  const T* lztl;
  const T* lzth;
  // fourth-order face values in z: c4z[4 f + s] weights face f's value on the
  // cells f-2+s ([nch*L + 1][4], zero rows for the walls and the padding);
  // c4zt[4 k + s] is cell k's weight in face k-1+s ([nch*L][4], the transpose)
  const T* c4z;
  const T* c4zt;
  // fourth-order face values in x and y: c4x[4 f + s] weights face f's value
  // on the cells f-2+s (wrapped on a periodic axis), [nx+1][4]; zero rows for
  // the wall faces of a walled axis, and face nx repeats face 0 on a periodic one
  const T* c4x;
  const T* c4y;
};

// Factors of one tridiagonal system (I - tau kappa Lz or its transpose) for
// the chunked line solver: Thomas factors and the chunk coupling vectors.
// Per-level tables hold nch*L rows; rows >= nz are decoupled identity rows.
struct ZSys {
  const double* m;   // 1/(diag_k - sub_k cp_{k-1})
  const double* a;   // -sub_k m_k
  const double* cp;  // sup_k m_k
  const double* G;   // response of x_k to the value entering its chunk from below
  const double* B;   // response of x_k to the value entering its chunk from above
  const double* Fe;  // [nch] product of a over each chunk
  const double* Gs;  // [nch] G at each chunk start
  const double* Bs;  // [nch] B at each chunk start
  const double* tkb; // tau kappa b_z (wall source); zeros for the transpose
};

// Factors of the implicit z system of one step type for the column-sweep
// kernels, both elimination directions (nz rows each):
//   upward:   e_k = up_m_k (r_k + tkb_k) + up_a_k e_{k-1}, then downward
//             x_k = e_k - up_cb_k x_{k+1};
//   downward: e_k = dn_m_k (r_k + tkb_k) + dn_a_k e_{k+1}, then upward
//             x_k = e_k - dn_cb_k x_{k-1}.
struct SweepSys {
  const double* up_m;
  const double* up_a;
  const double* up_cb;
  const double* dn_m;
  const double* dn_a;
  const double* dn_cb;
  const double* tkb;
};

}  // namespace mr

struct mr_ctx {
  int nx, ny, nz, ncx, ncy, ncz, mx, my, mz;
  int precision;
  double kappa, dt, ra, pr, t_bot, t_top;
  int bc_bot, bc_top, n_avg;
  int wx, wy;                      // x / y bounded by adiabatic no-slip walls (else periodic)
  int uniform_xy;                  // periodic x and y of equal widths (to 1e-13): uniform-width step kernels
  double uhx, uhy;                 // 1/h of the x and y widths (used by those kernels)
  double z_explicit;               // w: share of the z diffusion explicit on the lagged level
  int face_order;                  // face value of the advected scalar: 2 or 4
  int device;
  int last_err;
  int L, nch;                      // z chunk length and count of the line solver (0: columns too
                                   // tall for it; only the column-sweep step runs)
  double atot;                     // total horizontal area
  double vtot;                     // domain volume (atot times the height)
  double tau[mr::NKINDS];
  void* tables;                    // one device block with every table
  mr::Geom<double> g64;
  mr::Geom<float> g32;
  mr::ZSys zf[mr::NKINDS];         // forward systems per step kind
  mr::ZSys zt[mr::NKINDS];         // transposed systems per step kind
  mr::SweepSys sw[mr::NKINDS];     // column-sweep factors per step kind
  mr::SweepSys swt[mr::NKINDS];    // the same for the transposed systems (reverse steps)
  mr::SweepSys swid;               // identity factors (the start-up step's reverse: no solve)
  int sweep_shape;                 // column-sweep tile shape (index into kSweepShape)
  int sweep_pref;                  // run step sequences as column sweeps
  int sweep_single;                // run single steps as a column sweep and its back substitution
  void* sweep_e[2];                // elimination values of two consecutive sweep steps (lazy)
  const double* areaw;             // [ny] hy_j (area = hx_i * hy_j, built in kernel)
  const double* hx64;              // [nx]
  const double* dcz;               // [nz+1] centre distances across z faces (wall: half cell)
  const double* hz64;              // [nz]
  void* interp_tmp;                // forward refinement intermediates (lazy)
  size_t interp_tmp_bytes;
  void* interp_bwd_tmp;            // transposed refinement intermediates (lazy)
  size_t interp_bwd_tmp_bytes;
  double* red;                     // reduction partials
  size_t red_bytes;
};

// Launchers (return hipError_t of the launch).
namespace mr {
hipError_t launch_refine(mr_ctx* c, const void* U, const void* V, const void* W, void* u, void* v,
                         void* w, hipStream_t s);
hipError_t launch_refine_transpose(mr_ctx* c, const void* gu, const void* gv, const void* gw,
                                   void* gU, void* gV, void* gW, hipStream_t s);
hipError_t launch_step(mr_ctx* c, int64_t n, const void* thp, const void* thc, void* thn,
                       const void* u, const void* v, const void* w, hipStream_t s);
hipError_t launch_seed(mr_ctx* c, int64_t n, const void* lam, void* mu, hipStream_t s);
hipError_t launch_step_backward(mr_ctx* c, int64_t n, const void* mun, const void* muc,
                                const void* lam_add, void* out, const void* u, const void* v,
                                const void* w, hipStream_t s);
hipError_t launch_velocity_grad(mr_ctx* c, int count, const int64_t* steps,
                                const void* const* thetas, const void* const* mus, void* gu,
                                void* gv, void* gw, hipStream_t s);
hipError_t launch_divergence(mr_ctx* c, const void* u, const void* v, const void* w, double* out,
                             hipStream_t s);
hipError_t launch_nusselt(mr_ctx* c, const void* th, const void* w, double* prof, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, int64_t nbytes, hipStream_t s);
hipError_t launch_refine_time(mr_ctx* c, const void* U0, const void* V0, const void* W0,
                              const void* U1, const void* V1, const void* W1, double frac, void* u,
                              void* v, void* w, hipStream_t s);
hipError_t launch_integrate(mr_ctx* c, const void* th, void* tc, hipStream_t s);
hipError_t launch_dissipation(mr_ctx* c, const void* th, double* out, hipStream_t s);
// Column-sweep steps n0 .. n0+count-1 (outs[q] receives theta^{n0+q+1}).
// One sweep kernel per step: step n0 + q (q = 0 reads theta^{n0} from src0 and
// writes no scalar; q > 0 writes theta^{n0+q} into th_out), then one back
// substitution of the last step into out.
bool sweep_supported(const mr_ctx* c);
hipError_t launch_sweep_step(mr_ctx* c, int64_t n0, int q, const void* lag, const void* src0,
                             void* th_out, const void* u, const void* v, const void* w, hipStream_t s);
hipError_t launch_sweep_finish(mr_ctx* c, int64_t n0, int count, void* out, hipStream_t s);
hipError_t launch_sweep_steps(mr_ctx* c, int64_t n0, int count, const void* thp, const void* thc,
                              void* const* outs, const void* u, const void* v, const void* w,
                              hipStream_t s);
// Column-sweep reverse steps n0, n0-1, .., n0-count+1 (all >= 1): outs[q]
// receives mu^{n0-q-1}; mu_next = mu^{n0+1} or null after the last step.
hipError_t launch_sweep_bwd_steps(mr_ctx* c, int64_t n0, int count, const void* mu_next, const void* mu_cur,
                                  void* const* outs, const void* u, const void* v, const void* w,
                                  hipStream_t s);
// The start-up step's reverse (out = dL/dtheta^0) and the seed solve, for
// columns the line solver cannot hold.
hipError_t launch_sweep_bwd0(mr_ctx* c, const void* mu_next, const void* mu_cur, void* out, const void* u,
                             const void* v, const void* w, hipStream_t s);
hipError_t launch_sweep_seed(mr_ctx* c, int64_t n, const void* lam, void* out, hipStream_t s);
// Grows the context's reduction scratch to at least `bytes`.
hipError_t ensure_red(mr_ctx* c, size_t bytes);
// The fixed device memory of the allocation-free Nusselt entry point: looks up
// its address on `device` (the current device) once per device.
hipError_t scratch_init(int device);
// mr_nusselt's kernels on that fixed memory (status code; allocates nothing).
int nusselt_fixed(mr_ctx* c, const void* th, const void* w, double* prof, hipStream_t s);

// Double-double (error-free two-sum) accumulation for compensated reductions.
struct DD {
  double s, c;
};

__device__ __forceinline__ DD dd_add(DD a, double b) {
  const double t = a.s + b;
  const double bp = t - a.s;
  const double e = (a.s - (t - bp)) + (b - bp);
  return {t, a.c + e};
}

__device__ __forceinline__ DD dd_merge(DD a, DD b) {
  DD r = dd_add(a, b.s);
  r.c += b.c;
  return r;
}

__device__ __forceinline__ DD wave_sum(DD v) {
  for (int off = kWave / 2; off > 0; off >>= 1) {
    DD o{__shfl_down(v.s, off, kWave), __shfl_down(v.c, off, kWave)};
    v = dd_merge(v, o);
  }
  return v;
}

// Step-type bookkeeping shared by the host API and the launchers.
inline int step_kind(int64_t n, int n_avg) {
  if (n == 0) return KIND_STARTUP;
  if (n_avg > 0 && (n + 1) % n_avg == 0) return KIND_AVERAGE;
  return KIND_LEAPFROG;
}
inline double alpha_prev(int kind) { return kind == KIND_STARTUP ? 0.0 : (kind == KIND_AVERAGE ? 0.5 : 1.0); }
inline double alpha_cur(int kind) { return kind == KIND_STARTUP ? 1.0 : (kind == KIND_AVERAGE ? 0.5 : 0.0); }

// XCD-aware tile order: the hardware deals consecutive workgroups round-robin
// to the 8 XCDs; this remaps them so that each XCD walks a contiguous range of
// tiles (neighbouring rows share that XCD's L2).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int full = (nblocks / kXcd) * kXcd;
  if (bid >= full) return bid;
  const int per = full / kXcd;
  return (bid % kXcd) * per + bid / kXcd;
}
}  // namespace mr
