// Scalar step entry points: the fused forward step (Eqs. 5-7 with the z
// diffusion implicit), its fused reverse step, the transposed solve that seeds
// the reverse sweep (all three on the line kernel of line_kernel.h), and the
// velocity-gradient accumulation.
#include "line_kernel.h"

namespace mr {
namespace line {
// The forward and reverse variants of the line kernel are instantiated in
// k_line_fwd.hip, k_line_bwd64.hip, k_line_bwd32.hip and k_line_bwd0.hip
// (translation units of their own, so that they compile in parallel); the
// seed solve here.
extern template hipError_t launch_line<double, FWD>(mr_ctx*, LineArgs<double>, hipStream_t);
extern template hipError_t launch_line<float, FWD>(mr_ctx*, LineArgs<float>, hipStream_t);
extern template hipError_t launch_line<double, BWD>(mr_ctx*, LineArgs<double>, hipStream_t);
extern template hipError_t launch_line<float, BWD>(mr_ctx*, LineArgs<float>, hipStream_t);
extern template hipError_t launch_line<double, BWD0>(mr_ctx*, LineArgs<double>, hipStream_t);
extern template hipError_t launch_line<float, BWD0>(mr_ctx*, LineArgs<float>, hipStream_t);
}  // namespace line

namespace {
using namespace line;

template <typename T>
LineArgs<T> base_args(mr_ctx* c, const Geom<T>& g) {
  LineArgs<T> a;
  ::memset((void*)&a, 0, sizeof(a));
  a.g = g;
  a.nx = c->nx;
  a.ny = c->ny;
  a.nz = c->nz;
  a.nch = c->nch;
  a.wx = c->wx;
  a.wy = c->wy;
  return a;
}

template <typename T>
hipError_t step_t(mr_ctx* c, const Geom<T>& g, int64_t n, const void* thp, const void* thc,
                  void* thn, const void* u, const void* v, const void* w, hipStream_t s) {
  const int kind = step_kind(n, c->n_avg);
  LineArgs<T> a = base_args<T>(c, g);
  a.a0 = (const T*)thp;
  a.a1 = (const T*)thc;
  a.u = (const T*)u;
  a.v = (const T*)v;
  a.w = (const T*)w;
  a.out = (T*)thn;
  a.z = c->zf[kind];
  a.ap = (T)alpha_prev(kind);
  a.ac = (T)alpha_cur(kind);
  a.tau = (T)c->tau[kind];
  a.tk = (T)(c->tau[kind] * c->kappa);
  a.tkw = (T)(c->tau[kind] * c->kappa * c->z_explicit);
  return launch_line<T, FWD>(c, a, s);
}

template <typename T>
hipError_t seed_t(mr_ctx* c, const Geom<T>& g, int64_t n, const void* lam, void* mu, hipStream_t s) {
  LineArgs<T> a = base_args<T>(c, g);
  a.a0 = (const T*)lam;
  a.out = (T*)mu;
  a.z = c->zt[step_kind(n, c->n_avg)];
  return launch_line<T, SEED>(c, a, s);
}

template <typename T>
hipError_t bwd_t(mr_ctx* c, const Geom<T>& g, int64_t n, const void* mun, const void* muc,
                 const void* lam_add, void* out, const void* u, const void* v, const void* w,
                 hipStream_t s) {
  const int kind = step_kind(n, c->n_avg);
  LineArgs<T> a = base_args<T>(c, g);
  // absent inputs are replaced by mu^n with zero weights (no branches in the kernel)
  a.a0 = (const T*)muc;
  a.a1 = (const T*)(mun ? mun : muc);
  a.a2 = (const T*)(lam_add ? lam_add : muc);
  a.s2 = lam_add ? T(1) : T(0);
  a.u = (const T*)u;
  a.v = (const T*)v;
  a.w = (const T*)w;
  a.out = (T*)out;
  a.ac = (T)alpha_cur(kind);
  a.tau = (T)c->tau[kind];
  a.tk = (T)(c->tau[kind] * c->kappa);
  a.tkw = (T)(c->tau[kind] * c->kappa * c->z_explicit);
  if (mun) {
    const int k1 = step_kind(n + 1, c->n_avg);
    a.ap1 = (T)alpha_prev(k1);
    a.tk1 = (T)(c->tau[k1] * c->kappa);
    a.tkw1 = (T)(c->tau[k1] * c->kappa * c->z_explicit);
  }
  if (n == 0) return launch_line<T, BWD0>(c, a, s);
  a.z = c->zt[step_kind(n - 1, c->n_avg)];
  return launch_line<T, BWD>(c, a, s);
}

// ------------------------------------------------------- velocity gradient
constexpr int kMaxGradSteps = 16;

template <typename T>
struct GradArgs {
  const T* th[kMaxGradSteps];
  const T* mu[kMaxGradSteps];
  T tau[kMaxGradSteps];
  int count;
  T* gu;
  T* gv;
  T* gw;
  Geom<T> g;
  int nx, ny, nz;
  int wx, wy;
};

// Velocity gradient: every dense cell (i, j, k) owns the faces on its low
// side (x-face i, y-face j and, for k >= 1, z-face k) and adds
// tau theta_f (mu_R/h_R - mu_L/h_L) for every step, theta_f the step's face
// value (the mean of the two cells, or the fourth-order value).
// Fourth-order faces: one thread per cell (grad_kernel).  The walls' z faces carry no advective
// flux, so their gradient stays as it is; a side-wall face (x-face 0 or
// y-face 0 of a walled axis) gets zero.
template <typename T, bool ORD4>
__global__ void __launch_bounds__(256) grad_kernel(GradArgs<T> A) {
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int nxy = nx * ny;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= nxy * nz) return;
  const int i = tid % nx;
  const int j = (tid / nx) % ny;
  const int k = tid / nxy;
  const int im = i == 0 ? nx - 1 : i - 1;
  const int jm = j == 0 ? ny - 1 : j - 1;
  const int row = k * nxy + j * nx;
  const T half = T(0.5);
  const T ihx = A.g.ihx[i], ihxm = A.g.ihx[im], ihy = A.g.ihy[j], ihym = A.g.ihy[jm];
  const T ihz = A.g.ihz[k], ihzm = k > 0 ? A.g.ihz[k - 1] : T(0);
  // fourth-order stencils: cells i-2 and i+1 (j-2, j+1; k-2, k+1) and the weights
  const bool wx = A.wx, wy = A.wy;
  const int im2 = wx ? max(i - 2, 0) : (i - 2 + 2 * nx) % nx, ip = wx ? min(i + 1, nx - 1) : (i + 1) % nx;
  const int jm2 = wy ? max(j - 2, 0) : (j - 2 + 2 * ny) % ny, jp = wy ? min(j + 1, ny - 1) : (j + 1) % ny;
  const int km2 = max(k - 2, 0), kp = min(k + 1, nz - 1);
  line::W4<T> wxf{}, wyf{};
  if constexpr (ORD4) wxf = line::face_w4<T>(A.g.c4x, i, nx, wx), wyf = line::face_w4<T>(A.g.c4y, j, ny, wy);
  const T* cz = A.g.c4z + 4 * k;
  T su = T(0), sv = T(0), sw = T(0);
  for (int s = 0; s < A.count; ++s) {
    const T* th = A.th[s];
    const T* mu = A.mu[s];
    const T tc = th[row + i], mc = mu[row + i];
    const T* lvl = th + k * nxy;
    T fx, fy, fz = T(0);
    if constexpr (ORD4) {
      fx = wxf.a * lvl[j * nx + im2] + wxf.b * lvl[j * nx + im] + wxf.c * tc + wxf.d * lvl[j * nx + ip];
      fy = wyf.a * lvl[jm2 * nx + i] + wyf.b * lvl[jm * nx + i] + wyf.c * tc + wyf.d * lvl[jp * nx + i];
      if (k > 0)
        fz = cz[0] * th[km2 * nxy + j * nx + i] + cz[1] * th[row - nxy + i] + cz[2] * tc +
             cz[3] * th[kp * nxy + j * nx + i];
    } else {
      fx = half * (lvl[j * nx + im] + tc);
      fy = half * (lvl[jm * nx + i] + tc);
      if (k > 0) fz = half * (th[row - nxy + i] + tc);
    }
    su += A.tau[s] * fx * (mc * ihx - mu[row + im] * ihxm);
    sv += A.tau[s] * fy * (mc * ihy - mu[k * nxy + jm * nx + i] * ihym);
    if (k > 0) sw += A.tau[s] * fz * (mc * ihz - mu[row - nxy + i] * ihzm);
  }
  if (A.wx && i == 0) su = T(0);
  if (A.wy && j == 0) sv = T(0);
  A.gu[row + i] += su;
  A.gv[row + i] += sv;
  if (k > 0) A.gw[row + i] += sw;
}

// Second-order faces: a workgroup of kGradRows wavefronts owns a tile of 64
// columns by kGradRows rows and walks a run of consecutive z segments of ZS
// levels.  For each segment and step in turn every wavefront loads theta and
// mu of its row on the segment's levels, the first wavefront also the row
// below the tile, and publishes them in LDS, where the wavefront of the next
// row finds its y neighbours: a row is read from memory once per step and
// segment (the y halo is one row in kGradRows).  The level below a segment is
// loaded for the first segment of the run and then carried in registers from
// the segment before (CARRY; without it, loaded for every segment).  The loads
// of a step are independent of each other, so they are all in flight
// together.  The column to the left comes from the lane beside it (lane 0
// loads it).  The LDS buffer alternates from step to step, one barrier per
// step.  Every step's contribution goes to per-level accumulators in
// registers; gu, gv, gw are updated once per level.
// Timed at 1024x1024x512 against 16 rows (one workgroup of 139 KB of LDS per
// CU): 8 rows, two workgroups per CU, were 7% faster in FP64 and level in FP32.
constexpr int kGradRows = 8;    // wavefronts (rows of 64 columns) per workgroup
// FP32 runs of 2 segments: 14.2 ms per call of 10 steps at 1024x1024x512,
// against 14.6 ms for 4 and 15.3 ms for 8 (more workgroups, shorter walks).
constexpr int kGradRun = 2;     // FP32: segments per workgroup
constexpr int kGradWaves = 4;   // wavefronts per SIMD to fit (128 VGPRs)

template <typename T, int KM, int ZS, bool CARRY>
__global__ void __launch_bounds__(64 * kGradRows, kGradWaves) grad_seg(GradArgs<T> A, int run) {
  __shared__ T lt[2][ZS][kGradRows + 1][kWave];   // theta rows by step parity, level, tile row + 1
  __shared__ T lm[2][ZS][kGradRows + 1][kWave];   // mu rows
  // the steps' field pointers and weights, read from LDS at every use so that
  // they do not stay live in scalar registers across the segment loop
  __shared__ const T* sptr[2][KM];
  __shared__ T stau[KM];
  if (threadIdx.x < KM && (int)threadIdx.x < A.count) {
    sptr[0][threadIdx.x] = A.th[threadIdx.x];
    sptr[1][threadIdx.x] = A.mu[threadIdx.x];
    stau[threadIdx.x] = A.tau[threadIdx.x];
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int r = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int ntx = (nx + kWave - 1) / kWave, nty = (ny + kGradRows - 1) / kGradRows;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = b % (ntx * nty);
  const int seg0 = b / (ntx * nty) * run;   // first segment of this workgroup's run
  const int xt = tile % ntx, jt = tile / ntx;
  const int i_raw = xt * kWave + lane, j_raw = jt * kGradRows + r;
  const bool act = i_raw < nx && j_raw < ny;
  const bool wx = A.wx, wy = A.wy;
  // lanes and rows past a ragged end read valid cells and store nothing
  const int i = i_raw % nx, j = j_raw % ny;
  const int im = i == 0 ? (wx ? 0 : nx - 1) : i - 1;
  const int jm = j == 0 ? (wy ? 0 : ny - 1) : j - 1;
  // the row below the tile (the first wavefront loads it; on a walled y axis
  // the tile at j = 0 takes its own first row: that face gets no gradient)
  const int j0 = jt * kGradRows;
  const int jh = j0 == 0 ? (wy ? 0 : ny - 1) : j0 - 1;
  const int nxy = nx * ny;
  constexpr unsigned sz = sizeof(T);
  const unsigned oc = (unsigned)(j * nx + i) * sz;
  const unsigned oxe = (unsigned)(j * nx + im) * sz;   // lane 0: its left column
  const unsigned oh = (unsigned)(jh * nx + i) * sz;
  const T half = T(0.5);
  const T ihx = A.g.ihx[i], ihxm = A.g.ihx[im], ihy = A.g.ihy[j], ihym = A.g.ihy[jm];
  const bool zu = wx && i == 0, zv = wy && j == 0;   // side-wall faces: no gradient
  auto at = [&](const T* f, int k, unsigned off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(f + (size_t)k * nxy) + off);
  };
  T cbt[CARRY ? KM : 1], cbm[CARRY ? KM : 1];   // each step's theta and mu on the level below the segment
  int p = 0;                                    // LDS buffer of the next step
  for (int sg = 0; sg < run; ++sg) {
    const int k0 = (seg0 + sg) * ZS;
    if (k0 >= nz) break;
    const bool below = !CARRY || sg == 0;       // load the level below (else carried)
    T ihz[ZS + 1];   // 1/hz of the level below the segment and of its levels (scalar loads)
#pragma unroll
    for (int z = 0; z <= ZS; ++z) {
      const int k = min(max(k0 + z - 1, 0), nz - 1);
      ihz[z] = ((const __attribute__((address_space(4))) T*)(A.g.ihz))[k];
    }
    T su[ZS], sv[ZS], sw[ZS];
#pragma unroll
    for (int z = 0; z < ZS; ++z) su[z] = sv[z] = sw[z] = T(0);
#pragma unroll
    for (int s = 0; s < KM; ++s) {
      if (s < A.count) {
        const T* th = sptr[0][s];
        const T* mu = sptr[1][s];
        const T tau = stau[s];
        // levels k0-1 .. k0+ZS-1 (clamped into the grid; the ones outside add nothing)
        T tc[ZS + 1], mc[ZS + 1], te[ZS], me[ZS], th_h[ZS], mu_h[ZS];
        if (below) {
          const int k = max(k0 - 1, 0);
          tc[0] = at(th, k, oc);
          mc[0] = at(mu, k, oc);
        } else if constexpr (CARRY) {
          tc[0] = cbt[s];
          mc[0] = cbm[s];
        }
#pragma unroll
        for (int z = 1; z <= ZS; ++z) {
          const int k = min(k0 + z - 1, nz - 1);
          tc[z] = at(th, k, oc);
          mc[z] = at(mu, k, oc);
          if (lane == 0) {
            te[z - 1] = at(th, k, oxe);
            me[z - 1] = at(mu, k, oxe);
          }
          if (r == 0) {
            th_h[z - 1] = at(th, k, oh);
            mu_h[z - 1] = at(mu, k, oh);
          }
        }
#pragma unroll
        for (int z = 0; z < ZS; ++z) {
          lt[p][z][r + 1][lane] = tc[z + 1];
          lm[p][z][r + 1][lane] = mc[z + 1];
          if (r == 0) {
            lt[p][z][0][lane] = th_h[z];
            lm[p][z][0][lane] = mu_h[z];
          }
        }
        __syncthreads();
#pragma unroll
        for (int z = 0; z < ZS; ++z) {
          const T t = tc[z + 1], m = mc[z + 1];
          const T tl = line::lane_shr(t), ml = line::lane_shr(m);
          const T txm = lane == 0 ? te[z] : tl, mxm = lane == 0 ? me[z] : ml;
          const T ty = lt[p][z][r][lane], my = lm[p][z][r][lane];
          su[z] += tau * (half * (txm + t)) * (m * ihx - mxm * ihxm);
          sv[z] += tau * (half * (ty + t)) * (m * ihy - my * ihym);
          sw[z] += tau * (half * (tc[z] + t)) * (m * ihz[z + 1] - mc[z] * ihz[z]);
        }
        if constexpr (CARRY) {
          cbt[s] = tc[ZS];
          cbm[s] = mc[ZS];
        }
        p ^= 1;
      }
    }
#pragma unroll
    for (int z = 0; z < ZS; ++z) {
      const int k = k0 + z;
      if (act && k < nz) {
        const size_t o = (size_t)k * nxy + (size_t)j * nx + i;
        A.gu[o] += zu ? T(0) : su[z];
        A.gv[o] += zv ? T(0) : sv[z];
        if (k > 0) A.gw[o] += sw[z];   // the bottom wall face carries no flux
      }
    }
  }
}

// Segments of 8 levels in FP32 (runs of up to kGradRun segments, the level below
// carried), of 4 in FP64 (no carry: its registers would not fit beside the
// accumulators at 4 wavefronts per SIMD).
template <typename T, int KM>
void launch_grad_seg(mr_ctx* c, const GradArgs<T>& a, hipStream_t s) {
  constexpr bool f64 = sizeof(T) == 8;
  constexpr int ZS = f64 ? 4 : 8;   // levels per segment
  const int ntx = (c->nx + kWave - 1) / kWave, nty = (c->ny + kGradRows - 1) / kGradRows;
  const int nseg = (c->nz + ZS - 1) / ZS;
  const int run = f64 ? 1 : std::min(nseg, kGradRun);
  const int nrun = (nseg + run - 1) / run;
  const dim3 grid((unsigned)((int64_t)ntx * nty * nrun)), block(kWave * kGradRows);   // 74 KB of LDS
  hipLaunchKernelGGL((grad_seg<T, KM, ZS, !f64>), grid, block, 0, s, a, run);
}

template <typename T>
hipError_t grad_t(mr_ctx* c, const Geom<T>& g, int count, const int64_t* steps,
                  const void* const* thetas, const void* const* mus, void* gu, void* gv, void* gw,
                  hipStream_t s) {
  GradArgs<T> a;
  ::memset((void*)&a, 0, sizeof(a));
  for (int q = 0; q < count; ++q) {
    a.th[q] = (const T*)thetas[q];
    a.mu[q] = (const T*)mus[q];
    a.tau[q] = (T)c->tau[step_kind(steps[q], c->n_avg)];
  }
  a.count = count;
  a.gu = (T*)gu;
  a.gv = (T*)gv;
  a.gw = (T*)gw;
  a.g = g;
  a.nx = c->nx;
  a.ny = c->ny;
  a.nz = c->nz;
  a.wx = c->wx;
  a.wy = c->wy;
  if (c->face_order == 4) {
    const int64_t cells = (int64_t)c->nx * c->ny * c->nz;
    const dim3 grid((unsigned)((cells + 255) / 256));
    hipLaunchKernelGGL((grad_kernel<T, true>), grid, dim3(256), 0, s, a);
  } else if (count <= 4) {
    launch_grad_seg<T, 4>(c, a, s);
  } else if (count <= 8) {
    launch_grad_seg<T, 8>(c, a, s);
  } else {
    launch_grad_seg<T, kMaxGradSteps>(c, a, s);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(mr_ctx* c, int64_t n, const void* thp, const void* thc, void* thn,
                       const void* u, const void* v, const void* w, hipStream_t s) {
  if (c->precision == MR_FP64) return step_t<double>(c, c->g64, n, thp, thc, thn, u, v, w, s);
  return step_t<float>(c, c->g32, n, thp, thc, thn, u, v, w, s);
}

hipError_t launch_seed(mr_ctx* c, int64_t n, const void* lam, void* mu, hipStream_t s) {
  if (c->precision == MR_FP64) return seed_t<double>(c, c->g64, n, lam, mu, s);
  return seed_t<float>(c, c->g32, n, lam, mu, s);
}

hipError_t launch_step_backward(mr_ctx* c, int64_t n, const void* mun, const void* muc,
                                const void* lam_add, void* out, const void* u, const void* v,
                                const void* w, hipStream_t s) {
  if (c->precision == MR_FP64) return bwd_t<double>(c, c->g64, n, mun, muc, lam_add, out, u, v, w, s);
  return bwd_t<float>(c, c->g32, n, mun, muc, lam_add, out, u, v, w, s);
}

hipError_t launch_velocity_grad(mr_ctx* c, int count, const int64_t* steps,
                                const void* const* thetas, const void* const* mus, void* gu,
                                void* gv, void* gw, hipStream_t s) {
  if (c->precision == MR_FP64) return grad_t<double>(c, c->g64, count, steps, thetas, mus, gu, gv, gw, s);
  return grad_t<float>(c, c->g32, count, steps, thetas, mus, gu, gv, gw, s);
}

}  // namespace mr
