// Inter-grid kernels around the dense scalar step: the upscale integration of
// the scalar to the coarse grid (Sec. 3.3, Eq. 20, as the volume-weighted mean
// over the sub-cells) and the dissipation Nusselt number Nu_T = eps_T (Ra Pr)^(1/2)
// with eps_T = kappa <|grad theta|^2>_V (Sec. 4.1, Eq. 23).
//
// Integration: a workgroup of 256 lanes covers 256 consecutive dense columns
// of one coarse row (J, K), i.e. floor(256/mx) coarse cells; every lane sums
// its column over the my x mz dense rows of the coarse layer (coalesced row
// reads, FP64 accumulation), and the first lane of each coarse cell combines
// the mx columns through LDS.  The dense field is read once.
//
// Dissipation: every dense cell owns its low x face, low y face and low z face
// (and the top plate for the last level); each face adds its squared
// difference quotient times its dual volume.  Two-pass, fixed partition
// (row segments x level ranges) and fixed combining order with double-double
// partial sums, so the result is compensated and bitwise reproducible.
#include <algorithm>

#include "mr_internal.h"

namespace mr {
namespace {

constexpr int kIntBlock = 256;

template <typename T>
__global__ void __launch_bounds__(kIntBlock) integrate_kernel(const T* th, T* tc, const double* hx,
                                                              const double* hy, const double* hz,
                                                              int nx, int ny, int mx, int my, int mz,
                                                              int ncx, int ncy, int nbx) {
  __shared__ double s_acc[kIntBlock];
  __shared__ double s_hx[kIntBlock];
  const int cpb = kIntBlock / mx;   // coarse cells per workgroup
  const int b = blockIdx.x;
  const int bx = b % nbx, J = (b / nbx) % ncy, K = b / (nbx * ncy);
  const int t = threadIdx.x;
  const int cc = t / mx, sub = t - cc * mx;
  const int I = bx * cpb + cc;
  const bool on = cc < cpb && I < ncx;
  double acc = 0.0, vyz = 0.0, wx = 0.0;
  if (on) {
    const int i = I * mx + sub;
    wx = hx[i];
    for (int kk = 0; kk < mz; ++kk) {
      const int k = K * mz + kk;
      for (int jj = 0; jj < my; ++jj) {
        const int j = J * my + jj;
        const double wyz = hy[j] * hz[k];
        acc += (double)th[((size_t)k * ny + j) * nx + i] * wyz;
        vyz += wyz;
      }
    }
  }
  s_acc[t] = acc * wx;
  s_hx[t] = wx;
  __syncthreads();
  if (on && sub == 0) {
    double num = 0.0, hxs = 0.0;
    for (int q = 0; q < mx; ++q) {
      num += s_acc[t + q];
      hxs += s_hx[t + q];
    }
    tc[((size_t)K * ncy + J) * ncx + I] = (T)(num / (hxs * vyz));
  }
}

// Nu_T partials: a workgroup of 256 lanes covers 256 consecutive columns of
// one row j and a range of kb levels; each lane walks up its column carrying
// theta(k-1), reads its own value, its x neighbour (mostly the same cache
// lines) and the row j-1 value, and accumulates the faces on the low side of
// its cell (plus the top plate for the last level).  Fixed partition:
// part[b] holds workgroup b's three double-double sums.
constexpr int kDissMaxParts = 2048;

template <typename T>
__global__ void __launch_bounds__(256) diss_partial(const T* th, const double* hx, const double* hy,
                                                    const double* hz, const double* idxc,
                                                    const double* idyc, const double* dcz, int nx,
                                                    int ny, int nz, int nbx, int kb, int walx, int waly,
                                                    int dir_bot, int dir_top, double t_bot,
                                                    double t_top, double* part) {
  __shared__ DD sh[3][256 / kWave];
  const int b = blockIdx.x;
  const int bx = b % nbx, j = (b / nbx) % ny, kc = b / (nbx * ny);
  const int i_raw = bx * 256 + threadIdx.x;
  const bool on = i_raw < nx;
  const int i = on ? i_raw : nx - 1;
  // across a side wall the neighbour is the cell itself: the wall face adds nothing
  const int im = i == 0 ? (walx ? 0 : nx - 1) : i - 1;
  const int jm = j == 0 ? (waly ? 0 : ny - 1) : j - 1;
  const size_t nxy = (size_t)nx * ny;
  const int k0 = kc * kb, k1 = min(nz, k0 + kb);
  const double wx = idxc[i] * hy[j], wy = idyc[j] * hx[i], area = hx[i] * hy[j];
  DD sx{0.0, 0.0}, sy{0.0, 0.0}, sz{0.0, 0.0};
  double below = k0 > 0 ? (double)th[(size_t)(k0 - 1) * nxy + (size_t)j * nx + i] : 0.0;
  for (int k = k0; k < k1; ++k) {
    const T* lvl = th + (size_t)k * nxy;
    const double c = lvl[(size_t)j * nx + i];
    const double dx = c - (double)lvl[(size_t)j * nx + im];
    const double dy = c - (double)lvl[(size_t)jm * nx + i];
    if (on) {
      sx = dd_add(sx, dx * dx * wx * hz[k]);
      sy = dd_add(sy, dy * dy * wy * hz[k]);
      if (k > 0) {
        const double dz = c - below;
        sz = dd_add(sz, dz * dz / dcz[k] * area);
      } else if (dir_bot) {
        const double dz = c - t_bot;
        sz = dd_add(sz, dz * dz / dcz[0] * area);
      }
      if (k == nz - 1 && dir_top) {
        const double dz = t_top - c;
        sz = dd_add(sz, dz * dz / dcz[nz] * area);
      }
    }
    below = c;
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz = wave_sum(sz);
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0) {
    sh[0][wv] = sx;
    sh[1][wv] = sy;
    sh[2][wv] = sz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int p = 1; p < (int)blockDim.x / kWave; ++p) {
      sx = dd_merge(sx, sh[0][p]);
      sy = dd_merge(sy, sh[1][p]);
      sz = dd_merge(sz, sh[2][p]);
    }
    double* o = part + (size_t)b * 6;
    o[0] = sx.s; o[1] = sx.c;
    o[2] = sy.s; o[3] = sy.c;
    o[4] = sz.s; o[5] = sz.c;
  }
}

// One workgroup: strided double-double merge of the partials, the shuffle
// tree in each wavefront, then the four wavefronts in order;
// out = {Nu_T, <theta_x^2>, <theta_y^2>, <theta_z^2>}.
constexpr int kDissFinal = 256;

__global__ void __launch_bounds__(kDissFinal) diss_final(const double* part, int nb, double vtot,
                                                         double nufac, double* out) {
  __shared__ DD sh[3][kDissFinal / kWave];
  DD sx{0.0, 0.0}, sy{0.0, 0.0}, sz{0.0, 0.0};
  for (int p = threadIdx.x; p < nb; p += kDissFinal) {
    const double* o = part + (size_t)p * 6;
    sx = dd_merge(sx, DD{o[0], o[1]});
    sy = dd_merge(sy, DD{o[2], o[3]});
    sz = dd_merge(sz, DD{o[4], o[5]});
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz = wave_sum(sz);
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0) {
    sh[0][wv] = sx;
    sh[1][wv] = sy;
    sh[2][wv] = sz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kDissFinal / kWave; ++q) {
      sx = dd_merge(sx, sh[0][q]);
      sy = dd_merge(sy, sh[1][q]);
      sz = dd_merge(sz, sh[2][q]);
    }
    const double gx = (sx.s + sx.c) / vtot, gy = (sy.s + sy.c) / vtot, gz = (sz.s + sz.c) / vtot;
    out[0] = nufac * (gx + gy + gz);
    out[1] = gx;
    out[2] = gy;
    out[3] = gz;
  }
}

}  // namespace

hipError_t launch_integrate(mr_ctx* c, const void* th, void* tc, hipStream_t s) {
  const int cpb = kIntBlock / c->mx;
  if (cpb < 1) return hipErrorInvalidValue;
  const int nbx = (c->ncx + cpb - 1) / cpb;
  const int64_t nb = (int64_t)nbx * c->ncy * c->ncz;
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  if (c->precision == MR_FP64)
    hipLaunchKernelGGL(integrate_kernel<double>, dim3((unsigned)nb), dim3(kIntBlock), 0, s,
                       (const double*)th, (double*)tc, c->hx64, c->areaw, c->hz64, c->nx, c->ny,
                       c->mx, c->my, c->mz, c->ncx, c->ncy, nbx);
  else
    hipLaunchKernelGGL(integrate_kernel<float>, dim3((unsigned)nb), dim3(kIntBlock), 0, s,
                       (const float*)th, (float*)tc, c->hx64, c->areaw, c->hz64, c->nx, c->ny, c->mx,
                       c->my, c->mz, c->ncx, c->ncy, nbx);
  return hipGetLastError();
}

hipError_t launch_dissipation(mr_ctx* c, const void* th, double* out, hipStream_t s) {
  const int nbx = (c->nx + 255) / 256;
  const int64_t rows = (int64_t)nbx * c->ny;
  // levels per workgroup: enough workgroups to fill the chip, at most kDissMaxParts partials
  int nkb = (int)std::max<int64_t>(1, std::min<int64_t>(c->nz, kDissMaxParts / std::max<int64_t>(1, rows)));
  const int kb = (c->nz + nkb - 1) / nkb;
  nkb = (c->nz + kb - 1) / kb;
  const int64_t nb = rows * nkb;
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  hipError_t e = ensure_red(c, sizeof(double) * 6 * (size_t)nb);
  if (e != hipSuccess) return e;
  const int db = c->bc_bot == MR_DIRICHLET, dtp = c->bc_top == MR_DIRICHLET;
  const Geom<double>& g = c->g64;
  if (c->precision == MR_FP64)
    hipLaunchKernelGGL(diss_partial<double>, dim3((unsigned)nb), dim3(256), 0, s, (const double*)th,
                       c->hx64, c->areaw, c->hz64, g.idxc, g.idyc, c->dcz, c->nx, c->ny, c->nz, nbx,
                       kb, c->wx, c->wy, db, dtp, c->t_bot, c->t_top, c->red);
  else
    hipLaunchKernelGGL(diss_partial<float>, dim3((unsigned)nb), dim3(256), 0, s, (const float*)th,
                       c->hx64, c->areaw, c->hz64, g.idxc, g.idyc, c->dcz, c->nx, c->ny, c->nz, nbx,
                       kb, c->wx, c->wy, db, dtp, c->t_bot, c->t_top, c->red);
  hipLaunchKernelGGL(diss_final, dim3(1), dim3(kDissFinal), 0, s, (const double*)c->red, (int)nb, c->vtot,
                     c->kappa * sqrt(c->ra * c->pr), out);
  return hipGetLastError();
}

}  // namespace mr
