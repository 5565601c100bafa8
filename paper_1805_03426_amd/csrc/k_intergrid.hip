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
// difference quotient times its dual volume.  Two-pass, fixed partition and
// fixed combining order with double-double partial sums, so the result is
// compensated and bitwise reproducible.
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

constexpr int kDissBlocks = 2048;

template <typename T>
__global__ void __launch_bounds__(256) diss_partial(const T* th, const double* hx, const double* hy,
                                                    const double* hz, const double* idxc,
                                                    const double* idyc, const double* dcz, int nx,
                                                    int ny, int nz, int dir_bot, int dir_top,
                                                    double t_bot, double t_top, double* part) {
  __shared__ DD sh[3][256 / kWave];
  const int nxy = nx * ny;
  const int64_t cells = (int64_t)nxy * nz;
  DD sx{0.0, 0.0}, sy{0.0, 0.0}, sz{0.0, 0.0};
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < cells;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(q % nx), j = (int)((q / nx) % ny), k = (int)(q / nxy);
    const int im = i == 0 ? nx - 1 : i - 1;
    const int jm = j == 0 ? ny - 1 : j - 1;
    const int row = k * nxy + j * nx;
    const double c = th[row + i];
    const double dx = c - (double)th[row + im];
    const double dy = c - (double)th[k * nxy + jm * nx + i];
    sx = dd_add(sx, dx * dx * idxc[i] * (hy[j] * hz[k]));
    sy = dd_add(sy, dy * dy * idyc[j] * (hx[i] * hz[k]));
    const double area = hx[i] * hy[j];
    if (k > 0) {
      const double dz = c - (double)th[row - nxy + i];
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
    double* o = part + (size_t)blockIdx.x * 6;
    o[0] = sx.s; o[1] = sx.c;
    o[2] = sy.s; o[3] = sy.c;
    o[4] = sz.s; o[5] = sz.c;
  }
}

// One wavefront: strided double-double merge of the partials, then the
// shuffle tree; out = {Nu_T, <theta_x^2>, <theta_y^2>, <theta_z^2>}.
__global__ void __launch_bounds__(kWave) diss_final(const double* part, int nb, double vtot,
                                                    double nufac, double* out) {
  DD sx{0.0, 0.0}, sy{0.0, 0.0}, sz{0.0, 0.0};
  for (int p = threadIdx.x; p < nb; p += kWave) {
    const double* o = part + (size_t)p * 6;
    sx = dd_merge(sx, DD{o[0], o[1]});
    sy = dd_merge(sy, DD{o[2], o[3]});
    sz = dd_merge(sz, DD{o[4], o[5]});
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz = wave_sum(sz);
  if (threadIdx.x == 0) {
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
  const int64_t cells = (int64_t)c->nx * c->ny * c->nz;
  const int nb = (int)std::min<int64_t>(kDissBlocks, (cells + 255) / 256);
  hipError_t e = ensure_red(c, sizeof(double) * 6 * kDissBlocks);
  if (e != hipSuccess) return e;
  const int db = c->bc_bot == MR_DIRICHLET, dtp = c->bc_top == MR_DIRICHLET;
  const Geom<double>& g = c->g64;
  if (c->precision == MR_FP64)
    hipLaunchKernelGGL(diss_partial<double>, dim3(nb), dim3(256), 0, s, (const double*)th, c->hx64,
                       c->areaw, c->hz64, g.idxc, g.idyc, c->dcz, c->nx, c->ny, c->nz, db, dtp,
                       c->t_bot, c->t_top, c->red);
  else
    hipLaunchKernelGGL(diss_partial<float>, dim3(nb), dim3(256), 0, s, (const float*)th, c->hx64,
                       c->areaw, c->hz64, g.idxc, g.idyc, c->dcz, c->nx, c->ny, c->nz, db, dtp,
                       c->t_bot, c->t_top, c->red);
  hipLaunchKernelGGL(diss_final, dim3(1), dim3(kWave), 0, s, (const double*)c->red, nb, c->vtot,
                     c->kappa * sqrt(c->ra * c->pr), out);
  return hipGetLastError();
}

}  // namespace mr
