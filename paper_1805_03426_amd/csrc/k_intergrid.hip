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
// (tiles of columns x level ranges) and fixed combining order with double-double
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

// Nu_T partials: a workgroup of kDissRows wavefronts covers a tile of 64
// columns by kDissRows rows and a range of kb levels; the lane of wavefront r
// walks up column (i0 + lane, j0 + r) carrying theta(k-1), reads its own value
// and its x neighbour (the same cache lines but one), and accumulates the
// faces on the low side of its cell (plus the top plate for the last level).
// The row j-1 values come through LDS: every wavefront publishes its rows of
// a batch of kDissAhead levels, the first also the row below the tile, so a
// row is read from memory about once (1 + 1/kDissRows).  Batches alternate
// between two LDS buffers, one barrier per batch; the loads of the next batch
// are in flight while one is summed.  Fixed partition: part[b]
// holds the three double-double sums of the workgroup of logical index b;
// consecutive tiles run on one XCD.
constexpr int kDissMaxParts = 2048;
constexpr int kDissAhead = 4;
constexpr int kDissRows = 4;
constexpr int kDissWaves = 8192;   // wavefronts to aim for (32 per CU)

constexpr int kDissMaxKb = 512;     // levels per workgroup at most (LDS level tables of 8 KB)

template <typename T>
__global__ void __launch_bounds__(64 * kDissRows) diss_partial(const T* th, const double* hx, const double* hy,
                                                               const double* hz, const double* idxc,
                                                               const double* idyc, const double* dcz, int nx,
                                                               int ny, int nz, int nbx, int nby, int kb, int walx,
                                                               int waly, int dir_bot, int dir_top, double t_bot,
                                                               double t_top, double* part) {
  __shared__ T rows[2][kDissAhead][kDissRows + 1][kWave];
  __shared__ DD sh[3][kDissRows];
  // hz and 1/dcz of the level range (kb and kb + 1 values, dynamic LDS)
  extern __shared__ double ztabs[];
  double* const shz = ztabs;
  double* const sidz = ztabs + kb;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = b % nbx, by = (b / nbx) % nby, kc = b / (nbx * nby);
  const int lane = threadIdx.x, r = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int i_raw = bx * kWave + lane, j_raw = by * kDissRows + r;
  const bool on = i_raw < nx && j_raw < ny;
  const int i = i_raw < nx ? i_raw : nx - 1, j = j_raw < ny ? j_raw : ny - 1;
  // across a side wall the neighbour is the cell itself: the wall face adds nothing
  const int im = i == 0 ? (walx ? 0 : nx - 1) : i - 1;
  const bool ywall = waly && j_raw == 0;
  // the row below the tile (loaded by the first wavefront)
  const int j0 = by * kDissRows;
  const int jh = j0 == 0 ? (waly ? 0 : ny - 1) : j0 - 1;
  const size_t nxy = (size_t)nx * ny;
  const int k0 = kc * kb, k1 = min(nz, k0 + kb);
  for (int t = r * kWave + lane; t <= k1 - k0; t += kWave * kDissRows) {
    if (k0 + t < k1) shz[t] = hz[k0 + t];
    sidz[t] = 1.0 / dcz[k0 + t];
  }
  const double wx = idxc[i] * hy[j], wy = idyc[j] * hx[i], area = hx[i] * hy[j];
  DD sx{0.0, 0.0}, sy{0.0, 0.0}, sz{0.0, 0.0};
  double below = k0 > 0 ? (double)th[(size_t)(k0 - 1) * nxy + (size_t)j * nx + i] : 0.0;
  const T* colc = th + (size_t)j * nx;
  const T* colh = th + (size_t)jh * nx;
  // batch loads: own row, x neighbour, and (first wavefront) the row below
  T vc[kDissAhead], vx[kDissAhead], vh[kDissAhead], nc[kDissAhead], nxv[kDissAhead], nh[kDissAhead];
  auto load = [&](int kk, T* c, T* x, T* h) {
#pragma unroll
    for (int q = 0; q < kDissAhead; ++q) {
      const size_t lv = (size_t)min(kk + q, k1 - 1) * nxy;
      c[q] = colc[lv + i];
      x[q] = colc[lv + im];
      if (r == 0) h[q] = colh[lv + i];
    }
  };
  if (k0 < k1) load(k0, vc, vx, vh);
  int p = 0;
  for (int kk = k0; kk < k1; kk += kDissAhead, p ^= 1) {
    // the next batch's loads go out before this batch is used
    const bool more = kk + kDissAhead < k1;
    if (more) load(kk + kDissAhead, nc, nxv, nh);
#pragma unroll
    for (int q = 0; q < kDissAhead; ++q) {
      rows[p][q][r + 1][lane] = vc[q];
      if (r == 0) rows[p][q][0][lane] = vh[q];
    }
    __syncthreads();
    // the batch's faces summed in double (positive terms: relative error at
    // most kDissAhead eps), then added to the double-double sums
    double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
    for (int q = 0; q < kDissAhead; ++q) {
      const int k = kk + q;
      if (k >= k1) break;
      const double c = vc[q];
      const double dx = c - (double)vx[q];
      const double dy = ywall ? 0.0 : c - (double)rows[p][q][r][lane];
      const double hzk = shz[k - k0];
      ax += dx * dx * hzk;
      ay += dy * dy * hzk;
      if (k > 0) {
        const double dz = c - below;
        az += dz * dz * sidz[k - k0];
      } else if (dir_bot) {
        const double dz = c - t_bot;
        az += dz * dz * sidz[0];
      }
      if (k == nz - 1 && dir_top) {
        const double dz = t_top - c;
        az += dz * dz * sidz[nz - k0];
      }
      below = c;
    }
    if (on) {
      sx = dd_add(sx, ax * wx);
      sy = dd_add(sy, ay * wy);
      sz = dd_add(sz, az * area);
    }
    if (more) {
#pragma unroll
      for (int q = 0; q < kDissAhead; ++q) {
        vc[q] = nc[q];
        vx[q] = nxv[q];
        vh[q] = nh[q];
      }
    }
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz = wave_sum(sz);
  if (lane == 0) {
    sh[0][r] = sx;
    sh[1][r] = sy;
    sh[2][r] = sz;
  }
  __syncthreads();
  if (lane == 0 && r == 0) {
    for (int q = 1; q < kDissRows; ++q) {
      sx = dd_merge(sx, sh[0][q]);
      sy = dd_merge(sy, sh[1][q]);
      sz = dd_merge(sz, sh[2][q]);
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
constexpr int kDissFinal = 1024;

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
  const int nbx = (c->nx + kWave - 1) / kWave, nby = (c->ny + kDissRows - 1) / kDissRows;
  const int64_t tiles = (int64_t)nbx * nby;
  // level ranges: about kDissWaves wavefronts in all (ranges as long as that
  // allows: each workgroup ends with a reduction), at most kDissMaxParts partials
  const int64_t want = (kDissWaves / kDissRows + tiles - 1) / tiles;
  int nkb = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)c->nz, want, kDissMaxParts / tiles}));
  nkb = std::max(nkb, (c->nz + kDissMaxKb - 1) / kDissMaxKb);
  const int kb = (c->nz + nkb - 1) / nkb;
  nkb = (c->nz + kb - 1) / kb;
  const int64_t nb = tiles * nkb;
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  hipError_t e = ensure_red(c, sizeof(double) * 6 * (size_t)nb);
  if (e != hipSuccess) return e;
  const int db = c->bc_bot == MR_DIRICHLET, dtp = c->bc_top == MR_DIRICHLET;
  const Geom<double>& g = c->g64;
  const dim3 block(kWave, kDissRows);
  const size_t lds = sizeof(double) * (2 * (size_t)kb + 1);
  if (c->precision == MR_FP64)
    hipLaunchKernelGGL(diss_partial<double>, dim3((unsigned)nb), block, lds, s, (const double*)th, c->hx64,
                       c->areaw, c->hz64, g.idxc, g.idyc, c->dcz, c->nx, c->ny, c->nz, nbx, nby, kb, c->wx,
                       c->wy, db, dtp, c->t_bot, c->t_top, c->red);
  else
    hipLaunchKernelGGL(diss_partial<float>, dim3((unsigned)nb), block, lds, s, (const float*)th, c->hx64,
                       c->areaw, c->hz64, g.idxc, g.idyc, c->dcz, c->nx, c->ny, c->nz, nbx, nby, kb, c->wx,
                       c->wy, db, dtp, c->t_bot, c->t_top, c->red);
  hipLaunchKernelGGL(diss_final, dim3(1), dim3(kDissFinal), 0, s, (const double*)c->red, (int)nb, c->vtot,
                     c->kappa * sqrt(c->ra * c->pr), out);
  return hipGetLastError();
}

}  // namespace mr
