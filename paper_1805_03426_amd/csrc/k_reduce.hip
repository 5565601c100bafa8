// Reductions: the discrete divergence check of the refined velocity
// (Sec. 3.2), the heat-flux Nusselt profile and mean scalar (Eq. 22), and a
// plain streaming copy used as the bandwidth reference.
//
// Every reduction is two-pass with a fixed partition and a fixed combining
// order (wavefront shuffles, then LDS, then a single final block), so results
// are bitwise reproducible.  Nusselt sums are double-double (error-free
// two-sum), i.e. compensated.
#include <algorithm>
#include <mutex>

#include "mr_internal.h"

namespace mr {

// Fixed device memory for the Nusselt partials of the allocation-free entry
// point: (nz + 1) faces x at most kNuMaxParts horizontal parts x 6 doubles,
// for nz up to kNuMaxFaces (3.15 MB per GPU, held until the process ends).
// In host code the array's name is only a stand-in: its device address comes
// from hipGetSymbolAddress, once per device, with that device current.
constexpr int kNuMaxParts = 64;
constexpr size_t kNuScratchDoubles = (size_t)(1024 + 1) * kNuMaxParts * 6;
static __device__ __align__(256) double scratch[kNuScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = (double*)ptr;
  return hipSuccess;
}

namespace {

__device__ __forceinline__ double shfl_down_d(double v, int off) {
  return __shfl_down(v, off, kWave);
}

// ------------------------------------------------------------- divergence
// Workgroups stride over the dense rows (k, j); the 256 lanes of a workgroup
// cover the row's x range.  The row's indices and widths are workgroup-uniform
// (no 64-bit division per cell), and the largest relative divergence is kept
// as a fraction (|div|, sum |flux|) compared by cross-multiplication, so that
// a cell costs no division.
constexpr int kDivBlocks = 2048;

__device__ __forceinline__ double rtab(const double* p, int k) {
  return ((const __attribute__((address_space(4))) double*)(p))[k];
}

template <typename T>
__global__ void __launch_bounds__(256) div_kernel(const T* u, const T* v, const T* w, const double* hx,
                                                  const double* hy, const double* hz, int nx, int ny,
                                                  int nz, int wx, int wy, double* part) {
  __shared__ double sh[2][256 / kWave];
  const size_t nxy = (size_t)nx * ny;
  const int rows = ny * nz;
  double mabs = 0.0, rnum = 0.0, rden = 1.0;   // largest |div| and largest |div| / sum |flux|
  for (int row = blockIdx.x; row < rows; row += gridDim.x) {
    const int k = row / ny, j = row - k * ny;
    const int jp = j == ny - 1 ? 0 : j + 1;
    const double hyj = rtab(hy, j), hzk = rtab(hz, k);
    const double ax = hyj * hzk;
    const bool vl0 = wy && j == 0, vr0 = wy && j == ny - 1;
    const size_t c0 = (size_t)k * nxy + (size_t)j * nx, cp = (size_t)k * nxy + (size_t)jp * nx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
      const int ip = i == nx - 1 ? 0 : i + 1;
      const double hxi = hx[i];
      const double ay = hxi * hzk, az = hxi * hyj;
      // side walls: the low wall face (stored) and the high one (not stored) carry nothing
      const double ul = wx && i == 0 ? 0.0 : (double)u[c0 + i];
      const double ur = wx && i == nx - 1 ? 0.0 : (double)u[c0 + ip];
      const double vl = vl0 ? 0.0 : (double)v[c0 + i];
      const double vr = vr0 ? 0.0 : (double)v[cp + i];
      const double wl = w[c0 + i], wr = w[c0 + nxy + i];
      const double dv = fabs((ur - ul) * ax + (vr - vl) * ay + (wr - wl) * az);
      const double tot = (fabs(ul) + fabs(ur)) * ax + (fabs(vl) + fabs(vr)) * ay + (fabs(wl) + fabs(wr)) * az;
      mabs = fmax(mabs, dv);
      if (tot > 0.0 && dv * rden > rnum * tot) {
        rnum = dv;
        rden = tot;
      }
    }
  }
  double mrel = rnum / rden;
  for (int off = kWave / 2; off > 0; off >>= 1) {
    mabs = fmax(mabs, shfl_down_d(mabs, off));
    mrel = fmax(mrel, shfl_down_d(mrel, off));
  }
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0) {
    sh[0][wv] = mabs;
    sh[1][wv] = mrel;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < (int)blockDim.x / kWave; ++q) {
      mabs = fmax(mabs, sh[0][q]);
      mrel = fmax(mrel, sh[1][q]);
    }
    part[2 * blockIdx.x] = mabs;
    part[2 * blockIdx.x + 1] = mrel;
  }
}

__global__ void __launch_bounds__(kWave) max_final(const double* part, int n, double* out) {
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < n; q += kWave) {
    a = fmax(a, part[2 * q]);
    b = fmax(b, part[2 * q + 1]);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    a = fmax(a, shfl_down_d(a, off));
    b = fmax(b, shfl_down_d(b, off));
  }
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

// ---------------------------------------------------------------- Nusselt
// partials[(k*P + p)*6 + {conv s,c, grad s,c, mean s,c}].  Block (p, q) covers
// the horizontal range p of faces kNuFaces*q .. kNuFaces*q + kNuFaces-1: each
// lane walks those faces for its cells carrying theta of the level below, so a
// level is read once per group of faces instead of once per face.
constexpr int kNuFaces = 2;   // timed: 2 faces per group beat 1, 3, 4, 8 and 16

template <typename T>
__global__ void __launch_bounds__(256) nu_partial(const T* th, const T* w, const double* hx,
                                                  const double* hy, int nx, int ny, int nz, int P,
                                                  int dir_bot, int dir_top, double t_bot,
                                                  double t_top, double* part) {
  __shared__ DD sh[3][256 / kWave];
  const int kf0 = blockIdx.y * kNuFaces;   // first face of the group (faces 0..nz)
  const int p = blockIdx.x;
  const int nxy = nx * ny;
  const int per = (nxy + P - 1) / P;
  const int lo = p * per, hi = min(nxy, lo + per);
  DD conv[kNuFaces], grad[kNuFaces], mean[kNuFaces];
#pragma unroll
  for (int f = 0; f < kNuFaces; ++f) conv[f] = grad[f] = mean[f] = DD{0.0, 0.0};
  for (int e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    const int i = e % nx, j = e / nx;
    const double area = hx[i] * hy[j];
    double below = kf0 > 0 && kf0 <= nz ? (double)th[(size_t)(kf0 - 1) * nxy + e] : 0.0;
#pragma unroll
    for (int f = 0; f < kNuFaces; ++f) {
      const int k = kf0 + f;
      if (k > nz) break;
      const double cur = k < nz ? (double)th[(size_t)k * nxy + e] : 0.0;
      if (k > 0 && k < nz) {
        conv[f] = dd_add(conv[f], (double)w[(size_t)k * nxy + e] * (0.5 * (below + cur)) * area);
        grad[f] = dd_add(grad[f], (cur - below) * area);
      } else if (k == 0) {
        if (dir_bot) grad[f] = dd_add(grad[f], (cur - t_bot) * area);
      } else {
        if (dir_top) grad[f] = dd_add(grad[f], (t_top - below) * area);
      }
      if (k < nz) mean[f] = dd_add(mean[f], cur * area);
      below = cur;
    }
  }
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
  for (int f = 0; f < kNuFaces; ++f) {
    const int k = kf0 + f;
    if (k > nz) break;
    DD c = wave_sum(conv[f]), g = wave_sum(grad[f]), m = wave_sum(mean[f]);
    __syncthreads();   // the previous face's merge has read sh
    if (lane == 0) {
      sh[0][wv] = c;
      sh[1][wv] = g;
      sh[2][wv] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < (int)blockDim.x / kWave; ++q) {
        c = dd_merge(c, sh[0][q]);
        g = dd_merge(g, sh[1][q]);
        m = dd_merge(m, sh[2][q]);
      }
      double* o = part + ((size_t)k * P + p) * 6;
      o[0] = c.s; o[1] = c.c;
      o[2] = g.s; o[3] = g.c;
      o[4] = m.s; o[5] = m.c;
    }
  }
}

// One workgroup: Nu_k of every face from the partials (fixed order), then the
// summary sums as a fixed tree (per-thread strided double-double sums, wave
// shuffles, then the four waves in order).  Per-face values stay in LDS.
constexpr int kNuMaxFaces = 1024;

__device__ __forceinline__ DD block_sum(DD v, DD* scratch) {
  v = wave_sum(v);
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  __syncthreads();
  if (lane == 0) scratch[wv] = v;
  __syncthreads();
  DD r = scratch[0];
  for (int q = 1; q < (int)blockDim.x / kWave; ++q) r = dd_merge(r, scratch[q]);
  return r;
}

__global__ void __launch_bounds__(256) nu_final(const double* part, int P, int nz,
                                                const double* dcz, const double* hz, double atot,
                                                double sq, double* prof) {
  __shared__ double s_nu[kNuMaxFaces + 1];
  __shared__ double s_mean[kNuMaxFaces];
  __shared__ DD scratch[256 / kWave];
  for (int k = threadIdx.x; k <= nz; k += blockDim.x) {
    DD conv{0.0, 0.0}, grad{0.0, 0.0}, mean{0.0, 0.0};
#pragma unroll 4
    for (int p = 0; p < P; ++p) {
      const double* o = part + ((size_t)k * P + p) * 6;
      conv = dd_merge(conv, DD{o[0], o[1]});
      grad = dd_merge(grad, DD{o[2], o[3]});
      mean = dd_merge(mean, DD{o[4], o[5]});
    }
    const double cs = conv.s + conv.c, gs = grad.s + grad.c;
    const double nu = sq * (cs / atot) - (gs / dcz[k]) / atot;
    prof[k] = nu;
    s_nu[k] = nu;
    if (k < nz) s_mean[k] = (mean.s + mean.c) * hz[k];
  }
  __syncthreads();
  DD vol{0.0, 0.0}, pap{0.0, 0.0}, mt{0.0, 0.0}, hsum{0.0, 0.0};
  for (int k = threadIdx.x; k <= nz; k += blockDim.x) {
    vol = dd_add(vol, dcz[k] * s_nu[k]);
    if (k > 0 && k < nz) pap = dd_add(pap, s_nu[k]);
    if (k < nz) {
      mt = dd_add(mt, s_mean[k]);
      hsum = dd_add(hsum, hz[k]);
    }
  }
  vol = block_sum(vol, scratch);
  pap = block_sum(pap, scratch);
  mt = block_sum(mt, scratch);
  hsum = block_sum(hsum, scratch);
  if (threadIdx.x == 0) {
    prof[nz + 1] = s_nu[0];
    prof[nz + 2] = s_nu[nz];
    prof[nz + 3] = vol.s + vol.c;
    prof[nz + 4] = nz > 1 ? (pap.s + pap.c) / (nz - 1) : 0.0;
    prof[nz + 5] = (mt.s + mt.c) / (atot * (hsum.s + hsum.c));
  }
}

// ------------------------------------------------------------------- copy
__global__ void __launch_bounds__(256) copy_kernel(const int4* __restrict__ src, int4* __restrict__ dst,
                                                   int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = src[t];
}

int nu_parts(const mr_ctx* c) {
  const int64_t nxy = (int64_t)c->nx * c->ny;
  int64_t P = (nxy + 256 * 16 - 1) / (256 * 16);
  return (int)std::max<int64_t>(1, std::min<int64_t>(P, kNuMaxParts));
}

// The two Nusselt kernels with the partials in `part`.
void nusselt_kernels(mr_ctx* c, const void* th, const void* w, double* prof, double* part, int P,
                     hipStream_t s) {
  const dim3 grid(P, (c->nz + 1 + kNuFaces - 1) / kNuFaces);
  const int db = c->bc_bot == MR_DIRICHLET, dtp = c->bc_top == MR_DIRICHLET;
  if (c->precision == MR_FP64)
    hipLaunchKernelGGL(nu_partial<double>, grid, dim3(256), 0, s, (const double*)th, (const double*)w,
                       c->hx64, c->areaw, c->nx, c->ny, c->nz, P, db, dtp, c->t_bot, c->t_top, part);
  else
    hipLaunchKernelGGL(nu_partial<float>, grid, dim3(256), 0, s, (const float*)th, (const float*)w,
                       c->hx64, c->areaw, c->nx, c->ny, c->nz, P, db, dtp, c->t_bot, c->t_top, part);
  hipLaunchKernelGGL(nu_final, dim3(1), dim3(256), 0, s, (const double*)part, P, c->nz, c->dcz,
                     c->hz64, c->atot, sqrt(c->ra * c->pr), prof);
}

}  // namespace

hipError_t ensure_red(mr_ctx* c, size_t bytes) {
  if (c->red_bytes >= bytes) return hipSuccess;
  if (c->red) (void)hipFree(c->red);
  c->red = nullptr;
  c->red_bytes = 0;
  hipError_t e = hipMalloc((void**)&c->red, bytes);
  if (e == hipSuccess) c->red_bytes = bytes;
  return e;
}

hipError_t launch_divergence(mr_ctx* c, const void* u, const void* v, const void* w, double* out,
                             hipStream_t s) {
  const int64_t cells = (int64_t)c->nx * c->ny * c->nz;
  const int nb = (int)std::min<int64_t>(kDivBlocks, (cells + 255) / 256);
  hipError_t e = ensure_red(c, sizeof(double) * 2 * kDivBlocks);
  if (e != hipSuccess) return e;
  if (c->precision == MR_FP64)
    hipLaunchKernelGGL(div_kernel<double>, dim3(nb), dim3(256), 0, s, (const double*)u, (const double*)v,
                       (const double*)w, c->hx64, c->areaw, c->hz64, c->nx, c->ny, c->nz, c->wx, c->wy,
                       c->red);
  else
    hipLaunchKernelGGL(div_kernel<float>, dim3(nb), dim3(256), 0, s, (const float*)u, (const float*)v,
                       (const float*)w, c->hx64, c->areaw, c->hz64, c->nx, c->ny, c->nz, c->wx, c->wy,
                       c->red);
  hipLaunchKernelGGL(max_final, dim3(1), dim3(kWave), 0, s, (const double*)c->red, nb, out);
  return hipGetLastError();
}

hipError_t launch_nusselt(mr_ctx* c, const void* th, const void* w, double* prof, hipStream_t s) {
  const int P = nu_parts(c);
  const size_t part = (size_t)(c->nz + 1) * P * 6;
  if (c->nz > kNuMaxFaces) return hipErrorInvalidValue;
  hipError_t e = ensure_red(c, sizeof(double) * part);
  if (e != hipSuccess) return e;
  nusselt_kernels(c, th, w, prof, c->red, P, s);
  return hipGetLastError();
}

int nusselt_fixed(mr_ctx* c, const void* th, const void* w, double* prof, hipStream_t s) {
  const int P = nu_parts(c);
  if (c->nz > kNuMaxFaces || (size_t)(c->nz + 1) * P * 6 > kNuScratchDoubles) return MR_ESHAPE;
  if (c->device < 0 || c->device >= kMaxDevices) return MR_EINVAL;
  double* part;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    part = g_scratch[c->device];
  }
  if (!part) return MR_EINVAL;   // mr_init sets it up for the context's device
  nusselt_kernels(c, th, w, prof, part, P, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    c->last_err = (int)e;
    return MR_EHIP;
  }
  return MR_OK;
}

hipError_t launch_copy(const void* src, void* dst, int64_t nbytes, hipStream_t s) {
  const int64_t n = nbytes / 16;
  if (n == 0) return hipSuccess;
  const int nb = (int)std::min<int64_t>(65536, (n + 255) / 256);
  hipLaunchKernelGGL(copy_kernel, dim3(nb), dim3(256), 0, s, (const int4*)src, (int4*)dst, n);
  return hipGetLastError();
}

}  // namespace mr
