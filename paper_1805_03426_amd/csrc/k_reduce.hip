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

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

__device__ __forceinline__ double shfl_down_d(double v, int off) {
  return __shfl_down(v, off, kWave);
}

// ------------------------------------------------------------- divergence
// Workgroups stride over the dense rows (k, j); the 256 lanes of a workgroup
// cover the row's x range, V consecutive cells a lane (16-byte vector loads
// where V divides nx and the fields are 16-byte aligned).  The row's indices
// and widths are workgroup-uniform (no 64-bit division per cell), and the
// largest relative divergence is kept as a fraction (|div|, sum |flux|)
// compared by cross-multiplication, so that a cell costs no division.
// Workgroups of the row's lanes (up to 256) and about kDivWaves wavefronts in
// all (16 a CU).  Timed at 1024x1024x512 FP64: 3.24 ms with 2048 workgroups
// of 256 lanes, 2.83 ms with 1024; at 256^3 (128 lanes a row in FP64) 2048
// workgroups of which half the lanes idle took 93 us, 1024 took 124 us.
constexpr int kDivWaves = 4096;

__device__ __forceinline__ double rtab(const double* p, int k) {
  return ((const __attribute__((address_space(4))) double*)(p))[k];
}

// V consecutive values from p (16-byte aligned when V > 1).
template <typename T, int V>
__device__ __forceinline__ void ldv(const T* p, T* o) {
  if constexpr (V == 1) {
    o[0] = *p;
  } else {
    typedef T vt __attribute__((ext_vector_type(V)));
    const vt x = *reinterpret_cast<const vt*>(p);
#pragma unroll
    for (int q = 0; q < V; ++q) o[q] = x[q];
  }
}

template <typename T, int V>
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
    for (int i0 = threadIdx.x * V; i0 < nx; i0 += blockDim.x * V) {
      T uu[V + 1], vl_[V], vr_[V], wl_[V], wr_[V];
      ldv<T, V>(u + c0 + i0, uu);
      uu[V] = u[c0 + (i0 + V == nx ? 0 : i0 + V)];
      ldv<T, V>(v + c0 + i0, vl_);
      ldv<T, V>(v + cp + i0, vr_);
      ldv<T, V>(w + c0 + i0, wl_);
      ldv<T, V>(w + c0 + nxy + i0, wr_);
#pragma unroll
      for (int q = 0; q < V; ++q) {
        const int i = i0 + q;
        const double hxi = hx[i];
        const double ay = hxi * hzk, az = hxi * hyj;
        // side walls: the low wall face (stored) and the high one (not stored) carry nothing
        const double ul = wx && i == 0 ? 0.0 : (double)uu[q];
        const double ur = wx && i == nx - 1 ? 0.0 : (double)uu[q + 1];
        const double vl = vl0 ? 0.0 : (double)vl_[q];
        const double vr = vr0 ? 0.0 : (double)vr_[q];
        const double wl = wl_[q], wr = wr_[q];
        const double dv = fabs((ur - ul) * ax + (vr - vl) * ay + (wr - wl) * az);
        const double tot = (fabs(ul) + fabs(ur)) * ax + (fabs(vl) + fabs(vr)) * ay + (fabs(wl) + fabs(wr)) * az;
        mabs = fmax(mabs, dv);
        if (tot > 0.0 && dv * rden > rnum * tot) {
          rnum = dv;
          rden = tot;
        }
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
// the horizontal range p of faces kNuFaces*q .. kNuFaces*q + kNuFaces-1, V
// consecutive cells of one row a lane (16-byte vector loads where V divides
// nx and the fields are 16-byte aligned; the row index is one division per V
// cells).  Each lane walks the group's faces for its cells carrying theta of
// the level below, so a level is read once per group of faces instead of once
// per face.
constexpr int kNuFaces = 2;   // timed: 2 faces per group beat 1, 3, 4, 8 and 16

template <typename T, int V>
__global__ void __launch_bounds__(256) nu_partial(const T* th, const T* w, const double* hx,
                                                  const double* hy, int nx, int ny, int nz, int P,
                                                  int dir_bot, int dir_top, double t_bot,
                                                  double t_top, double* part) {
  __shared__ DD sh[3][256 / kWave];
  const int kf0 = blockIdx.y * kNuFaces;   // first face of the group (faces 0..nz)
  const int p = blockIdx.x;
  const int nxy = nx * ny;
  const int per = ((nxy + P - 1) / P + V - 1) / V * V;   // whole vectors (V divides nx)
  const int lo = p * per, hi = min(nxy, lo + per);
  DD conv[kNuFaces], grad[kNuFaces], mean[kNuFaces];
#pragma unroll
  for (int f = 0; f < kNuFaces; ++f) conv[f] = grad[f] = mean[f] = DD{0.0, 0.0};
  for (int e0 = lo + threadIdx.x * V; e0 < hi; e0 += blockDim.x * V) {
    const int j = e0 / nx, i0 = e0 - j * nx;
    const double hyj = hy[j];
    double area[V], below[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      area[q] = hx[i0 + q] * hyj;
      below[q] = 0.0;
    }
    if (kf0 > 0 && kf0 <= nz) {
      T b[V];
      ldv<T, V>(th + (size_t)(kf0 - 1) * nxy + e0, b);
#pragma unroll
      for (int q = 0; q < V; ++q) below[q] = (double)b[q];
    }
#pragma unroll
    for (int f = 0; f < kNuFaces; ++f) {
      const int k = kf0 + f;
      if (k > nz) break;
      T ct[V], wt[V];
#pragma unroll
      for (int q = 0; q < V; ++q) ct[q] = wt[q] = T(0);
      if (k < nz) ldv<T, V>(th + (size_t)k * nxy + e0, ct);
      if (k > 0 && k < nz) ldv<T, V>(w + (size_t)k * nxy + e0, wt);
#pragma unroll
      for (int q = 0; q < V; ++q) {
        const double cur = (double)ct[q];
        if (k > 0 && k < nz) {
          conv[f] = dd_add(conv[f], (double)wt[q] * (0.5 * (below[q] + cur)) * area[q]);
          grad[f] = dd_add(grad[f], (cur - below[q]) * area[q]);
        } else if (k == 0) {
          if (dir_bot) grad[f] = dd_add(grad[f], (cur - t_bot) * area[q]);
        } else {
          if (dir_top) grad[f] = dd_add(grad[f], (t_top - below[q]) * area[q]);
        }
        if (k < nz) mean[f] = dd_add(mean[f], cur * area[q]);
        below[q] = cur;
      }
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

// Vector width of the Nusselt partials (16-byte loads where it divides nx) and
// the number of horizontal parts (about 4096 cells each, at most kNuMaxParts).
int nu_vec(const mr_ctx* c) {
  const int v = c->precision == MR_FP64 ? 2 : 4;
  return c->nx % v == 0 ? v : 1;
}

int nu_parts(const mr_ctx* c) {
  const int64_t nxy = (int64_t)c->nx * c->ny;
  int64_t P = (nxy + 256 * 16 - 1) / (256 * 16);
  return (int)std::max<int64_t>(1, std::min<int64_t>(P, kNuMaxParts));
}

// The two Nusselt kernels with the partials in `part`.
void nusselt_kernels(mr_ctx* c, const void* th, const void* w, double* prof, double* part, int P,
                     hipStream_t s) {
  const dim3 grid(P, (c->nz + 1 + kNuFaces - 1) / kNuFaces), block(256);
  const int db = c->bc_bot == MR_DIRICHLET, dtp = c->bc_top == MR_DIRICHLET;
  // unaligned fields: one cell a lane, the same parts
  const bool vec = aligned16(th) && aligned16(w) && nu_vec(c) > 1;
  if (c->precision == MR_FP64) {
    auto k = vec ? nu_partial<double, 2> : nu_partial<double, 1>;
    hipLaunchKernelGGL(k, grid, block, 0, s, (const double*)th, (const double*)w, c->hx64, c->areaw, c->nx,
                       c->ny, c->nz, P, db, dtp, c->t_bot, c->t_top, part);
  } else {
    auto k = vec ? nu_partial<float, 4> : nu_partial<float, 1>;
    hipLaunchKernelGGL(k, grid, block, 0, s, (const float*)th, (const float*)w, c->hx64, c->areaw, c->nx,
                       c->ny, c->nz, P, db, dtp, c->t_bot, c->t_top, part);
  }
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
  const bool f64 = c->precision == MR_FP64;
  const int vw = f64 ? 2 : 4;
  const bool vec = aligned16(u) && aligned16(v) && aligned16(w) && c->nx % vw == 0;
  const int lanes = vec ? c->nx / vw : c->nx;
  const int threads = std::min(256, (lanes + kWave - 1) / kWave * kWave);
  const int64_t rows = (int64_t)c->ny * c->nz;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kDivWaves / (threads / kWave), rows));
  hipError_t e = ensure_red(c, sizeof(double) * 2 * kDivWaves);
  if (e != hipSuccess) return e;
  if (f64) {
    auto k = vec ? div_kernel<double, 2> : div_kernel<double, 1>;
    hipLaunchKernelGGL(k, dim3(nb), dim3(threads), 0, s, (const double*)u, (const double*)v, (const double*)w,
                       c->hx64, c->areaw, c->hz64, c->nx, c->ny, c->nz, c->wx, c->wy, c->red);
  } else {
    auto k = vec ? div_kernel<float, 4> : div_kernel<float, 1>;
    hipLaunchKernelGGL(k, dim3(nb), dim3(threads), 0, s, (const float*)u, (const float*)v, (const float*)w,
                       c->hx64, c->areaw, c->hz64, c->nx, c->ny, c->nz, c->wx, c->wy, c->red);
  }
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
