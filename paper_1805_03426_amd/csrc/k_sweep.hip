// Column-sweep form of the scalar step (Eqs. 5-7 with the z diffusion
// implicit), pipelined across consecutive steps.
//
// The implicit z solve of step n is a Thomas solve per (x, y) column: an
// elimination sweep in one z direction, then a back substitution in the other.
// Here a sequence of steps n0 .. n0+count-1 runs as count + 1 kernels.  The
// kernel of step m walks every column once, level by level, in one z
// direction; at each level it
//   1. finishes theta^m there: the back substitution of step m-1, whose
//      elimination the previous kernel ran in the other direction (the first
//      kernel of a sequence reads theta^m itself);
//   2. exchanges the new theta^m row and the lagged theta^{m-1} row with the
//      rows beside it (LDS) and the columns beside it (lane shifts), and builds
//      the right-hand side of step m one level behind (it needs theta^m on the
//      level on either side): central-flux advection of theta^m, lagged x/y
//      diffusion of theta^{m-1}, leapfrog / start-up / averaging weights;
//   3. runs the elimination of step m in the walking direction in double and
//      writes its values e^m, and writes theta^m.
// The next kernel walks the other way.  A last kernel back-substitutes the
// final step.  Every cell of a step is read as 5 values (e^{m-1}, theta^{m-1},
// u, v, w) and written as 2 (theta^m, e^m); nothing else goes to memory, and
// no column is held whole anywhere, so the column height is not limited by
// registers.
//
// Workgroup: TX x TY wavefronts over a tile of 64 TX x columns by TY rows;
// lane l of the wavefront of segment c and row r owns column i0 + 64 c + l of
// row j0 + r.  The rows beside the tile (j0 - 1 and j0 + TY) are
// back-substituted by the wavefronts of the first and the last row as a
// second column each, the columns beside each segment (64 c - 1 and 64 c +
// 64) by its lanes 0 and 63 as one more column (the other lanes repeat their
// own column in the same instructions, which the cache serves).
// Lanes and rows past a ragged end take the periodic continuation and never
// store.  The step needs x and y periodic with uniform widths and the plain
// second-order method (no explicit z share, no fourth-order faces).
#include <string.h>

#include "mr_internal.h"

namespace mr {
namespace sweep {

template <typename T>
struct SweepArgs {
  const T* src;       // e^{m-1} (theta^m itself in the first kernel of a sequence)
  const T* lag;       // theta^{m-1} (theta^m at the start-up step)
  const T* u;
  const T* v;
  const T* w;
  T* th_out;          // theta^m (not written by the first kernel)
  T* e_out;           // e^m
  const double* cb;   // back substitution of step m-1: theta_k = e_k - cb_k theta_(level before k)
  const double* em;   // elimination of step m: e_k = em_k (r_k + tkb_k) + ea_k e_(level before k)
  const double* ea;
  const double* tkb;
  const T* ihz;
  const T* zlo;       // 1 where level k has an interior z face below
  const T* zhi;       // 1 where level k has an interior z face above
  T ap, ac, tau, tk;  // step m: weights of theta^{m-1}, theta^m; tau; tau kappa
  T tk0;              // reverse start-up step: tau_0 kappa on the x/y diffusion of mu^0 itself
  T uhx, uhy, uxx, uyy;
  int nx, ny, nz;
  int band;           // x tiles per band of the tile walk
};

// Loads from a wave-uniform level base at a 32-bit lane byte offset.
template <typename T>
__device__ __forceinline__ T ld(const T* base, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ T ld_nt(const T* base, unsigned off) {
  return __builtin_nontemporal_load(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off));
}
template <typename T>
__device__ __forceinline__ void st_nt(T* base, unsigned off, T v) {
  __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off));
}

// Per-level table values (the level is wave-uniform): read through the
// constant address space, so that they come by scalar loads and never hold up
// the vector loads in flight for the levels ahead.
template <typename T>
__device__ __forceinline__ T tab(const T* p, int k) {
  return ((const __attribute__((address_space(4))) T*)(p))[k];
}

__device__ __forceinline__ int dpp_shr(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_shl(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ float shr(float v) { return __int_as_float(dpp_shr(__float_as_int(v))); }
__device__ __forceinline__ float shl(float v) { return __int_as_float(dpp_shl(__float_as_int(v))); }
__device__ __forceinline__ double shr(double v) {
  const long long x = __double_as_longlong(v);
  return __longlong_as_double(((long long)dpp_shr((int)(x >> 32)) << 32) | (unsigned)dpp_shr((int)x));
}
__device__ __forceinline__ double shl(double v) {
  const long long x = __double_as_longlong(v);
  return __longlong_as_double(((long long)dpp_shl((int)(x >> 32)) << 32) | (unsigned)dpp_shl((int)x));
}

// What one level loads.
template <typename T>
struct Lv {
  T ec, ex, eh;   // e (or theta) of the own column, the edge column, the halo row
  T pc, px, ph;   // theta^{m-1} of the same three
  T u0, ue;       // u on face i; lane 63: face i0 + 64 (others: face i again)
  T v0, v1;       // v on faces j and j + 1
  T wf;           // w on the face of this level in the walking direction's rear
};

// One level of the right-hand side, kept from the level's own iteration to the
// next one (which completes its z stencil).
template <typename T>
struct Rh {
  T tc, txm, txp, tym, typ;   // theta^m and its x / y neighbours
  T pc, pxm, pxp, pym, pyp;   // theta^{m-1} and its x / y neighbours
  T u0, u1, v0, v1, wf;
};

template <typename T, int TX, int TY, bool DOWN, bool FIRST, int PF, bool REV>
__global__ void __launch_bounds__(64 * TX * TY) sweep_kernel(SweepArgs<T> A) {
  static_assert(TY >= 2, "the halo rows belong to two different wavefronts");
  constexpr int W = 64 * TX;          // tile width (TX wavefronts per row)
  __shared__ T shn[2][TY + 2][W];     // theta^m rows of a level (double-buffered by level parity)
  __shared__ T shp[2][TY + 2][W];     // theta^{m-1} rows
  const int lane = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int r = wv / TX, cx = wv - r * TX;   // tile row and 64-column segment of this wavefront
  const int lx = cx * 64 + lane;             // column inside the tile
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int ntx = (nx + W - 1) / W, nty = (ny + TY - 1) / TY;
  // tile walk: bands of A.band x tiles, walked row tile by row tile, x fastest
  // in a band; consecutive tiles of the walk go to one XCD
  const int t = xcd_remap(blockIdx.x, ntx * nty);
  const int per_band = A.band * nty;
  const int bnd = t / per_band;
  const int rt = t - bnd * per_band;
  const int wb = min(A.band, ntx - bnd * A.band);
  const int jt = rt / wb;
  const int xt = bnd * A.band + (rt - jt * wb);
  const int i_raw = xt * W + lx, j_raw = jt * TY + r;
  const bool act = i_raw < nx && j_raw < ny;
  const int i = i_raw % nx, j = j_raw % ny;
  const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
  const int jp = j == ny - 1 ? 0 : j + 1;
  // the edge column of lanes 0 and 63, the halo row of the first and last wavefront
  const int ie = lane == 0 ? im : (lane == 63 ? ip : i);
  const bool hlo = r == 0, hhi = r == TY - 1;
  const int jh = hlo ? (jt * TY + ny - 1) % ny : (hhi ? (jt * TY + TY) % ny : j);
  const int nxy = nx * ny;
  constexpr unsigned sz = sizeof(T);
  const unsigned oc = (unsigned)(j * nx + i) * sz, ox = (unsigned)(j * nx + ie) * sz;
  const unsigned oh = (unsigned)(jh * nx + i) * sz, oyp = (unsigned)(jp * nx + i) * sz;
  const unsigned oue = lane == 63 ? (unsigned)(j * nx + ip) * sz : oc;

  auto level = [&](int s) { return DOWN ? nz - 1 - s : s; };
  auto fetch = [&](int s) {
    Lv<T> f;
    const int k = level(min(s, nz - 1));
    const size_t base = (size_t)k * nxy;
    const T* e = A.src + base;
    const T* p = A.lag + base;
    f.ec = ld(e, oc);
    f.ex = ld(e, ox);
    f.pc = ld(p, oc);
    f.px = ld(p, ox);
    // the halo row (other wavefronts: their own row again, from the cache)
    f.eh = ld(e, oh);
    f.ph = ld(p, oh);
    f.u0 = ld(A.u + base, oc);
    f.ue = ld(A.u + base, oue);
    f.v0 = ld(A.v + base, oc);
    f.v1 = ld(A.v + base, oyp);
    // w on the face this level shares with the next level of the walk
    f.wf = ld_nt(A.w + (size_t)(DOWN ? k : k + 1) * nxy, oc);
    return f;
  };

  // back-substitution carries (double), the elimination carry, and the
  // right-hand-side pipeline: the level behind (q1) and the one behind it (t2)
  double bc = 0.0, bx = 0.0, bh = 0.0, ecar = 0.0;
  Rh<T> q1;
  T t2 = T(0), w2 = T(0);   // theta^m two levels behind (own column) and its rear w face
  const T half = T(0.5);

  // right-hand side and elimination of the level behind (s - 1), whose z
  // stencil closes with theta^m of the current level (tnext; masked at a wall)
  auto rhs = [&](int s1, T tnext) {
    const int k = level(s1);
    const T mlo = tab(A.zlo, k), mhi = tab(A.zhi, k);
    const T below = DOWN ? tnext : t2, above = DOWN ? t2 : tnext;
    const T wlo = DOWN ? q1.wf : w2, whi = DOWN ? w2 : q1.wf;
    T adv;
    if constexpr (REV) {
      // C_u^T mu: each face f (cells L, R) adds u_f (mu_R/h_R - mu_L/h_L)/2 to both cells
      const T ihzk = tab(A.ihz, k);
      const T czl = mlo * wlo * (q1.tc * ihzk - below * tab(A.ihz, k > 0 ? k - 1 : 0));
      const T czr = mhi * whi * (above * tab(A.ihz, k < nz - 1 ? k + 1 : nz - 1) - q1.tc * ihzk);
      adv = half * ((q1.u0 * (q1.tc - q1.txm) + q1.u1 * (q1.txp - q1.tc)) * A.uhx +
                    (q1.v0 * (q1.tc - q1.tym) + q1.v1 * (q1.typ - q1.tc)) * A.uhy + czl + czr);
    } else {
      const T fzl = mlo * wlo * (below + q1.tc);
      const T fzr = mhi * whi * (q1.tc + above);
      adv = -half * ((q1.u1 * (q1.tc + q1.txp) - q1.u0 * (q1.txm + q1.tc)) * A.uhx +
                     (q1.v1 * (q1.tc + q1.typ) - q1.v0 * (q1.tym + q1.tc)) * A.uhy + (fzr - fzl) * tab(A.ihz, k));
    }
    // the x/y diffusion of the second field (its transpose is itself on uniform widths)
    const T lap = (q1.pxp + q1.pxm - T(2) * q1.pc) * A.uxx + (q1.pyp + q1.pym - T(2) * q1.pc) * A.uyy;
    T rr = A.ap * q1.pc + A.ac * q1.tc + A.tau * adv + A.tk * lap;
    if constexpr (REV) {
      // the start-up step's reverse: its diffusion acts on theta^0, whose
      // adjoint this pass forms (tk0 = 0 for every other reverse step)
      rr += A.tk0 * ((q1.txp + q1.txm - T(2) * q1.tc) * A.uxx + (q1.typ + q1.tym - T(2) * q1.tc) * A.uyy);
    }
    ecar = tab(A.em, k) * ((double)rr + tab(A.tkb, k)) + tab(A.ea, k) * ecar;
    if (act) st_nt(A.e_out + (size_t)k * nxy, oc, (T)ecar);
  };

  // one level: finish theta^m, exchange, close the level behind
  auto work = [&](int s, const Lv<T>& cur) {
    const int k = level(s);
    // 1. theta^m on this level (own column, edge column, halo row)
    T tc, tx, th;
    if constexpr (FIRST) {
      tc = cur.ec;
      tx = cur.ex;
      th = cur.eh;
    } else {
      const double c = tab(A.cb, k);
      bc = (double)cur.ec - c * bc;
      bx = (double)cur.ex - c * bx;
      bh = (double)cur.eh - c * bh;
      tc = (T)bc;
      tx = (T)bx;
      th = (T)bh;
      if (act) st_nt(A.th_out + (size_t)k * nxy, oc, tc);
    }
    // 2. rows to LDS (double-buffered by level parity: one barrier per level)
    const int b = s & 1;
    shn[b][r + 1][lx] = tc;
    shp[b][r + 1][lx] = cur.pc;
    if (hlo) {
      shn[b][0][lx] = th;
      shp[b][0][lx] = cur.ph;
    }
    if (hhi) {
      shn[b][TY + 1][lx] = th;
      shp[b][TY + 1][lx] = cur.ph;
    }
    // 3. the level behind: its z stencil closes with this level's theta^m
    if (s > 0) {
      rhs(s - 1, tc);
      t2 = q1.tc;
      w2 = q1.wf;
    }
    __syncthreads();
    // 4. this level's stencil values: rows from LDS, columns by lane shifts
    q1.tc = tc;
    q1.tym = shn[b][r][lx];
    q1.typ = shn[b][r + 2][lx];
    q1.pym = shp[b][r][lx];
    q1.pyp = shp[b][r + 2][lx];
    const T tl = shr(tc), trr = shl(tc), pl = shr(cur.pc), pr = shl(cur.pc), ur = shl(cur.u0);
    q1.txm = lane == 0 ? tx : tl;
    q1.txp = lane == 63 ? tx : trr;
    q1.pc = cur.pc;
    q1.pxm = lane == 0 ? cur.px : pl;
    q1.pxp = lane == 63 ? cur.px : pr;
    q1.u0 = cur.u0;
    q1.u1 = lane == 63 ? cur.ue : ur;
    q1.v0 = cur.v0;
    q1.v1 = cur.v1;
    q1.wf = cur.wf;
  };

  // PF levels of loads in flight ahead of the level being worked on: a ring of
  // PF + 1 load sets, the loop unrolled over the ring so that every slot is a
  // fixed set of registers
  Lv<T> ring[PF + 1];
#pragma unroll
  for (int q = 0; q < PF; ++q) ring[q] = fetch(q);
  for (int s0 = 0; s0 < nz; s0 += PF + 1) {
#pragma unroll
    for (int u = 0; u <= PF; ++u) {
      const int s = s0 + u;
      if (s < nz) {
        ring[(u + PF) % (PF + 1)] = fetch(s + PF);
        work(s, ring[u]);
      }
    }
  }
  rhs(nz - 1, T(0));
}

// Back substitution of the last step of a sequence: theta_k = e_k - cb_k
// theta_(level before k), one lane per column.
template <typename T, bool DOWN>
__global__ void __launch_bounds__(256) backsub_kernel(const T* __restrict__ e, T* __restrict__ out,
                                                     const double* __restrict__ cb, int nxy, int nz) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= nxy) return;
  double x = 0.0;
#pragma unroll 8
  for (int s = 0; s < nz; ++s) {
    const int k = DOWN ? nz - 1 - s : s;
    const size_t o = (size_t)k * nxy + col;
    x = (double)__builtin_nontemporal_load(e + o) - tab(cb, k) * x;
    __builtin_nontemporal_store((T)x, out + o);
  }
}

// The adjoint's seed solve on columns the line solver cannot hold: the
// elimination walking up (its values stored in out), then the back
// substitution walking down, one lane per column.
template <typename T>
__global__ void __launch_bounds__(256) solve_kernel(const T* __restrict__ lam, T* __restrict__ out,
                                                   const double* __restrict__ m, const double* __restrict__ a,
                                                   const double* __restrict__ cb, int nxy, int nz) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= nxy) return;
  double e = 0.0;
  for (int k = 0; k < nz; ++k) {
    const size_t o = (size_t)k * nxy + col;
    e = tab(m, k) * (double)lam[o] + tab(a, k) * e;
    out[o] = (T)e;
  }
  double x = 0.0;
  for (int k = nz - 1; k >= 0; --k) {
    const size_t o = (size_t)k * nxy + col;
    x = (double)out[o] - tab(cb, k) * x;
    out[o] = (T)x;
  }
}

}  // namespace sweep

namespace {
using namespace sweep;

// Tile shapes, in the order each precision prefers them: FP64 256 x 4, 192 x 4,
// 128 x 8, 64 x 16; FP32 128 x 8, 192 x 4, 64 x 16.  The first whose
// width divides N_x is taken (else the one that leaves the fewest idle
// lanes): lanes past a ragged end still load, so a ragged tile costs reads.
// Timed in one run at 1024 x 1024 x 512: in FP64 the shapes were within 2%
// (5.78 ms per step for 256 x 4), in FP32 the 128- and 256-wide tiles took
// 2.66-2.75 ms against 2.93-3.14 ms for 64 x 16 (longer contiguous rows per
// level).  At 576^3 (M = 3), 192 x 4 took 2.36 ms (FP64) and 1.00 ms (FP32)
// against 2.84 and 1.26 ms for the ragged 256 x 4 and 128 x 8 and 2.51 and
// 1.17 ms for 64 x 8.  Tiles are walked in bands of 4 x tiles in FP64, 8 in
// FP32; loads run one level ahead in FP64 and three in FP32 (two ahead in
// FP64, 128 VGPRs, was 14% slower).
constexpr int kOrder64[] = {0, 1, 2, 3};
constexpr int kOrder32[] = {2, 1, 3};   // 256 x 4 in FP32 was no faster than 128 x 8

template <typename T>
struct SweepTile {
  static constexpr bool f64 = sizeof(T) == 8;
  static constexpr int band = f64 ? 4 : 8;   // x tiles per band of the tile walk
  static constexpr int pf = f64 ? 1 : 3;     // levels of loads ahead
};

template <typename T>
const Geom<T>& geom(const mr_ctx* c);
template <>
const Geom<double>& geom<double>(const mr_ctx* c) { return c->g64; }
template <>
const Geom<float>& geom<float>(const mr_ctx* c) { return c->g32; }

template <typename T, int TX, int TY, bool REV>
hipError_t launch_shape(int nx, int ny, bool first, bool down, SweepArgs<T>& a, hipStream_t s) {
  constexpr int PF = SweepTile<T>::pf;
  const int ntx = (nx + 64 * TX - 1) / (64 * TX), nty = (ny + TY - 1) / TY;
  a.band = SweepTile<T>::band < ntx ? SweepTile<T>::band : ntx;
  const dim3 grid((unsigned)(ntx * nty)), block(64, TX * TY);
  if (first) {
    if (down) hipLaunchKernelGGL((sweep_kernel<T, TX, TY, true, true, PF, REV>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((sweep_kernel<T, TX, TY, false, true, PF, REV>), grid, block, 0, s, a);
  } else {
    if (down) hipLaunchKernelGGL((sweep_kernel<T, TX, TY, true, false, PF, REV>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((sweep_kernel<T, TX, TY, false, false, PF, REV>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

// The launch of one sweep in the context's tile shape.
template <typename T, bool REV>
hipError_t launch_tiles(mr_ctx* c, bool first, bool down, SweepArgs<T>& a, hipStream_t s) {
  switch (c->sweep_shape) {
    case 0:
      if constexpr (sizeof(T) == 8)
        return launch_shape<T, kSweepShape[0].segs, kSweepShape[0].rows, REV>(c->nx, c->ny, first, down, a, s);
      return hipErrorInvalidValue;   // not an FP32 shape
    case 1: return launch_shape<T, kSweepShape[1].segs, kSweepShape[1].rows, REV>(c->nx, c->ny, first, down, a, s);
    case 2: return launch_shape<T, kSweepShape[2].segs, kSweepShape[2].rows, REV>(c->nx, c->ny, first, down, a, s);
    default: return launch_shape<T, kSweepShape[3].segs, kSweepShape[3].rows, REV>(c->nx, c->ny, first, down, a, s);
  }
}

template <typename T>
hipError_t sweep_t(mr_ctx* c, int64_t m, bool first, bool down, const void* src, const void* lag,
                   void* th_out, void* e_out, const void* u, const void* v, const void* w,
                   hipStream_t s) {
  const int kind = step_kind(m, c->n_avg);
  const Geom<T>& g = geom<T>(c);
  SweepArgs<T> a;
  ::memset((void*)&a, 0, sizeof(a));
  a.src = (const T*)src;
  a.lag = (const T*)lag;
  a.u = (const T*)u;
  a.v = (const T*)v;
  a.w = (const T*)w;
  a.th_out = (T*)th_out;
  a.e_out = (T*)e_out;
  if (!first) {
    // the previous kernel eliminated step m-1 walking the other way
    const SweepSys& pz = c->sw[step_kind(m - 1, c->n_avg)];
    a.cb = down ? pz.up_cb : pz.dn_cb;
  }
  const SweepSys& z = c->sw[kind];
  a.em = down ? z.dn_m : z.up_m;
  a.ea = down ? z.dn_a : z.up_a;
  a.tkb = z.tkb;
  a.ihz = g.ihz;
  a.zlo = g.zlo;
  a.zhi = g.zhi;
  a.ap = (T)alpha_prev(kind);
  a.ac = (T)alpha_cur(kind);
  a.tau = (T)c->tau[kind];
  a.tk = (T)(c->tau[kind] * c->kappa);
  a.uhx = (T)c->uhx;
  a.uhy = (T)c->uhy;
  a.uxx = (T)(c->uhx * c->uhx);
  a.uyy = (T)(c->uhy * c->uhy);
  a.nx = c->nx;
  a.ny = c->ny;
  a.nz = c->nz;
  return launch_tiles<T, false>(c, first, down, a, s);
}

template <typename T>
hipError_t backsub_t(mr_ctx* c, int64_t m, bool down, const void* e, void* out, hipStream_t s) {
  const SweepSys& z = c->sw[step_kind(m, c->n_avg)];
  // step m was eliminated walking the other way
  const double* cb = down ? z.up_cb : z.dn_cb;
  const int nxy = c->nx * c->ny;
  const dim3 grid((unsigned)((nxy + 255) / 256)), block(256);
  if (down) hipLaunchKernelGGL((backsub_kernel<T, true>), grid, block, 0, s, (const T*)e, (T*)out, cb, nxy, c->nz);
  else hipLaunchKernelGGL((backsub_kernel<T, false>), grid, block, 0, s, (const T*)e, (T*)out, cb, nxy, c->nz);
  return hipGetLastError();
}

// The reverse step n as a sweep, in the adjoint's mu form: the transposed
// stencils of step n applied to mu^n, the transposed lagged x/y diffusion of
// step n+1 applied to mu^{n+1} (absent after the last step: zero weights),
// then the elimination of the transposed implicit system of step n-1, whose
// solution is mu^{n-1}.  Walking the other way, the next kernel back-
// substitutes it.
template <typename T>
hipError_t sweep_bwd_t(mr_ctx* c, int64_t n, bool first, bool down, bool has_next, const void* src,
                       const void* lag, void* mu_out, void* e_out, const void* u, const void* v, const void* w,
                       hipStream_t s) {
  const int kind = step_kind(n, c->n_avg);
  const Geom<T>& g = geom<T>(c);
  SweepArgs<T> a;
  ::memset((void*)&a, 0, sizeof(a));
  a.src = (const T*)src;
  a.lag = (const T*)lag;
  a.u = (const T*)u;
  a.v = (const T*)v;
  a.w = (const T*)w;
  a.th_out = (T*)mu_out;
  a.e_out = (T*)e_out;
  if (!first) {
    // the previous kernel eliminated the system of mu^n (the transpose of
    // step n's) walking the other way
    const SweepSys& pz = c->swt[kind];
    a.cb = down ? pz.up_cb : pz.dn_cb;
  }
  // n = 0 (the start-up step's reverse): no solve, the right-hand side is
  // the adjoint of theta^0 itself (identity factors: e_k = r_k)
  const SweepSys& z = n > 0 ? c->swt[step_kind(n - 1, c->n_avg)] : c->swid;
  a.em = down ? z.dn_m : z.up_m;
  a.ea = down ? z.dn_a : z.up_a;
  a.tkb = z.tkb;
  if (n == 0) a.tk0 = (T)(c->tau[kind] * c->kappa);
  a.ihz = g.ihz;
  a.zlo = g.zlo;
  a.zhi = g.zhi;
  a.ac = (T)alpha_cur(kind);
  a.tau = (T)c->tau[kind];
  if (has_next) {
    const int k1 = step_kind(n + 1, c->n_avg);
    a.ap = (T)alpha_prev(k1);
    a.tk = (T)(c->tau[k1] * c->kappa);
  }
  a.uhx = (T)c->uhx;
  a.uhy = (T)c->uhy;
  a.uxx = (T)(c->uhx * c->uhx);
  a.uyy = (T)(c->uhy * c->uhy);
  a.nx = c->nx;
  a.ny = c->ny;
  a.nz = c->nz;
  return launch_tiles<T, true>(c, first, down, a, s);
}

template <typename T>
hipError_t backsub_bwd_t(mr_ctx* c, int64_t n, bool down, const void* e, void* out, hipStream_t s) {
  // mu^{n-1} was eliminated (transpose of step n-1) walking the other way
  const SweepSys& z = c->swt[step_kind(n - 1, c->n_avg)];
  const double* cb = down ? z.up_cb : z.dn_cb;
  const int nxy = c->nx * c->ny;
  const dim3 grid((unsigned)((nxy + 255) / 256)), block(256);
  if (down) hipLaunchKernelGGL((backsub_kernel<T, true>), grid, block, 0, s, (const T*)e, (T*)out, cb, nxy, c->nz);
  else hipLaunchKernelGGL((backsub_kernel<T, false>), grid, block, 0, s, (const T*)e, (T*)out, cb, nxy, c->nz);
  return hipGetLastError();
}

}  // namespace

int sweep_pick_shape(int nx, bool fp64) {
  const int* order = fp64 ? kOrder64 : kOrder32;
  const int n = fp64 ? (int)(sizeof(kOrder64) / sizeof(int)) : (int)(sizeof(kOrder32) / sizeof(int));
  int best = order[0];
  int64_t best_idle = -1;
  for (int q = 0; q < n; ++q) {
    const int w = 64 * kSweepShape[order[q]].segs;
    const int64_t idle = (int64_t)(nx + w - 1) / w * w - nx;
    if (idle == 0) return order[q];
    if (best_idle < 0 || idle < best_idle) {
      best = order[q];
      best_idle = idle;
    }
  }
  return best;
}

bool sweep_supported(const mr_ctx* c) {
  return c->uniform_xy && !c->wx && !c->wy && c->z_explicit == 0.0 && c->face_order == 2;
}

hipError_t ensure_sweep_buffers(mr_ctx* c) {
  const size_t need = (c->precision == MR_FP64 ? 8 : 4) * (size_t)c->nx * c->ny * c->nz;
  for (int q = 0; q < 2; ++q) {
    if (c->sweep_e[q]) continue;
    hipError_t e = hipMalloc(&c->sweep_e[q], need);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_sweep_step(mr_ctx* c, int64_t n0, int q, const void* lag, const void* src0,
                             void* th_out, const void* u, const void* v, const void* w, hipStream_t s) {
  hipError_t e = ensure_sweep_buffers(c);
  if (e != hipSuccess) return e;
  // step n0 + q walks down for even q; its elimination values go to buffer q % 2
  const int64_t m = n0 + q;
  const bool down = (q & 1) == 0;
  const void* src = q == 0 ? src0 : c->sweep_e[(q - 1) & 1];
  return c->precision == MR_FP64
             ? sweep_t<double>(c, m, q == 0, down, src, lag, q == 0 ? nullptr : th_out, c->sweep_e[q & 1], u, v,
                               w, s)
             : sweep_t<float>(c, m, q == 0, down, src, lag, q == 0 ? nullptr : th_out, c->sweep_e[q & 1], u, v,
                              w, s);
}

hipError_t launch_sweep_finish(mr_ctx* c, int64_t n0, int count, void* out, hipStream_t s) {
  // the last step (q = count - 1) was eliminated walking down for even q:
  // its back substitution walks up
  const int64_t last = n0 + count - 1;
  const bool down = ((count - 1) & 1) != 0;
  const void* e = c->sweep_e[(count - 1) & 1];
  return c->precision == MR_FP64 ? backsub_t<double>(c, last, down, e, out, s)
                                 : backsub_t<float>(c, last, down, e, out, s);
}

hipError_t launch_sweep_steps(mr_ctx* c, int64_t n0, int count, const void* thp, const void* thc,
                              void* const* outs, const void* u, const void* v, const void* w,
                              hipStream_t s) {
  for (int q = 0; q < count; ++q) {
    // step n0 + q reads theta^{n0+q-1} as its lagged level and finishes theta^{n0+q}
    const void* lag = q == 0 ? thp : (q == 1 ? thc : outs[q - 2]);
    hipError_t e = launch_sweep_step(c, n0, q, lag, thc, q == 0 ? nullptr : outs[q - 1], u, v, w, s);
    if (e != hipSuccess) return e;
  }
  return launch_sweep_finish(c, n0, count, outs[count - 1], s);
}

hipError_t launch_sweep_bwd_steps(mr_ctx* c, int64_t n0, int count, const void* mu_next, const void* mu_cur,
                                  void* const* outs, const void* u, const void* v, const void* w, hipStream_t s) {
  hipError_t e = ensure_sweep_buffers(c);
  if (e != hipSuccess) return e;
  const bool f64 = c->precision == MR_FP64;
  for (int q = 0; q < count; ++q) {
    // reverse step n0 - q reads mu^{n0-q+1} as its second field and finishes
    // mu^{n0-q} (q > 0); its elimination (of mu^{n0-q-1}) goes to buffer q % 2
    const int64_t n = n0 - q;
    const bool down = (q & 1) == 0, first = q == 0;
    const void* src = first ? mu_cur : c->sweep_e[(q - 1) & 1];
    const void* lag = q == 0 ? (mu_next ? mu_next : mu_cur) : (q == 1 ? mu_cur : outs[q - 2]);
    const bool has_next = q > 0 || mu_next != nullptr;
    void* out = first ? nullptr : outs[q - 1];
    e = f64 ? sweep_bwd_t<double>(c, n, first, down, has_next, src, lag, out, c->sweep_e[q & 1], u, v, w, s)
            : sweep_bwd_t<float>(c, n, first, down, has_next, src, lag, out, c->sweep_e[q & 1], u, v, w, s);
    if (e != hipSuccess) return e;
  }
  const int64_t last = n0 - count + 1;
  const bool down = ((count - 1) & 1) != 0;
  const void* el = c->sweep_e[(count - 1) & 1];
  return f64 ? backsub_bwd_t<double>(c, last, down, el, outs[count - 1], s)
             : backsub_bwd_t<float>(c, last, down, el, outs[count - 1], s);
}

hipError_t launch_sweep_bwd0(mr_ctx* c, const void* mu_next, const void* mu_cur, void* out, const void* u,
                             const void* v, const void* w, hipStream_t s) {
  // one pass walking down that reads mu^0 itself and writes the right-hand side
  const void* lag = mu_next ? mu_next : mu_cur;
  return c->precision == MR_FP64
             ? sweep_bwd_t<double>(c, 0, true, true, mu_next != nullptr, mu_cur, lag, nullptr, out, u, v, w, s)
             : sweep_bwd_t<float>(c, 0, true, true, mu_next != nullptr, mu_cur, lag, nullptr, out, u, v, w, s);
}

hipError_t launch_sweep_seed(mr_ctx* c, int64_t n, const void* lam, void* out, hipStream_t s) {
  const SweepSys& z = c->swt[step_kind(n, c->n_avg)];
  const int nxy = c->nx * c->ny;
  const dim3 grid((unsigned)((nxy + 255) / 256)), block(256);
  if (c->precision == MR_FP64)
    hipLaunchKernelGGL(solve_kernel<double>, grid, block, 0, s, (const double*)lam, (double*)out, z.up_m, z.up_a,
                       z.up_cb, nxy, c->nz);
  else
    hipLaunchKernelGGL(solve_kernel<float>, grid, block, 0, s, (const float*)lam, (float*)out, z.up_m, z.up_a,
                       z.up_cb, nxy, c->nz);
  return hipGetLastError();
}

}  // namespace mr
