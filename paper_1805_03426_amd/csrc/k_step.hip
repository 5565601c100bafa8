// Scalar step kernels: the fused forward step (Eqs. 5-7 with the z diffusion
// implicit), its fused reverse step, the transposed solve that seeds the
// reverse sweep, and the velocity-gradient accumulation.
//
// Layout of one workgroup: 64 lanes = 64 consecutive x columns (coalesced
// x-fastest rows), one wavefront per z chunk of L levels, one y row.  Each
// lane builds the right-hand side of its L cells from the stencil (x and y
// neighbours from the cache, z neighbours carried in registers while it walks
// up the chunk), runs the forward elimination and back substitution of its
// chunk in double from zero boundary values, and keeps the L results in
// registers.  The chunks of one column are then coupled through two scalars
// per chunk (the elimination value entering from below, the solution value
// entering from above) exchanged in LDS, and every cell gets its exact value
// x = x_hat + D G + X B (G, B precomputed because the matrix is the same for
// every line).  Each cell is read once and written once: no intermediate
// field goes back to HBM.
//
// Optionally a share w of the z diffusion is explicit on the lagged level
// (w = 1/2: Crank-Nicolson across the step's time span): the solved system is
// I - (1-w) tau kappa Lz0, and the right-hand side gains w tau kappa Lz0
// applied to the lagged level (the reverse step: its transpose applied to the
// adjoint of the step that reads the level as its lag).
#include <string.h>

#include "mr_internal.h"

namespace mr {
namespace {

enum Mode { FWD = 0, BWD = 1, BWD0 = 2, SEED = 3 };

template <typename T>
struct LineArgs {
  const T* a0;   // FWD: theta^{n-1} (lag);  BWD/BWD0: mu^n;          SEED: lambda
  const T* a1;   // FWD: theta^n;           BWD/BWD0: mu^{n+1} (mu^n when absent)
  const T* a2;   // BWD/BWD0: lam_add (mu^n when absent)
  const T* u;
  const T* v;
  const T* w;
  T* out;
  Geom<T> g;
  ZSys z;        // system solved for the output (FWD: step n; BWD: transpose of step n-1)
  T ap, ac, tau, tk;   // FWD: step n;  BWD: a_c(n), tau_n, tau_n kappa (ap unused)
  T ap1, tk1;          // BWD: a_p(n+1), tau_{n+1} kappa (0 when there is no step n+1)
  T tkw, tkw1;         // w tk and w tk1: explicit share of the z diffusion (EXPZ kernels)
  T s2;                // BWD: 1 with lam_add, 0 without
  int nx, ny, nz, nch;
  int band;            // x tiles per band of the tile walk (see line_kernel)
  int wx, wy;          // x / y bounded by adiabatic no-slip walls (else periodic)
};

// Values one z level of the stencil reads.
template <typename T>
struct Lvl {
  T zp, w1;                 // z-stencil field one level up; w on the face above
  T xm, xp, ym, yp;         // x/y neighbours of the z-stencil field
  T u0, u1, v0, v1;         // u on faces i, i+1; v on faces j, j+1
  T pc, pxm, pxp, pym, pyp; // second field (theta^{n-1} or mu^{n+1}) and its x/y neighbours
  T pzp;                    // second field one level up (EXPZ only)
  T q;                      // lam_add (reverse step)
};

// Load from a wave-uniform base at a 32-bit byte offset (scalar base + vector
// offset addressing).
template <typename T>
__device__ __forceinline__ T ldb(const T* base, unsigned boff) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
}

template <typename T>
__device__ __forceinline__ void stb(T* base, unsigned boff, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff) = v;
}

// Whole-wavefront lane shifts (DPP wave_shr:1 / wave_shl:1): lane l receives
// the value of lane l-1 (shr) or l+1 (shl); the lane with no source keeps its
// own value, which every caller replaces.
__device__ __forceinline__ int dpp_shr_i(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_shl_i(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ float lane_shr(float v) { return __int_as_float(dpp_shr_i(__float_as_int(v))); }
__device__ __forceinline__ float lane_shl(float v) { return __int_as_float(dpp_shl_i(__float_as_int(v))); }
__device__ __forceinline__ double lane_shr(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = dpp_shr_i((int)x), hi = dpp_shr_i((int)(x >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_shl(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = dpp_shl_i((int)x), hi = dpp_shl_i((int)(x >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

#ifndef MR_XDPP
#define MR_XDPP 1
#endif

// A wavefront covers 64/ROWS columns of ROWS consecutive y rows.  With
// ROWS > 1 the y neighbours inside the patch are other lanes' centre values
// (cross-lane shuffles), and one load per field fetches the two halo rows
// (the row below the patch for its first row, the row above for its last).
// The x neighbours are the centre values of the lanes beside it (lane
// shifts); only the first and last column of each row load their outer
// neighbour, in the same load instruction in which the other lanes re-read
// their own (already cached) centre.  Lanes past the end of a ragged row take
// the periodic continuation of the row (column i mod nx), so the lane after
// the last column holds column 0, the periodic right neighbour of the last
// column; such lanes never store.
// Side walls: on a walled axis the neighbour across a wall is the cell itself
// (lanes past the end repeat the last column), so no diffusive flux crosses
// it, and the velocity on the wall faces is taken as zero, so no advective
// flux crosses it either.
//
// Tile walk: the x tiles are grouped into bands of A.band tiles; a band is
// walked row patch by row patch, x fastest inside the band.  Workgroups that
// run together on one XCD (consecutive after the XCD remap) then cover a few
// tiles in x and many rows in y, so the y neighbour rows of one workgroup are
// the centre rows of another that reads them at nearly the same time (L2
// hits), while the lines holding the x halo of a tile are shared with the
// tiles beside it in the band.
//
// EXPZ: the second field (the lagged level, or the adjoint of the step that
// reads this level as its lag) also needs its z neighbours: the level above is
// one more load per level, which is the next level's centre value (reused
// there instead of loaded again), and the level below is carried.
template <typename T, int L, int MODE, int ROWS, int MINB, int PFD, bool WALLS, bool EXPZ>
__global__ void __launch_bounds__(1024, MINB) line_kernel(LineArgs<T> A) {
  static_assert(!(EXPZ && MODE == SEED), "the seed solve has no explicit part");
  __shared__ double sh[4][kMaxChunks][kWave];
  constexpr int COLS = kWave / ROWS;
  const int lane = threadIdx.x;
  const int c = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int ntx = (nx + COLS - 1) / COLS, nty = (ny + ROWS - 1) / ROWS;
  const int t = xcd_remap(blockIdx.x, ntx * nty);
  const int per_band = A.band * nty;
  const int bnd = t / per_band;
  const int rt = t - bnd * per_band;
  const int wb = min(A.band, ntx - bnd * A.band);   // the last band may be narrower
  const int jt = rt / wb;
  const int xt = bnd * A.band + (rt - jt * wb);
  const int hrow = lane / COLS;
  const int i_raw = xt * COLS + lane % COLS;
  const int j_raw = jt * ROWS + hrow;
  const bool act = i_raw < nx && j_raw < ny;
  const bool wx = WALLS && A.wx, wy = WALLS && A.wy;
  const int i = wx ? min(i_raw, nx - 1) : i_raw % nx;
  // a row past the last one wraps around (periodic) or repeats the last row
  // (walls), so that the other half still sees the right neighbour row; its
  // results are not stored
  const int j = wy ? min(j_raw, ny - 1) : j_raw % ny;
  const int im = i == 0 ? (wx ? 0 : nx - 1) : i - 1;
  const int ip = i == nx - 1 ? (wx ? nx - 1 : 0) : i + 1;
  const int jm = j == 0 ? (wy ? 0 : ny - 1) : j - 1;
  const int jp = j == ny - 1 ? (wy ? ny - 1 : 0) : j + 1;
  // side faces that are walls (their velocity is taken as zero)
  const bool zu0 = wx && i == 0, zu1 = wx && i == nx - 1;
  const bool zv0 = wy && j == 0, zv1 = wy && j == ny - 1;
  const int nxy = nx * ny;
  const int k0 = c * L;
  // offsets of the stencil points inside one z level; a level's base pointer
  // is wave-uniform, so every load is scalar base + 32-bit lane offset
  constexpr unsigned sz = sizeof(T);
  const unsigned oc = (j * nx + i) * sz, oxm = (j * nx + im) * sz, oxp = (j * nx + ip) * sz;
  const unsigned oym = (jm * nx + i) * sz, oyp = (jp * nx + i) * sz;
  // ROWS > 1: the halo row of the patch (below for its first row, above otherwise)
  const unsigned ohalo = hrow == 0 ? oym : oyp;
  // first / last column of a row: its outer x neighbour; other lanes: their centre
  const int col = lane % COLS;
  const bool xfirst = col == 0, xlast = col == COLS - 1;
  const unsigned oedge = xfirst ? oxm : (xlast ? oxp : oc);
  const unsigned oedge_r = xlast ? oxp : oc;
  const int lane_dn = (lane - COLS) & (kWave - 1), lane_up = (lane + COLS) & (kWave - 1);
  const Geom<T>& g = A.g;

  const T ihx = g.ihx[i], ihxm = g.ihx[im], ihxp = g.ihx[ip];
  const T idx0 = g.idxc[i], idx1 = g.idxc[ip];
  const T ihy = g.ihy[j], ihym = g.ihy[jm], ihyp = g.ihy[jp];
  const T idy0 = g.idyc[j], idy1 = g.idyc[jp];
  const T half = T(0.5);

  double d[L];
  double dprev = 0.0;
  // field whose z neighbours the stencil needs (theta^n or mu^n), carried up the chunk
  const T* f = MODE == FWD ? A.a1 : A.a0;
  // second stencil field: theta^{n-1} (FWD) or mu^{n+1} (BWD, a0 with zero weights if absent)
  const T* p = MODE == FWD ? A.a0 : A.a1;
  T zm = T(0), zc = T(0), w0 = T(0);
  T pzm = T(0), pnext = T(0);
  if (MODE != SEED) {
    zc = ldb(f + k0 * nxy, oc);
    zm = ldb(f + max(k0 - 1, 0) * nxy, oc);
    w0 = ldb(A.w + k0 * nxy, oc);
    if constexpr (EXPZ) pzm = ldb(p + max(k0 - 1, 0) * nxy, oc);
  }

  // All loads of level k0 + kk.  Rows k >= nz (padding of the last chunk) read
  // the top level; their values never reach a real row (decoupled identity rows).
  auto fetch = [&](int kk) {
    Lvl<T> v;
    const int k = k0 + kk;
    const int kc = min(k, nz - 1);
    if (MODE == SEED) {
      v.pc = ldb(A.a0 + kc * nxy, oc);
      return v;
    }
    const T* fk = f + kc * nxy;
    const T* uk = A.u + kc * nxy;
    const T* vk = A.v + kc * nxy;
    const T* pk = p + kc * nxy;
    v.zp = ldb(f + min(k + 1, nz - 1) * nxy, oc);
    v.w1 = ldb(A.w + (kc + 1) * nxy, oc);
    if constexpr (MR_XDPP) {
      v.xm = ldb(fk, oedge);     // edge values, resolved after the lane shifts
      v.u1 = ldb(uk, oedge_r);
      v.pxm = ldb(pk, oedge);
    } else {
      v.xm = ldb(fk, oxm); v.xp = ldb(fk, oxp);
      v.u1 = ldb(uk, oxp);
      v.pxm = ldb(pk, oxm); v.pxp = ldb(pk, oxp);
    }
    v.u0 = ldb(uk, oc);
    v.v0 = ldb(vk, oc); v.v1 = ldb(vk, oyp);
    if constexpr (EXPZ) {
      // levels are fetched in order, so pnext holds this level's centre value
      v.pc = kk > 0 ? pnext : ldb(pk, oc);
      v.pzp = ldb(p + min(k + 1, nz - 1) * nxy, oc);
      pnext = v.pzp;
    } else {
      v.pc = ldb(pk, oc);
    }
    if constexpr (ROWS == 1) {
      v.ym = ldb(fk, oym); v.yp = ldb(fk, oyp);
      v.pym = ldb(pk, oym); v.pyp = ldb(pk, oyp);
    } else {
      v.ym = ldb(fk, ohalo);   // halo row of f (resolved to ym/yp below)
      v.pym = ldb(pk, ohalo);  // halo row of p
    }
    if (MODE != FWD) v.q = ldb(A.a2 + kc * nxy, oc);
    return v;
  };

  // PFD levels ahead of the one being computed have their loads in flight
  Lvl<T> cur = fetch(0);
  Lvl<T> n1, n2;
  if (PFD >= 2 && L > 1) n1 = fetch(1);
#pragma unroll
  for (int kk = 0; kk < L; ++kk) {
    const int k = k0 + kk;
    const int kc = min(k, nz - 1);
    if (PFD == 1 && kk + 1 < L) n1 = fetch(kk + 1);
    if (PFD == 2 && kk + 2 < L) n2 = fetch(kk + 2);
    T r;
    if (MODE == SEED) {
      r = cur.pc;
    } else {
      if constexpr (MR_XDPP) {
        const T fe = cur.xm, pe = cur.pxm, ue = cur.u1;
        const T fl = lane_shr(zc), fr = lane_shl(zc);
        const T pl = lane_shr(cur.pc), pr = lane_shl(cur.pc);
        const T ur = lane_shl(cur.u0);
        cur.xm = xfirst ? fe : fl;
        cur.xp = xlast ? fe : fr;
        cur.pxm = xfirst ? pe : pl;
        cur.pxp = xlast ? pe : pr;
        cur.u1 = xlast ? ue : ur;
      }
      if constexpr (ROWS > 1) {
        const T fdn = __shfl(zc, lane_dn), fup = __shfl(zc, lane_up);
        const T pdn = __shfl(cur.pc, lane_dn), pup = __shfl(cur.pc, lane_up);
        const T fh = cur.ym, ph = cur.pym;
        cur.ym = hrow == 0 ? fh : fdn;
        cur.yp = hrow == ROWS - 1 ? fh : fup;
        cur.pym = hrow == 0 ? ph : pdn;
        cur.pyp = hrow == ROWS - 1 ? ph : pup;
      }
      if constexpr (WALLS) {
        // wall faces carry no velocity (lane selects, branch-free)
        cur.u0 = zu0 ? T(0) : cur.u0;
        cur.u1 = zu1 ? T(0) : cur.u1;
        cur.v0 = zv0 ? T(0) : cur.v0;
        cur.v1 = zv1 ? T(0) : cur.v1;
      }
      const T zp = cur.zp, w1 = cur.w1;
      const T ihz = g.ihz[kc];
      const T mlo = g.zlo[k], mhi = g.zhi[k];
      if (MODE == FWD) {
        // central-flux advection of theta^n (face value = mean of the two cells)
        const T fzl = mlo * w0 * (zm + zc);
        const T fzr = mhi * w1 * (zc + zp);
        const T adv = -half * ((cur.u1 * (zc + cur.xp) - cur.u0 * (cur.xm + zc)) * ihx +
                               (cur.v1 * (zc + cur.yp) - cur.v0 * (cur.ym + zc)) * ihy + (fzr - fzl) * ihz);
        // lagged x/y diffusion of theta^{n-1}
        const T lap = ((cur.pxp - cur.pc) * idx1 - (cur.pc - cur.pxm) * idx0) * ihx +
                      ((cur.pyp - cur.pc) * idy1 - (cur.pc - cur.pym) * idy0) * ihy;
        r = A.ap * cur.pc + A.ac * zc + A.tau * adv + A.tk * lap;
        if constexpr (EXPZ)   // explicit share of the z diffusion of the lagged level
          r += A.tkw * (g.lzd[k] * cur.pc + g.lzl[k] * pzm + g.lzh[k] * cur.pzp);
      } else {
        // C_u^T mu^n: each face f (cells L, R) adds u_f (mu_R/h_R - mu_L/h_L)/2 to both cells
        const T qc_x = zc * ihx, qc_y = zc * ihy, qc_z = zc * ihz;
        const T czl = mlo * w0 * (qc_z - zm * g.ihz[max(kc - 1, 0)]);
        const T czr = mhi * w1 * (zp * g.ihz[min(kc + 1, nz - 1)] - qc_z);
        const T cu = half * (cur.u0 * (qc_x - cur.xm * ihxm) + cur.u1 * (cur.xp * ihxp - qc_x) +
                             cur.v0 * (qc_y - cur.ym * ihym) + cur.v1 * (cur.yp * ihyp - qc_y) + czl + czr);
        // contribution of step n+1 through theta^n as its lagged level
        const T qx = cur.pc * ihx, qy = cur.pc * ihy;
        const T lt = ((cur.pxm * ihxm - qx) * idx0 - (qx - cur.pxp * ihxp) * idx1) +
                     ((cur.pym * ihym - qy) * idy0 - (qy - cur.pyp * ihyp) * idy1);
        r = A.ac * zc + A.tau * cu + A.ap1 * cur.pc + A.tk1 * lt + A.s2 * cur.q;
        if (MODE == BWD0) {
          // the start-up step also reads theta^0 for its diffusion
          const T l0 = ((cur.xm * ihxm - qc_x) * idx0 - (qc_x - cur.xp * ihxp) * idx1) +
                       ((cur.ym * ihym - qc_y) * idy0 - (qc_y - cur.yp * ihyp) * idy1);
          r += A.tk * l0;
          if constexpr (EXPZ) r += A.tkw * (g.lzd[k] * zc + g.lztl[k] * zm + g.lzth[k] * zp);
        }
        if constexpr (EXPZ)   // step n+1's explicit z share, transposed, through its lag
          r += A.tkw1 * (g.lzd[k] * cur.pc + g.lztl[k] * pzm + g.lzth[k] * cur.pzp);
      }
      zm = zc;
      zc = zp;
      w0 = w1;
      if constexpr (EXPZ) pzm = cur.pc;
    }
    if (MODE == BWD0) {
      if (act && k < nz) stb(A.out + k * nxy, oc, r);
    } else {
      dprev = A.z.m[k] * ((double)r + A.z.tkb[k]) + A.z.a[k] * dprev;
      d[kk] = dprev;
    }
    if (kk + 1 < L) {
      if (PFD == 0) {
        cur = fetch(kk + 1);
      } else {
        cur = n1;
        if (PFD == 2) n1 = n2;
      }
    }
  }
  if (MODE == BWD0) return;

  // local back substitution from a zero value above the chunk
  double xh = 0.0;
#pragma unroll
  for (int kk = L - 1; kk >= 0; --kk) {
    xh = d[kk] - A.z.cp[k0 + kk] * xh;
    d[kk] = xh;
  }
  sh[0][c][lane] = dprev;  // elimination value at the top of the chunk
  sh[1][c][lane] = xh;     // local solution at the bottom of the chunk
  __syncthreads();
  if (c == 0) {
    double D = 0.0;
    for (int cc = 0; cc < A.nch; ++cc) {
      sh[2][cc][lane] = D;
      D = sh[0][cc][lane] + A.z.Fe[cc] * D;
    }
    double X = 0.0;
    for (int cc = A.nch - 1; cc >= 0; --cc) {
      sh[3][cc][lane] = X;
      X = sh[1][cc][lane] + sh[2][cc][lane] * A.z.Gs[cc] + X * A.z.Bs[cc];
    }
  }
  __syncthreads();
  const double D = sh[2][c][lane];
  const double X = sh[3][c][lane];
#pragma unroll
  for (int kk = 0; kk < L; ++kk) {
    const int k = k0 + kk;
    const double x = d[kk] + D * A.z.G[k] + X * A.z.B[k];
    if (act && k < nz) stb(A.out + k * nxy, oc, (T)x);
  }
}

// Patch shape and tile walk per precision (timed on MI355X).
#ifndef MR_ROWS64
#define MR_ROWS64 2
#endif
#ifndef MR_ROWS32
#define MR_ROWS32 1
#endif
#ifndef MR_BAND64
#define MR_BAND64 1
#endif
#ifndef MR_BAND32
#define MR_BAND32 4
#endif
#ifndef MR_F32_MINB
#define MR_F32_MINB 1
#endif
#ifndef MR_PFD64
#define MR_PFD64 0
#endif
#ifndef MR_PFD32
#define MR_PFD32 1
#endif
template <typename T>
struct StepLayout {
  static constexpr int rows = sizeof(T) == 8 ? MR_ROWS64 : MR_ROWS32;
  static constexpr int band = sizeof(T) == 8 ? MR_BAND64 : MR_BAND32;   // 0: whole rows
  static constexpr int min_blocks = sizeof(T) == 8 ? 1 : MR_F32_MINB;   // minimum waves per SIMD
  static constexpr int prefetch = sizeof(T) == 8 ? MR_PFD64 : MR_PFD32;  // levels whose loads run ahead of the arithmetic
};

// Compile-time variants: side walls, explicit z share (never for the seed solve).
template <typename T, int LL, int MODE, int R, int MB, int PF>
void launch_variant(bool walls, bool expz, dim3 grid, dim3 block, hipStream_t s, const LineArgs<T>& a) {
  if constexpr (MODE != SEED) {
    if (expz) {
      if (walls)
        hipLaunchKernelGGL((line_kernel<T, LL, MODE, R, MB, PF, true, true>), grid, block, 0, s, a);
      else
        hipLaunchKernelGGL((line_kernel<T, LL, MODE, R, MB, PF, false, true>), grid, block, 0, s, a);
      return;
    }
  }
  if (walls)
    hipLaunchKernelGGL((line_kernel<T, LL, MODE, R, MB, PF, true, false>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((line_kernel<T, LL, MODE, R, MB, PF, false, false>), grid, block, 0, s, a);
}

template <typename T, int MODE>
hipError_t launch_line(mr_ctx* c, LineArgs<T> a, hipStream_t s) {
  constexpr int rows = StepLayout<T>::rows, cols = kWave / rows;
  constexpr int mb = StepLayout<T>::min_blocks;
  constexpr int pf = StepLayout<T>::prefetch;
  const int ntx = (c->nx + cols - 1) / cols, nty = (c->ny + rows - 1) / rows;
  a.band = StepLayout<T>::band > 0 && StepLayout<T>::band < ntx ? StepLayout<T>::band : ntx;
  const dim3 grid((unsigned)(ntx * nty));
  const dim3 block(kWave, c->nch);
  const bool walls = a.wx || a.wy;
  const bool expz = MODE != SEED && c->z_explicit > 0.0;
  switch (c->L) {
#define MR_CASE(LL)                                                                             \
  case LL:                                                                                      \
    launch_variant<T, LL, MODE, rows, mb, pf>(walls, expz, grid, block, s, a);                  \
    break;
    MR_CASE(8)
    MR_CASE(16)
    MR_CASE(24)
    MR_CASE(32)
    MR_CASE(40)
#undef MR_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

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

// One thread per dense cell (i, j, k) owns the faces on its low side: x-face i,
// y-face j and, for k >= 1, z-face k.  The walls' z faces carry no advective
// flux, so their gradient stays as it is; a side-wall face (x-face 0 or
// y-face 0 of a walled axis) gets zero.
template <typename T>
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
  T su = T(0), sv = T(0), sw = T(0);
  for (int s = 0; s < A.count; ++s) {
    const T* th = A.th[s];
    const T* mu = A.mu[s];
    const T tc = th[row + i], mc = mu[row + i];
    const T gx = half * (th[row + im] + tc) * (mc * ihx - mu[row + im] * ihxm);
    const T gy = half * (th[k * nxy + jm * nx + i] + tc) * (mc * ihy - mu[k * nxy + jm * nx + i] * ihym);
    su += A.tau[s] * gx;
    sv += A.tau[s] * gy;
    if (k > 0) {
      const T gz = half * (th[row - nxy + i] + tc) * (mc * ihz - mu[row - nxy + i] * ihzm);
      sw += A.tau[s] * gz;
    }
  }
  if (A.wx && i == 0) su = T(0);
  if (A.wy && j == 0) sv = T(0);
  A.gu[row + i] += su;
  A.gv[row + i] += sv;
  if (k > 0) A.gw[row + i] += sw;
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
  const int64_t cells = (int64_t)c->nx * c->ny * c->nz;
  hipLaunchKernelGGL(grad_kernel<T>, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, a);
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
