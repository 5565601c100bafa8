// Template definitions of the fused line kernel of the scalar step (forward,
// reverse, seed) and its launcher, shared by the translation units that
// instantiate its variants.
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
#pragma once

#include <string.h>

#include "mr_internal.h"

namespace mr {
namespace line {

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
  T uhx, uhy;          // UXY kernels: 1/h of the uniform x and y widths
  T uxx, uyy;          // UXY kernels: 1/h^2 of x and y
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
  // fourth-order faces (ORD4 only)
  T xm2, xp2, ym2, yp2;     // the z-stencil field two cells away in x and y
  T zp2;                    // the z-stencil field two levels up
  T um, up2, vm, vp2;       // reverse step: u on faces i-1 and i+2, v on faces j-1 and j+2
  T w2;                     // reverse step: w on the face two levels up
};

// Weights of the fourth-order face value on face f of an axis of n cells, for
// the cells f-2, f-1, f, f+1, read from the axis's table (Sec. 2.2: the face
// value of the polynomial whose means over the stencil cells equal their
// values; on a uniform axis (-1, 7, 7, -1)/12 away from walls).  f runs from
// -1 to n+1: a periodic axis wraps it, a walled one clamps it to a wall face,
// whose row is zero (wall faces and faces beyond them carry no velocity).
template <typename T>
struct W4 {
  T a, b, c, d;
};

template <typename T>
__device__ __forceinline__ W4<T> face_w4(const T* tab, int f, int n, bool walled) {
  const int r = walled ? min(max(f, 0), n) : (f % n + n) % n;
  const T* p = tab + 4 * r;
  return W4<T>{p[0], p[1], p[2], p[3]};
}

// Load from a wave-uniform base at a 32-bit byte offset (scalar base + vector
// offset addressing).
template <typename T>
__device__ __forceinline__ T ldb(const T* base, unsigned boff) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff);
}

// Non-temporal (streaming) forms: for values used once, so that their lines
// leave room in L2 for the lines that neighbouring rows and tiles re-read.
// Timed: w loads and result stores non-temporal make the step 3-11% faster;
// u (its edge lines are re-read by the tile beside) is slower that way.
template <typename T>
__device__ __forceinline__ T ldb_nt(const T* base, unsigned boff) {
  return __builtin_nontemporal_load(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + boff));
}
template <typename T>
__device__ __forceinline__ void stb_nt(T* base, unsigned boff, T v) {
  __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff));
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
//
// ORD4: fourth-order face values of the advected field, with per-face weight
// tables on every axis (face_w4 for x and y, held per lane for the column).  The stencil field is then needed two cells away on every axis: the
// x pair comes from two lane shifts, with the first two and last two columns
// of a row loading theirs in one more edge load; the y pair from one more halo
// load (two rows per patch: the other row's halo value by a cross-lane
// shuffle); the z pair from carrying one more level.  The reverse step's
// transposed faces also need u, v, w on the faces one beyond each side.
template <typename T, int L, int MODE, int ROWS, int MINB, int PFD, bool WALLS, bool EXPZ, bool ORD4,
          bool UXY = false, int MT = 1024>
__global__ void __launch_bounds__(MT, MINB) line_kernel(LineArgs<T> A) {
  static_assert(!((EXPZ || ORD4) && MODE == SEED), "the seed solve has no stencil");
  static_assert(!ORD4 || ROWS <= 2, "fourth-order faces need patches of at most two rows");
  static_assert(!UXY || !(WALLS || EXPZ || ORD4), "uniform-width kernels exist for the plain variant only");
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
  // ORD4: cells two away, the edge and halo loads that fetch them, face weights
  int im2 = i, ip2 = i, jm2 = j, jp2 = j;
  if constexpr (ORD4) {
    im2 = wx ? max(i - 2, 0) : (i - 2 + 2 * nx) % nx;
    ip2 = wx ? min(i + 2, nx - 1) : (i + 2) % nx;
    jm2 = wy ? max(j - 2, 0) : (j - 2 + 2 * ny) % ny;
    jp2 = wy ? min(j + 2, ny - 1) : (j + 2) % ny;
  }
  const unsigned oxm2 = (j * nx + im2) * sz, oxp2 = (j * nx + ip2) * sz;
  const unsigned oym2 = (jm2 * nx + i) * sz, oyp2 = (jp2 * nx + i) * sz;
  const bool x2lo = col < 2, x2hi = col >= COLS - 2;
  const unsigned oedge2 = x2lo ? oxm2 : (x2hi ? oxp2 : oc);    // two columns out (first / last two)
  const unsigned ohalo2 = hrow == 0 ? oym2 : oyp2;             // ROWS = 2: two rows out
  const unsigned oedge_u = xfirst ? oxm : (xlast ? oxp2 : oc); // reverse: u on face i-1 / i+2
  const unsigned ohalo_v = hrow == 0 ? oym : oyp2;             // reverse, ROWS = 2: v on face j-1 / j+2
  W4<T> wxl{}, wxh{}, wxa{}, wxd{}, wyl{}, wyh{}, wya{}, wyd{};
  if constexpr (ORD4) {
    wxl = face_w4<T>(g.c4x, i, nx, wx); wxh = face_w4<T>(g.c4x, i + 1, nx, wx);
    wyl = face_w4<T>(g.c4y, j, ny, wy); wyh = face_w4<T>(g.c4y, j + 1, ny, wy);
    if constexpr (MODE != FWD) {
      wxa = face_w4<T>(g.c4x, i - 1, nx, wx); wxd = face_w4<T>(g.c4x, i + 2, nx, wx);
      wya = face_w4<T>(g.c4y, j - 1, ny, wy); wyd = face_w4<T>(g.c4y, j + 2, ny, wy);
    }
  }
  // reverse: faces i-1 / i+2 (j-1 / j+2) that are walls or beyond carry no velocity
  const bool zum = wx && i <= 1, zup2 = wx && i + 2 >= nx;
  const bool zvm = wy && j <= 1, zvp2 = wy && j + 2 >= ny;

  // UXY (uniform x and y widths, periodic): every width and centre distance
  // of an axis is one wave-uniform kernel argument, so no lane holds them
  const T ihx = UXY ? A.uhx : g.ihx[i], ihxm = UXY ? A.uhx : g.ihx[im], ihxp = UXY ? A.uhx : g.ihx[ip];
  const T idx0 = UXY ? A.uhx : g.idxc[i], idx1 = UXY ? A.uhx : g.idxc[ip];
  const T ihy = UXY ? A.uhy : g.ihy[j], ihym = UXY ? A.uhy : g.ihy[jm], ihyp = UXY ? A.uhy : g.ihy[jp];
  const T idy0 = UXY ? A.uhy : g.idyc[j], idy1 = UXY ? A.uhy : g.idyc[jp];
  const T half = T(0.5);
  T ihxm2 = T(0), ihxp2 = T(0), ihym2 = T(0), ihyp2 = T(0);
  if constexpr (ORD4 && MODE != FWD) {
    ihxm2 = g.ihx[im2]; ihxp2 = g.ihx[ip2];
    ihym2 = g.ihy[jm2]; ihyp2 = g.ihy[jp2];
  }

  double d[L];
  double dprev = 0.0;
  // field whose z neighbours the stencil needs (theta^n or mu^n), carried up the chunk
  const T* f = MODE == FWD ? A.a1 : A.a0;
  // second stencil field: theta^{n-1} (FWD) or mu^{n+1} (BWD, a0 with zero weights if absent)
  const T* p = MODE == FWD ? A.a0 : A.a1;
  T zm = T(0), zc = T(0), w0 = T(0);
  T pzm = T(0), pnext = T(0);
  T zm2 = T(0), znext = T(0), wm = T(0), wnext = T(0);
  if (MODE != SEED) {
    zc = ldb(f + k0 * nxy, oc);
    zm = ldb(f + max(k0 - 1, 0) * nxy, oc);
    w0 = ldb(A.w + k0 * nxy, oc);
    if constexpr (EXPZ) pzm = ldb(p + max(k0 - 1, 0) * nxy, oc);
    if constexpr (ORD4) zm2 = ldb(f + max(k0 - 2, 0) * nxy, oc);
    if constexpr (ORD4 && MODE != FWD) wm = ldb(A.w + max(k0 - 1, 0) * nxy, oc);
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
    if constexpr (ORD4) {
      // levels are fetched in order: znext / wnext hold this level's k+1 values
      v.zp = kk > 0 ? znext : ldb(f + min(k + 1, nz - 1) * nxy, oc);
      v.zp2 = ldb(f + min(k + 2, nz - 1) * nxy, oc);
      znext = v.zp2;
      if constexpr (MODE != FWD) {
        v.w1 = kk > 0 ? wnext : ldb(A.w + (kc + 1) * nxy, oc);
        v.w2 = ldb(A.w + min(kc + 2, nz) * nxy, oc);
        wnext = v.w2;
      } else {
        v.w1 = ldb(A.w + (kc + 1) * nxy, oc);
      }
      v.xm2 = ldb(fk, oedge2);   // resolved after the lane shifts
      if constexpr (ROWS == 1) {
        v.ym2 = ldb(fk, oym2); v.yp2 = ldb(fk, oyp2);
      } else {
        v.ym2 = ldb(fk, ohalo2);
      }
      if constexpr (MODE != FWD) {
        v.um = ldb(uk, oedge_u);
        if constexpr (ROWS == 1) {
          v.vm = ldb(vk, oym); v.vp2 = ldb(vk, oyp2);
        } else {
          v.vm = ldb(vk, ohalo_v);
        }
      }
    } else {
      v.zp = ldb(f + min(k + 1, nz - 1) * nxy, oc);
      v.w1 = ldb_nt(A.w + (kc + 1) * nxy, oc);   // used once: z faces are carried
    }
    v.xm = ldb(fk, oedge);     // edge values, resolved after the lane shifts
    v.u1 = ldb(uk, oedge_r);
    v.pxm = ldb(pk, oedge);
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
      const T fe = cur.xm, pe = cur.pxm, ue = cur.u1;
      const T fl = lane_shr(zc), fr = lane_shl(zc);
      const T pl = lane_shr(cur.pc), pr = lane_shl(cur.pc);
      const T ur = lane_shl(cur.u0);
      cur.xm = xfirst ? fe : fl;
      cur.xp = xlast ? fe : fr;
      cur.pxm = xfirst ? pe : pl;
      cur.pxp = xlast ? pe : pr;
      cur.u1 = xlast ? ue : ur;
      if constexpr (ORD4) {
        // two lanes over by a cross-lane permute (a second DPP shift on the
        // first one's result makes the compiler keep every level live)
        const T e2 = cur.xm2;
        const T l2 = __shfl(zc, (lane - 2) & (kWave - 1)), r2 = __shfl(zc, (lane + 2) & (kWave - 1));
        cur.xm2 = x2lo ? e2 : l2;
        cur.xp2 = x2hi ? e2 : r2;
        if constexpr (MODE != FWD) {
          const T eu = cur.um;
          const T ul = lane_shr(cur.u0), ur2 = __shfl(cur.u1, (lane + 1) & (kWave - 1));
          cur.um = xfirst ? eu : ul;
          cur.up2 = xlast ? eu : ur2;
        }
      }
      if constexpr (ROWS > 1) {
        const T fdn = __shfl(zc, lane_dn), fup = __shfl(zc, lane_up);
        const T pdn = __shfl(cur.pc, lane_dn), pup = __shfl(cur.pc, lane_up);
        const T fh = cur.ym, ph = cur.pym;
        cur.ym = hrow == 0 ? fh : fdn;
        cur.yp = hrow == ROWS - 1 ? fh : fup;
        cur.pym = hrow == 0 ? ph : pdn;
        cur.pyp = hrow == ROWS - 1 ? ph : pup;
        if constexpr (ORD4) {
          // the other row's halo value is this row's value two rows out
          const T fh2 = cur.ym2;
          const T hdn = __shfl(fh, lane_dn), hup = __shfl(fh, lane_up);
          cur.ym2 = hrow == 0 ? fh2 : hdn;
          cur.yp2 = hrow == ROWS - 1 ? fh2 : hup;
          if constexpr (MODE != FWD) {
            const T vh = cur.vm;
            const T v0dn = __shfl(cur.v0, lane_dn), v1up = __shfl(cur.v1, lane_up);
            cur.vm = hrow == 0 ? vh : v0dn;
            cur.vp2 = hrow == ROWS - 1 ? vh : v1up;
          }
        }
      }
      if constexpr (WALLS) {
        // wall faces carry no velocity (lane selects, branch-free)
        cur.u0 = zu0 ? T(0) : cur.u0;
        cur.u1 = zu1 ? T(0) : cur.u1;
        cur.v0 = zv0 ? T(0) : cur.v0;
        cur.v1 = zv1 ? T(0) : cur.v1;
        if constexpr (ORD4 && MODE != FWD) {
          cur.um = zum ? T(0) : cur.um;
          cur.up2 = zup2 ? T(0) : cur.up2;
          cur.vm = zvm ? T(0) : cur.vm;
          cur.vp2 = zvp2 ? T(0) : cur.vp2;
        }
      }
      const T zp = cur.zp, w1 = cur.w1;
      const T ihz = g.ihz[kc];
      const T mlo = g.zlo[k], mhi = g.zhi[k];
      if (MODE == FWD) {
        T adv;
        if constexpr (ORD4) {
          // fourth-order face values of theta^n (zero weights on the z walls)
          const T* cz = g.c4z + 4 * k;
          const T txl = wxl.a * cur.xm2 + wxl.b * cur.xm + wxl.c * zc + wxl.d * cur.xp;
          const T txh = wxh.a * cur.xm + wxh.b * zc + wxh.c * cur.xp + wxh.d * cur.xp2;
          const T tyl = wyl.a * cur.ym2 + wyl.b * cur.ym + wyl.c * zc + wyl.d * cur.yp;
          const T tyh = wyh.a * cur.ym + wyh.b * zc + wyh.c * cur.yp + wyh.d * cur.yp2;
          const T tzl = cz[0] * zm2 + cz[1] * zm + cz[2] * zc + cz[3] * zp;
          const T tzh = cz[4] * zm + cz[5] * zc + cz[6] * zp + cz[7] * cur.zp2;
          adv = -((cur.u1 * txh - cur.u0 * txl) * ihx + (cur.v1 * tyh - cur.v0 * tyl) * ihy +
                  (w1 * tzh - w0 * tzl) * ihz);
        } else {
          // central-flux advection of theta^n (face value = mean of the two cells)
          const T fzl = mlo * w0 * (zm + zc);
          const T fzr = mhi * w1 * (zc + zp);
          adv = -half * ((cur.u1 * (zc + cur.xp) - cur.u0 * (cur.xm + zc)) * ihx +
                         (cur.v1 * (zc + cur.yp) - cur.v0 * (cur.ym + zc)) * ihy + (fzr - fzl) * ihz);
        }
        // lagged x/y diffusion of theta^{n-1}
        const T lap = UXY ? (cur.pxp + cur.pxm - T(2) * cur.pc) * A.uxx + (cur.pyp + cur.pym - T(2) * cur.pc) * A.uyy
                          : ((cur.pxp - cur.pc) * idx1 - (cur.pc - cur.pxm) * idx0) * ihx +
                                ((cur.pyp - cur.pc) * idy1 - (cur.pc - cur.pym) * idy0) * ihy;
        r = A.ap * cur.pc + A.ac * zc + A.tau * adv + A.tk * lap;
        if constexpr (EXPZ)   // explicit share of the z diffusion of the lagged level
          r += A.tkw * (g.lzd[k] * cur.pc + g.lzl[k] * pzm + g.lzh[k] * cur.pzp);
      } else {
        // C_u^T mu^n: each face f (cells L, R) adds u_f (mu_R/h_R - mu_L/h_L)/2 to both cells
        const T qc_x = zc * ihx, qc_y = zc * ihy, qc_z = zc * ihz;
        T cu;
        if constexpr (ORD4) {
          // every face f (cells L, R) gives s_f = u_f (mu_R/h_R - mu_L/h_L) to its
          // four stencil cells; this cell is slot d of face i-1, c of face i, b of
          // face i+1 and a of face i+2
          const T qxm2 = cur.xm2 * ihxm2, qxm = cur.xm * ihxm, qxp = cur.xp * ihxp, qxp2 = cur.xp2 * ihxp2;
          const T qym2 = cur.ym2 * ihym2, qym = cur.ym * ihym, qyp = cur.yp * ihyp, qyp2 = cur.yp2 * ihyp2;
          const T izm2 = g.ihz[max(kc - 2, 0)], izm = g.ihz[max(kc - 1, 0)];
          const T izp = g.ihz[min(kc + 1, nz - 1)], izp2 = g.ihz[min(kc + 2, nz - 1)];
          const T* ct = g.c4zt + 4 * k;
          const T cx = wxa.d * cur.um * (qxm - qxm2) + wxl.c * cur.u0 * (qc_x - qxm) +
                       wxh.b * cur.u1 * (qxp - qc_x) + wxd.a * cur.up2 * (qxp2 - qxp);
          const T cy = wya.d * cur.vm * (qym - qym2) + wyl.c * cur.v0 * (qc_y - qym) +
                       wyh.b * cur.v1 * (qyp - qc_y) + wyd.a * cur.vp2 * (qyp2 - qyp);
          const T cz = ct[0] * wm * (zm * izm - zm2 * izm2) + ct[1] * w0 * (qc_z - zm * izm) +
                       ct[2] * w1 * (zp * izp - qc_z) + ct[3] * cur.w2 * (cur.zp2 * izp2 - zp * izp);
          cu = cx + cy + cz;
        } else {
          const T czl = mlo * w0 * (qc_z - zm * g.ihz[max(kc - 1, 0)]);
          const T czr = mhi * w1 * (zp * g.ihz[min(kc + 1, nz - 1)] - qc_z);
          cu = half * (cur.u0 * (qc_x - cur.xm * ihxm) + cur.u1 * (cur.xp * ihxp - qc_x) +
                       cur.v0 * (qc_y - cur.ym * ihym) + cur.v1 * (cur.yp * ihyp - qc_y) + czl + czr);
        }
        // contribution of step n+1 through theta^n as its lagged level
        const T qx = cur.pc * ihx, qy = cur.pc * ihy;
        const T lt = UXY ? (cur.pxp + cur.pxm - T(2) * cur.pc) * A.uxx + (cur.pyp + cur.pym - T(2) * cur.pc) * A.uyy
                         : ((cur.pxm * ihxm - qx) * idx0 - (qx - cur.pxp * ihxp) * idx1) +
                               ((cur.pym * ihym - qy) * idy0 - (qy - cur.pyp * ihyp) * idy1);
        r = A.ac * zc + A.tau * cu + A.ap1 * cur.pc + A.tk1 * lt + A.s2 * cur.q;
        if (MODE == BWD0) {
          // the start-up step also reads theta^0 for its diffusion
          const T l0 = UXY ? (cur.xp + cur.xm - T(2) * zc) * A.uxx + (cur.yp + cur.ym - T(2) * zc) * A.uyy
                           : ((cur.xm * ihxm - qc_x) * idx0 - (qc_x - cur.xp * ihxp) * idx1) +
                                 ((cur.ym * ihym - qc_y) * idy0 - (qc_y - cur.yp * ihyp) * idy1);
          r += A.tk * l0;
          if constexpr (EXPZ) r += A.tkw * (g.lzd[k] * zc + g.lztl[k] * zm + g.lzth[k] * zp);
        }
        if constexpr (EXPZ)   // step n+1's explicit z share, transposed, through its lag
          r += A.tkw1 * (g.lzd[k] * cur.pc + g.lztl[k] * pzm + g.lzth[k] * cur.pzp);
      }
      if constexpr (ORD4) {
        zm2 = zm;
        if constexpr (MODE != FWD) wm = w0;
      }
      zm = zc;
      zc = zp;
      w0 = w1;
      if constexpr (EXPZ) pzm = cur.pc;
    }
    if (MODE == BWD0) {
      if (act && k < nz) stb_nt(A.out + k * nxy, oc, r);
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
    if (act && k < nz) stb_nt(A.out + k * nxy, oc, (T)x);
  }
}

// Patch shape and tile walk per precision (timed on MI355X).
template <typename T>
struct StepLayout {
  static constexpr int rows = sizeof(T) == 8 ? 2 : 1;
  static constexpr int band = sizeof(T) == 8 ? 1 : 4;   // x tiles per band of the walk
  static constexpr int min_blocks = 1;                  // minimum waves per SIMD
  static constexpr int prefetch = sizeof(T) == 8 ? 0 : 1;  // levels whose loads run ahead of the arithmetic
};

// Compile-time variants: side walls, explicit z share, fourth-order faces,
// and for the plain periodic variant uniform x and y widths (the seed solve
// has no stencil: one variant).
template <typename T, int LL, int MODE, int R, int MB, int PF, bool W, bool E, bool O, bool U = false, int MT = 1024>
void launch_one(dim3 grid, dim3 block, hipStream_t s, const LineArgs<T>& a) {
  hipLaunchKernelGGL((line_kernel<T, LL, MODE, R, MB, PF, W, E, O, U, MT>), grid, block, 0, s, a);
}

template <typename T, int LL, int MODE, int R, int MB, int PF, bool W, int MT>
void launch_eo(bool expz, bool ord4, dim3 grid, dim3 block, hipStream_t s, const LineArgs<T>& a) {
  if (ord4) {
    if (expz) launch_one<T, LL, MODE, R, MB, PF, W, true, true, false, MT>(grid, block, s, a);
    else launch_one<T, LL, MODE, R, MB, PF, W, false, true, false, MT>(grid, block, s, a);
  } else {
    if (expz) launch_one<T, LL, MODE, R, MB, PF, W, true, false, false, MT>(grid, block, s, a);
    else launch_one<T, LL, MODE, R, MB, PF, W, false, false, false, MT>(grid, block, s, a);
  }
}

// MT: the largest workgroup the kernel is compiled for.  At 1024 threads (16
// chunks) a wavefront gets at most 128 VGPRs, and the variants (side walls,
// explicit z share, fourth-order faces, stretched x or y) spill there; columns
// of at most 8 chunks launch them compiled for 512 threads (up to 256 VGPRs,
// no spill).  The plain uniform-width kernels fit either way and stay at 1024.
template <typename T, int LL, int MODE, int R, int MB, int PF, int MT>
void launch_variant(bool walls, bool expz, bool ord4, bool uxy, dim3 grid, dim3 block, hipStream_t s,
                    const LineArgs<T>& a) {
  if constexpr (MODE == SEED) {
    launch_one<T, LL, MODE, R, MB, PF, false, false, false, false, MT>(grid, block, s, a);
  } else {
    if (walls) launch_eo<T, LL, MODE, R, MB, PF, true, MT>(expz, ord4, grid, block, s, a);
    else if (uxy && !expz && !ord4) {
      // the plain FP32 step runs two levels of loads ahead (forward with chunks
      // of up to 36 levels: 1-3% faster; reverse with chunks of 32: 1%); those
      // kernels do not spill at that depth, the other variants do
      constexpr int PFU = (sizeof(T) == 4 && ((MODE == FWD && LL <= 36) || (MODE == BWD && LL == 32))) ? 2 : PF;
      launch_one<T, LL, MODE, R, MB, PFU, false, false, false, true>(grid, block, s, a);
    }
    else launch_eo<T, LL, MODE, R, MB, PF, false, MT>(expz, ord4, grid, block, s, a);
  }
}

// FP64 columns of more than 8 chunks (one 1024-thread workgroup per CU): the
// plain uniform-width step in one-row patches walked in bands of 4, as in FP32.
// Timed at 576^3: 12% faster than two-row patches, which stay faster where a
// column fits 8 chunks (two workgroups per CU: 13% at 256^3).  The other
// variants spill in that layout, and so do the forward step with chunks of
// 40 levels and the reverse step with chunks of 36 or 40.
template <int MODE>
constexpr bool wide64_ok(int LL) { return MODE == FWD ? LL <= 36 : (MODE == BWD ? LL == 32 : true); }

template <typename T, int MODE>
hipError_t launch_line_wide64(mr_ctx* c, LineArgs<T> a, hipStream_t s) {
  constexpr int mb = StepLayout<T>::min_blocks;
  const int ntx = (c->nx + kWave - 1) / kWave, nty = c->ny;
  a.band = 4 < ntx ? 4 : ntx;
  const dim3 grid((unsigned)(ntx * nty));
  const dim3 block(kWave, c->nch);
  switch (c->L) {
#define MR_CASE(LL)                                                                             \
  case LL:                                                                                      \
    if constexpr (wide64_ok<MODE>(LL)) {                                                        \
      launch_one<T, LL, MODE, 1, mb, 0, false, false, false, true>(grid, block, s, a);          \
      break;                                                                                    \
    } else {                                                                                    \
      return hipErrorInvalidValue;                                                              \
    }
    MR_CASE(32)
    MR_CASE(36)
    MR_CASE(40)
#undef MR_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
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
  const bool ord4 = MODE != SEED && c->face_order == 4;
  const bool uxy = c->uniform_xy != 0;
  a.uhx = (T)c->uhx;
  a.uhy = (T)c->uhy;
  a.uxx = (T)(c->uhx * c->uhx);
  a.uyy = (T)(c->uhy * c->uhy);
  if constexpr (sizeof(T) == 8 && MODE != SEED) {
    if (uxy && !walls && !expz && !ord4 && c->nch > 8 && wide64_ok<MODE>(c->L))
      return launch_line_wide64<T, MODE>(c, a, s);
  }
  switch (c->L) {
#define MR_CASE(LL)                                                                             \
  case LL:                                                                                      \
    if (c->nch <= 8) launch_variant<T, LL, MODE, rows, mb, pf, 512>(walls, expz, ord4, uxy, grid, block, s, a); \
    else launch_variant<T, LL, MODE, rows, mb, pf, 1024>(walls, expz, ord4, uxy, grid, block, s, a); \
    break;
    MR_CASE(32)
    MR_CASE(36)
    MR_CASE(40)
#undef MR_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace line
}  // namespace mr
