// Divergence-free coarse -> dense refinement of the staggered velocity
// (paper Sec. 3.2, Fig. 5a, Eqs. 12-19) and its transpose.
//
// Stages z, then y, then x.  In each stage one coarse cell along the refined
// axis splits the two pairs of outer normal face velocities of its column with
// R (Eq. 19, three-cell stencil) and marches the inner faces of the refined
// axis upward from the coarse face below, each from zero net outward flux of
// the sub-cell under it.  The forward refinement runs the three stages in one
// kernel with the intermediates in LDS (refine_fused); the three separate
// stage kernels, with the intermediates in a context-owned buffer, serve the
// cases it does not cover (side walls, mz > 4, a tile beyond its LDS budget).
// Side walls: the low wall face of a walled axis is taken as zero velocity and
// the high one (not stored) is zero, so the marches see no flow through walls.
//
// The transpose runs the stages in reverse order; a march becomes a suffix
// sum inside each coarse cell, a split an R^T gather (no atomics: every output
// value is written by exactly one thread, in a fixed order).
#include <string.h>

#include <algorithm>

#include "mr_internal.h"

namespace mr {
namespace {

template <typename T>
struct RefArgs {
  const T* in0;
  const T* in1;
  const T* in2;
  T* out0;
  T* out1;
  T* out2;
  T* out3;   // extra output of some transposed stages
  T* out4;
  Geom<T> g;
  int nx, ny, nz, ncx, ncy, ncz, mx, my, mz;
  int wx, wy;     // x / y bounded by walls: the wall faces carry zero velocity
};

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// A wave-uniform table value, read through the constant address space (a
// scalar load that does not wait behind the vector loads in flight).
template <typename T>
__device__ __forceinline__ T tab(const T* p, int k) {
  return ((const __attribute__((address_space(4))) T*)(p))[k];
}

template <typename T>
__device__ __forceinline__ T rdot(const T* R, const T q[3]) {
  return R[0] * q[0] + R[1] * q[1] + R[2] * q[2];
}

// ---------------------------------------------------------------- forward
// stage z: thread per coarse cell (I, J, K)
template <typename T>
__global__ void __launch_bounds__(256) stage_z(RefArgs<T> A) {
  const int ncx = A.ncx, ncy = A.ncy, ncz = A.ncz, mz = A.mz;
  const int ncxy = ncx * ncy;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= ncxy * ncz) return;
  const int I = tid % ncx, J = (tid / ncx) % ncy, K = tid / ncxy;
  const int Ip = wrap(I + 1, ncx), Jp = wrap(J + 1, ncy);
  const T* U = A.in0;
  const T* V = A.in1;
  const T* W = A.in2;
  T u0[3], u1[3], v0[3], v1[3];
  for (int r = 0; r < 3; ++r) {
    const int kc = A.g.sz[K * 3 + r];
    u0[r] = U[kc * ncxy + J * ncx + I];
    u1[r] = U[kc * ncxy + J * ncx + Ip];
    v0[r] = V[kc * ncxy + J * ncx + I];
    v1[r] = V[kc * ncxy + Jp * ncx + I];
    // side walls: the low wall face is taken as zero, the high one is not stored
    if (A.wx && I == 0) u0[r] = T(0);
    if (A.wx && I == ncx - 1) u1[r] = T(0);
    if (A.wy && J == 0) v0[r] = T(0);
    if (A.wy && J == ncy - 1) v1[r] = T(0);
  }
  const T iHX = A.g.iHX[I], iHY = A.g.iHY[J];
  T wv = W[K * ncxy + J * ncx + I];
  for (int m = 0; m < mz; ++m) {
    const int k = K * mz + m;
    const T* R = A.g.Rz + (K * mz + m) * 3;
    const T a = rdot(R, u0), b = rdot(R, u1), c = rdot(R, v0), d = rdot(R, v1);
    A.out0[k * ncxy + J * ncx + I] = a;
    A.out1[k * ncxy + J * ncx + I] = c;
    A.out2[k * ncxy + J * ncx + I] = wv;
    if (m < mz - 1) wv = wv - A.g.hz[k] * ((b - a) * iHX + (d - c) * iHY);
  }
  if (K == ncz - 1) A.out2[A.nz * ncxy + J * ncx + I] = W[ncz * ncxy + J * ncx + I];
}

// stage y: thread per (coarse I, coarse J, dense k)
template <typename T>
__global__ void __launch_bounds__(256) stage_y(RefArgs<T> A) {
  const int ncx = A.ncx, ncy = A.ncy, nz = A.nz, my = A.my, ny = A.ny;
  const int ncxy = ncx * ncy, nyx = ny * ncx;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= ncxy * nz) return;
  const int I = tid % ncx, J = (tid / ncx) % ncy, k = tid / ncxy;
  const int Ip = wrap(I + 1, ncx);
  const T* Uz = A.in0;
  const T* Vz = A.in1;
  const T* Wz = A.in2;
  T u0[3], u1[3], w0[3], w1[3];
  for (int r = 0; r < 3; ++r) {
    const int jc = A.g.sy[J * 3 + r];
    u0[r] = Uz[k * ncxy + jc * ncx + I];
    u1[r] = A.wx && I == ncx - 1 ? T(0) : Uz[k * ncxy + jc * ncx + Ip];
    w0[r] = Wz[k * ncxy + jc * ncx + I];
    w1[r] = Wz[(k + 1) * ncxy + jc * ncx + I];
  }
  const T iHX = A.g.iHX[I], ihz = A.g.ihz[k];
  T vv = Vz[k * ncxy + J * ncx + I];
  for (int m = 0; m < my; ++m) {
    const int j = J * my + m;
    const T* R = A.g.Ry + (J * my + m) * 3;
    const T a = rdot(R, u0), b = rdot(R, u1), c = rdot(R, w0), d = rdot(R, w1);
    A.out0[k * nyx + j * ncx + I] = a;
    A.out1[k * nyx + j * ncx + I] = vv;
    A.out2[k * nyx + j * ncx + I] = c;
    if (k == nz - 1) A.out2[nz * nyx + j * ncx + I] = d;
    if (m < my - 1) vv = vv - A.g.hy[j] * ((b - a) * iHX + (d - c) * ihz);
  }
}

// stage x: thread per (coarse I, dense j, dense k)
template <typename T>
__global__ void __launch_bounds__(256) stage_x(RefArgs<T> A) {
  const int ncx = A.ncx, nz = A.nz, mx = A.mx, ny = A.ny, nx = A.nx;
  const int nyx = ny * ncx, nxy = nx * ny;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= nyx * nz) return;
  const int I = tid % ncx, j = (tid / ncx) % ny, k = tid / nyx;
  const int jp = wrap(j + 1, ny);
  const T* Uzy = A.in0;
  const T* Vzy = A.in1;
  const T* Wzy = A.in2;
  T v0[3], v1[3], w0[3], w1[3];
  for (int r = 0; r < 3; ++r) {
    const int ic = A.g.sx[I * 3 + r];
    v0[r] = Vzy[k * nyx + j * ncx + ic];
    v1[r] = A.wy && j == ny - 1 ? T(0) : Vzy[k * nyx + jp * ncx + ic];
    w0[r] = Wzy[k * nyx + j * ncx + ic];
    w1[r] = Wzy[(k + 1) * nyx + j * ncx + ic];
  }
  const T ihy = A.g.ihy[j], ihz = A.g.ihz[k];
  T uu = Uzy[k * nyx + j * ncx + I];
  for (int m = 0; m < mx; ++m) {
    const int i = I * mx + m;
    const T* R = A.g.Rx + (I * mx + m) * 3;
    const T a = rdot(R, v0), b = rdot(R, v1), c = rdot(R, w0), d = rdot(R, w1);
    A.out0[k * nxy + j * nx + i] = uu;
    A.out1[k * nxy + j * nx + i] = a;
    A.out2[k * nxy + j * nx + i] = c;
    if (k == nz - 1) A.out2[nz * nxy + j * nx + i] = d;
    if (m < mx - 1) uu = uu - A.g.hx[i] * ((b - a) * ihy + (d - c) * ihz);
  }
}

// ------------------------------------------------------------ fused forward
// The three stages in one kernel.  A workgroup owns TI coarse columns
// [I0, I0+TI) (TI*mx <= 64 dense columns) of TJ coarse rows [J0, J0+TJ) and a
// range of coarse layers, walked one layer K at a time:
//   Z: for halo columns I0-1 .. I0+TI+1 and rows J0-1 .. J0+TJ, split U, V
//      along z and march W (as stage_z), into LDS.  The coarse values of
//      layer K+1 are loaded into registers while layer K is refined;
//   Y: for the layer's dense levels, the tile's rows and halo columns
//      I0-1 .. I0+TI, split the z-refined U, W along y and march V (as
//      stage_y), into LDS;
//   X: for the tile's dense cells, split V, W along x; each lane runs the x
//      march of U up to its own sub-column (the same operations in the same
//      order as stage_x).
// Each dense value is written once, 64 consecutive columns per row; the only
// HBM reads are the coarse levels (cache-resident halo re-reads).  On a
// periodic axis the halo wraps and the stencil of cell I is I-1 .. I+1; on a
// walled axis the stencil is the one-sided one of the R tables next to the
// walls (every stencil cell of the tile then lies in the halo as long as a
// tile holds at least two cells along that axis, which the launcher ensures),
// the wall faces are taken as zero, and halo cells beyond a wall are computed
// but never read.
constexpr int kFuseCols = 64;

__device__ __forceinline__ int wrapm(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

constexpr int kFuseMaxMz = 4;   // z refinement factors the fused kernel is built for

// The coarse values one stage-z item reads for one layer.
template <typename T>
struct ZLoad {
  T u0[3], u1[3], v0[3], v1[3], wb, wt;
};

template <typename T>
__device__ __forceinline__ void z_load(const RefArgs<T>& A, int K, int Ig, int Ip, int Jg, int Jp, ZLoad<T>& z) {
  const int ncx = A.ncx, ncxy = A.ncx * A.ncy, mz = A.mz;
  for (int q = 0; q < 3; ++q) {
    const int kc3 = A.g.sz[K * 3 + q];
    z.u0[q] = A.in0[kc3 * ncxy + Jg * ncx + Ig];
    z.u1[q] = A.in0[kc3 * ncxy + Jg * ncx + Ip];
    z.v0[q] = A.in1[kc3 * ncxy + Jg * ncx + Ig];
    z.v1[q] = A.in1[kc3 * ncxy + Jp * ncx + Ig];
  }
  z.wb = A.in2[K * ncxy + Jg * ncx + Ig];
  z.wt = A.in2[(K + 1) * ncxy + Jg * ncx + Ig];
}

// Per-layer z tables in LDS, one slot per layer parity: R_z rows, hz, 1/hz.
constexpr int kZTab = 5 * kFuseMaxMz;

// The table value lane t contributes for layer K (lanes t < 5 mz).
template <typename T>
__device__ __forceinline__ T ztab_load(const Geom<T>& g, int K, int mz, int t) {
  if (t < 3 * mz) return g.Rz[(K * mz + t / 3) * 3 + t % 3];
  if (t < 4 * mz) return g.hz[K * mz + t - 3 * mz];
  if (t < 5 * mz) return g.ihz[K * mz + t - 4 * mz];
  return T(0);
}

template <typename T>
__device__ __forceinline__ void ztab_store(T* slot, int mz, int t, T v) {
  if (t < 3 * mz) slot[t] = v;                                   // rz[m][r] at 3 m + r
  else if (t < 4 * mz) slot[3 * kFuseMaxMz + t - 3 * mz] = v;    // hz[m]
  else if (t < 5 * mz) slot[4 * kFuseMaxMz + t - 4 * mz] = v;    // 1/hz[m]
}

template <typename T>
__device__ __forceinline__ T rdot3(const T* R, const T q[3]) {
  return R[0] * q[0] + R[1] * q[1] + R[2] * q[2];
}

// LDS element counts of refine_fused (tables first, then the stage fields).
__host__ __device__ inline int fused_tables(int TI, int TJ, int mx, int my) {
  const int NXH = TI + 3, RY = TJ * my, CX = TI * mx;
  return NXH + 5 * RY + 4 * CX + 2 * kZTab;
}
__host__ __device__ inline int fused_fields(int TI, int TJ, int my, int mz) {
  const int NXH = TI + 3, NYH = TJ + 2, RY = TJ * my;
  return 2 * mz * NYH * NXH + (mz + 1) * NYH * NXH + mz * RY * NXH + (mz + 1) * RY * NXH +
         mz * TJ * (my + 1) * NXH;
}

template <typename T, bool NT>
__global__ void __launch_bounds__(256) refine_fused(RefArgs<T> A, int TI, int TJ, int nbx, int nby,
                                                    int KC) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* const sm = reinterpret_cast<T*>(smem_raw);
  const int ncx = A.ncx, ncy = A.ncy, ncz = A.ncz, mx = A.mx, my = A.my, mz = A.mz;
  const int nx = A.nx, nz = A.nz;
  const int nxy = nx * A.ny;
  const int NXH = TI + 3, NYH = TJ + 2, RY = TJ * my, CX = TI * mx;
  // per-workgroup tables
  T* const tIHX = sm;                          // [NXH] 1/HX of the halo columns
  T* const tRy = tIHX + NXH;                   // [RY][3]
  T* const tHy = tRy + 3 * RY;                 // [RY]
  T* const tIhy = tHy + RY;                    // [RY]
  T* const tRx = tIhy + RY;                    // [CX][3]
  T* const tHx = tRx + 3 * CX;                 // [CX]
  T* const tZ = tHx + CX;                      // [2][kZTab] per-layer z tables, by layer parity
  // stage fields
  T* const Uz = tZ + 2 * kZTab;                // [mz][NYH][NXH]
  T* const Vz = Uz + mz * NYH * NXH;           // [mz][NYH][NXH]
  T* const Wz = Vz + mz * NYH * NXH;           // [mz+1][NYH][NXH]
  T* const Uzy = Wz + (mz + 1) * NYH * NXH;    // [mz][RY][NXH]
  T* const Wzy = Uzy + mz * RY * NXH;          // [mz+1][RY][NXH]
  T* const Vzy = Wzy + (mz + 1) * RY * NXH;    // [mz][TJ][my+1][NXH]
  const int b = blockIdx.x;
  const int bx = b % nbx, by = (b / nbx) % nby, kc = b / (nbx * nby);
  const int I0 = bx * TI, J0 = by * TJ;
  const int TJv = min(TJ, ncy - J0);           // rows of this tile
  const int K0 = kc * KC, K1 = min(ncz, K0 + KC);
  const int t = threadIdx.x;
  const Geom<T>& g = A.g;

  for (int e = t; e < NXH; e += blockDim.x) tIHX[e] = g.iHX[wrapm(I0 - 1 + e, ncx)];
  for (int e = t; e < TJv * my; e += blockDim.x) {
    const int j = J0 * my + e;
    for (int r = 0; r < 3; ++r) tRy[3 * e + r] = g.Ry[j * 3 + r];
    tHy[e] = g.hy[j];
    tIhy[e] = g.ihy[j];
  }
  for (int e = t; e < CX; e += blockDim.x) {
    const int i = min(I0 * mx + e, nx - 1);
    for (int r = 0; r < 3; ++r) tRx[3 * e + r] = g.Rx[i * 3 + r];
    tHx[e] = g.hx[i];
  }

  // stage-z item of this thread: halo row zr, halo column zl
  const bool zon = t < NYH * NXH;
  const int zr = zon ? t / NXH : 0, zl = zon ? t - zr * NXH : 0;
  const int zI = wrapm(I0 - 1 + zl, ncx), zIp = wrapm(zI + 1, ncx);
  const int zJ = wrapm(J0 - 1 + zr, ncy), zJp = wrapm(zJ + 1, ncy);
  // walled axes: faces on or beyond a wall carry no velocity (lane selects)
  const int fI = I0 - 1 + zl, fJ = J0 - 1 + zr;
  const bool zu0 = A.wx && (fI <= 0 || fI >= ncx), zu1 = A.wx && (fI + 1 <= 0 || fI + 1 >= ncx);
  const bool zv0 = A.wy && (fJ <= 0 || fJ >= ncy), zv1 = A.wy && (fJ + 1 <= 0 || fJ + 1 >= ncy);
  const T ziHX = g.iHX[zI], ziHY = g.iHY[zJ];
  // stage-x lane roles: column col of the tile, sub-column sub of coarse column Ix
  const int col = t % kFuseCols, grp = t / kFuseCols;
  const int Ix = I0 + col / mx, sub = col - (col / mx) * mx;
  const bool xon = col < CX && Ix < ncx;
  // (M_x = 1: R = [0 1 0] on the centred stencil, whose table entries wrap
  // even on a walled axis; the halo column of the cell itself is Ix - I0 + 1)
  int xloc[3];
  for (int r = 0; r < 3; ++r) {
    const int p = !xon ? 0 : (mx == 1 ? Ix - I0 + r : g.sx[Ix * 3 + r] - (I0 - 1));
    xloc[r] = A.wx ? p : wrapm(p, ncx);
  }

  ZLoad<T> cur, nxt;
  if (zon && K0 < K1) z_load<T>(A, K0, zI, zIp, zJ, zJp, cur);
  if (K0 < K1) ztab_store(tZ + (K0 & 1) * kZTab, mz, t, ztab_load(g, K0, mz, t));
  __syncthreads();   // tables
  for (int K = K0; K < K1; ++K) {
    // the next layer's coarse values and z tables, in flight while this one is refined
    if (zon && K + 1 < K1) z_load<T>(A, K + 1, zI, zIp, zJ, zJp, nxt);
    const T tnext = K + 1 < K1 ? ztab_load(g, K + 1, mz, t) : T(0);
    const T* const zt = tZ + (K & 1) * kZTab;
    const T* const ihzK = zt + 4 * kFuseMaxMz;
    // ---- Z
    if (zon) {
      T u0[3], u1[3], v0[3], v1[3];
      for (int q = 0; q < 3; ++q) {
        u0[q] = zu0 ? T(0) : cur.u0[q];
        u1[q] = zu1 ? T(0) : cur.u1[q];
        v0[q] = zv0 ? T(0) : cur.v0[q];
        v1[q] = zv1 ? T(0) : cur.v1[q];
      }
      T wv = cur.wb;
      for (int m = 0; m < mz; ++m) {
        const T* R = zt + 3 * m;
        const T a = rdot3(R, u0), bb = rdot3(R, u1), c = rdot3(R, v0), d = rdot3(R, v1);
        Uz[(m * NYH + zr) * NXH + zl] = a;
        Vz[(m * NYH + zr) * NXH + zl] = c;
        Wz[(m * NYH + zr) * NXH + zl] = wv;
        if (m < mz - 1) wv = wv - zt[3 * kFuseMaxMz + m] * ((bb - a) * ziHX + (d - c) * ziHY);
      }
      Wz[(mz * NYH + zr) * NXH + zl] = cur.wt;
    }
    __syncthreads();
    // ---- Y: items (tile row jt, level m, halo column l)
    const int ny_items = TJv * mz * (NXH - 1);
    for (int it = t; it < ny_items; it += blockDim.x) {
      const int l = it % (NXH - 1), rest = it / (NXH - 1);
      const int m = rest % mz, jt = rest / mz;
      T u0[3], u1[3], w0[3], w1[3];
      // first stencil row of tile row jt (centred unless next to a y wall)
      // (M_y = 1: the centred rows, as for M_x = 1 above)
      const int rs = A.wy && my > 1 ? g.sy[(J0 + jt) * 3] - (J0 - 1) : jt;
      for (int r = 0; r < 3; ++r) {
        u0[r] = Uz[(m * NYH + rs + r) * NXH + l];
        u1[r] = Uz[(m * NYH + rs + r) * NXH + l + 1];
        w0[r] = Wz[(m * NYH + rs + r) * NXH + l];
        w1[r] = Wz[((m + 1) * NYH + rs + r) * NXH + l];
      }
      const T iHX = tIHX[l], ihz = ihzK[m];
      T vv = Vz[(m * NYH + jt + 1) * NXH + l];
      for (int q = 0; q < my; ++q) {
        const int row = jt * my + q;
        const T* R = tRy + 3 * row;
        const T a = rdot3(R, u0), bb = rdot3(R, u1), c = rdot3(R, w0), d = rdot3(R, w1);
        Uzy[(m * RY + row) * NXH + l] = a;
        if (l == NXH - 2) Uzy[(m * RY + row) * NXH + l + 1] = bb;
        Vzy[((m * TJ + jt) * (my + 1) + q) * NXH + l] = vv;
        Wzy[(m * RY + row) * NXH + l] = c;
        if (m == mz - 1) Wzy[(mz * RY + row) * NXH + l] = d;
        if (q < my - 1) vv = vv - tHy[row] * ((bb - a) * iHX + (d - c) * ihz);
      }
      Vzy[((m * TJ + jt) * (my + 1) + my) * NXH + l] = Vz[(m * NYH + jt + 2) * NXH + l];
    }
    // publish the next layer's z tables into the other parity slot: its last
    // readers (stage z and x of layer K-1) are behind the barrier after stage z
    if (K + 1 < K1) ztab_store(tZ + ((K + 1) & 1) * kZTab, mz, t, tnext);
    __syncthreads();
    // ---- X: items (dense row of the tile, level m) x 64 columns.  The next
    // layer's stage z writes only Uz, Vz, Wz, which stage x does not read, and
    // its tables sit in the other parity slot, so no barrier is needed after it.
    const int npairs = TJv * my * mz;
    for (int pr = grp; pr < npairs; pr += 4) {
      if (!xon) continue;
      const int m = pr % mz, row = pr / mz;
      const int jt = row / my, q = row - jt * my;
      const int i = Ix * mx + sub, j = (J0 + jt) * my + q, k = K * mz + m;
      T v0[3], v1[3], w0[3], w1[3];
      for (int r = 0; r < 3; ++r) {
        v0[r] = Vzy[((m * TJ + jt) * (my + 1) + q) * NXH + xloc[r]];
        v1[r] = Vzy[((m * TJ + jt) * (my + 1) + q + 1) * NXH + xloc[r]];
        w0[r] = Wzy[(m * RY + row) * NXH + xloc[r]];
        w1[r] = Wzy[((m + 1) * RY + row) * NXH + xloc[r]];
      }
      const T ihy = tIhy[row], ihz = ihzK[m];
      // the x march up to this sub-column, in the order of stage_x
      T uu = Uzy[(m * RY + row) * NXH + (col / mx) + 1];
      for (int mp = 0; mp < sub; ++mp) {
        const T* Rp = tRx + 3 * (col - sub + mp);
        const T ap = rdot3(Rp, v0), bp = rdot3(Rp, v1), cp = rdot3(Rp, w0), dp = rdot3(Rp, w1);
        uu = uu - tHx[col - sub + mp] * ((bp - ap) * ihy + (dp - cp) * ihz);
      }
      const T* R = tRx + 3 * col;
      const T a = rdot3(R, v0), c = rdot3(R, w0);
      const int o = k * nxy + j * nx + i;
      // NT: the dense faces are written once, so streaming stores keep L2 for
      // the coarse halo; used when the tile's rows are whole 128-byte lines
      // (partial lines stored that way were 37% slower at M_x = 3).  A compile-
      // time flag: a runtime branch lets the compiler merge the two stores and
      // drop the streaming hint.
      if constexpr (NT) {
        __builtin_nontemporal_store(uu, A.out0 + o);
        __builtin_nontemporal_store(a, A.out1 + o);
        __builtin_nontemporal_store(c, A.out2 + o);
        if (k == nz - 1) __builtin_nontemporal_store(rdot3(R, w1), A.out2 + o + nxy);
      } else {
        A.out0[o] = uu;
        A.out1[o] = a;
        A.out2[o] = c;
        if (k == nz - 1) A.out2[o + nxy] = rdot3(R, w1);
      }
    }
    cur = nxt;
  }
}

// -------------------------------------------------------------- transpose
// Sum over the refined sub-faces p+1..m-1 of coarse cell I of g(I*m + q):
// the adjoint of the increment that the march adds at sub-face p.
template <typename T, typename F>
__device__ __forceinline__ T suffix(int I, int m, int p, F g) {
  T s = T(0);
  for (int q = p + 1; q < m; ++q) s += g(I * m + q);
  return s;
}

// R^T gather: sum over coarse cells I whose stencil holds cell c of
// R_I[p][r] * val(I*m + p) with r the position of c in that stencil.
template <typename T, typename F>
__device__ __forceinline__ T gather(const T* R, const int* sidx, int nc, int m, bool periodic, int c, F val) {
  if (m == 1) return val(c);
  T acc = T(0);
  const int lo = periodic ? c - 1 : max(0, c - 2);
  const int hi = periodic ? c + 1 : min(nc - 1, c + 2);
  for (int Iu = lo; Iu <= hi; ++Iu) {
    const int I = periodic ? wrap(Iu, nc) : Iu;
    for (int r = 0; r < 3; ++r) {
      if (sidx[I * 3 + r] != c) continue;
      for (int p = 0; p < m; ++p) acc += R[(I * m + p) * 3 + r] * val(I * m + p);
    }
  }
  return acc;
}

// X1: thread per (coarse I, dense j, dense k).  in0..2 = gu, gv, gw (dense);
// out0 = gUzy, out1 = gv_tot (dense), out2 = gw_tot (dense).
template <typename T>
__global__ void __launch_bounds__(256) tx_march(RefArgs<T> A) {
  const int ncx = A.ncx, nz = A.nz, mx = A.mx, ny = A.ny, nx = A.nx;
  const int nyx = ny * ncx, nxy = nx * ny;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= nyx * nz) return;
  const int I = tid % ncx, j = (tid / ncx) % ny, k = tid / nyx;
  const int jm = wrap(j - 1, ny);
  const T* gu = A.in0;
  const T* gv = A.in1;
  const T* gw = A.in2;
  const T ihy = A.g.ihy[j], ihym = A.g.ihy[jm], ihz = A.g.ihz[k];
  const T ihzm = k > 0 ? A.g.ihz[k - 1] : T(0);
  T tot = T(0);
  for (int p = 0; p < mx; ++p) {
    const int i = I * mx + p;
    const T hx = A.g.hx[i];
    tot += gu[k * nxy + j * nx + i];
    // adjoint of the march increment at sub-face p (zero for the last one)
    const T c0 = -suffix<T>(I, mx, p, [&](int q) { return gu[k * nxy + j * nx + q]; });
    const T cjm = A.wy && j == 0 ? T(0) : -suffix<T>(I, mx, p, [&](int q) { return gu[k * nxy + jm * nx + q]; });
    const T ckm = k > 0 ? -suffix<T>(I, mx, p, [&](int q) { return gu[(k - 1) * nxy + j * nx + q]; }) : T(0);
    A.out1[k * nxy + j * nx + i] = gv[k * nxy + j * nx + i] + cjm * hx * ihym - c0 * hx * ihy;
    A.out2[k * nxy + j * nx + i] = gw[k * nxy + j * nx + i] + ckm * hx * ihzm - c0 * hx * ihz;
    if (k == nz - 1) A.out2[nz * nxy + j * nx + i] = gw[nz * nxy + j * nx + i] + c0 * hx * ihz;
  }
  A.out0[k * nyx + j * ncx + I] = tot;
}

// X2: thread per (coarse I, dense j, dense level k <= nz).  in1 = gv_tot,
// in2 = gw_tot; out1 = gVzy, out2 = gWzy.
template <typename T>
__global__ void __launch_bounds__(256) tx_split(RefArgs<T> A) {
  const int ncx = A.ncx, nz = A.nz, mx = A.mx, ny = A.ny, nx = A.nx;
  const int nyx = ny * ncx, nxy = nx * ny;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= nyx * (nz + 1)) return;
  const int I = tid % ncx, j = (tid / ncx) % ny, k = tid / nyx;
  const T* gv = A.in1;
  const T* gw = A.in2;
  A.out2[k * nyx + j * ncx + I] =
      gather<T>(A.g.Rx, A.g.sx, ncx, mx, !A.wx, I, [&](int i) { return gw[k * nxy + j * nx + i]; });
  if (k < nz)
    A.out1[k * nyx + j * ncx + I] =
        gather<T>(A.g.Rx, A.g.sx, ncx, mx, !A.wx, I, [&](int i) { return gv[k * nxy + j * nx + i]; });
}

// X^T in one kernel: a workgroup owns one dense row j and a range of levels;
// per level it stages the row of gu (and of the row below, and keeps the level
// below's) in LDS, forms the march adjoints gv_tot and gw_tot of every dense
// column there (as tx_march), and gathers them into the coarse columns with
// R^T (as tx_split), so that the two dense intermediates never go to memory.
// The rows j and j - 1 of one level are read by neighbouring workgroups of the
// same XCD at nearly the same time.
constexpr size_t kFuseMaxLds = 64 * 1024;   // LDS budget of the fused refinement kernels
constexpr int kRowCells = 1;      // coarse cells per thread of tx_row
constexpr int kRowThreads = 512;  // most threads of a tx_row workgroup (rows up to 512 coarse cells)

// R^T gather of coarse column c on a periodic axis: the cells whose stencils
// hold c are c-1, c, c+1, at stencil positions 2, 1, 0; their R entries are
// level-invariant, so a thread loads them once (rc) and gathers every level
// from the dense values in LDS.
template <typename T, int MX>
struct RowGather {
  T rc[3][MX];
  int base[3];   // first dense column of cells c-1, c, c+1
  __device__ void init(const RefArgs<T>& A, int c) {
    const int cs[3] = {wrap(c - 1, A.ncx), c, wrap(c + 1, A.ncx)};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      base[q] = cs[q] * MX;
#pragma unroll
      for (int p = 0; p < MX; ++p) rc[q][p] = A.g.Rx[(cs[q] * MX + p) * 3 + (2 - q)];
    }
  }
  __device__ T operator()(const T* val) const {
    T acc = T(0);
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int p = 0; p < MX; ++p) acc += rc[q][p] * val[base[q] + p];
    return acc;
  }
};

template <typename T, int MX>
__device__ __forceinline__ T gather_row(const RefArgs<T>& A, const RowGather<T, MX>& G, const T* val, int c) {
  if (MX == 1) return val[c];
  if (!A.wx) return G(val);
  // walled axis: the general search (one-sided stencils next to the walls)
  return gather<T>(A.g.Rx, A.g.sx, A.ncx, MX, false, c, [&](int i) { return val[i]; });
}

// X^T in one kernel: a workgroup owns one dense row j and a range of levels,
// a thread whole coarse cells of the row.  Per level each thread forms the
// march adjoints of its cells' dense columns from its own gu values (this
// level, the row below, and the level below, carried) as tx_march does,
// writes them to LDS, and after one barrier gathers its coarse columns with
// R^T from its own and the neighbouring cells (as tx_split), so that the two
// dense intermediates never go to memory.  Loads run one level ahead; the LDS
// rows alternate by level parity (one barrier per level).
template <typename T, int MX>
__global__ void __launch_bounds__(kRowThreads) tx_row(RefArgs<T> A, int kc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* const sm = reinterpret_cast<T*>(smem_raw);
  const int nx = A.nx, ny = A.ny, nz = A.nz, ncx = A.ncx;
  const int nxy = nx * ny, nyx = ny * ncx;
  T* const gvt[2] = {sm, sm + nx};            // gv_tot of a level, by parity
  T* const gwt[2] = {sm + 2 * nx, sm + 3 * nx};  // gw_tot on a level's bottom face
  T* const gwn = sm + 4 * nx;                 // gw_tot on the top face (last level)
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int j = b % ny, chunk = b / ny;
  const int k0 = chunk * kc, k1 = min(nz, k0 + kc);
  const int jm = wrap(j - 1, ny);
  const bool zjm = A.wy && j == 0;
  const T ihy = A.g.ihy[j], ihym = A.g.ihy[jm];
  const T* gu = A.in0;
  const T* gv = A.in1;
  const T* gw = A.in2;
  const int t = threadIdx.x, nt = blockDim.x;
  struct Lvl {
    T a[kRowCells][MX], bm[kRowCells][MX], v[kRowCells][MX], w[kRowCells][MX];
  };
  auto fetch = [&](int k, Lvl& L) {
    const size_t lv = (size_t)min(k, nz - 1) * nxy;
#pragma unroll
    for (int c = 0; c < kRowCells; ++c) {
      const int I = t + c * nt;
      if (I < ncx) {
#pragma unroll
        for (int p = 0; p < MX; ++p) {
          const int i = I * MX + p;
          L.a[c][p] = gu[lv + j * nx + i];
          L.bm[c][p] = gu[lv + jm * nx + i];
          L.v[c][p] = gv[lv + j * nx + i];
          L.w[c][p] = gw[lv + j * nx + i];
        }
      }
    }
  };
  // level-invariant per-thread values: R entries of the gather, widths
  RowGather<T, MX> G[kRowCells];
  T hx[kRowCells][MX];
#pragma unroll
  for (int c = 0; c < kRowCells; ++c) {
    const int I = min(t + c * nt, ncx - 1);
    G[c].init(A, I);
#pragma unroll
    for (int p = 0; p < MX; ++p) hx[c][p] = A.g.hx[I * MX + p];
  }
  // suffix sums of gu on the level below (for the bottom faces' adjoint)
  T sprev[kRowCells][MX];
#pragma unroll
  for (int c = 0; c < kRowCells; ++c) {
    const int I = t + c * nt;
#pragma unroll
    for (int p = 0; p < MX; ++p) sprev[c][p] = T(0);
    if (k0 > 0 && I < ncx) {
      const size_t lv = (size_t)(k0 - 1) * nxy + j * nx + I * MX;
#pragma unroll
      for (int p = 0; p < MX; ++p)
        sprev[c][p] = suffix<T>(0, MX, p, [&](int q) { return gu[lv + q]; });
    }
  }
  Lvl cur, nxt;
  fetch(k0, cur);
  for (int k = k0; k < k1; ++k) {
    if (k + 1 < k1) fetch(k + 1, nxt);
    T* const vt = gvt[k & 1];
    T* const wt = gwt[k & 1];
    const T ihz = tab(A.g.ihz, k);
    const T ihzm = k > 0 ? tab(A.g.ihz, k - 1) : T(0);
    const size_t orow = (size_t)k * nyx + j * ncx;
#pragma unroll
    for (int c = 0; c < kRowCells; ++c) {
      const int I = t + c * nt;
      if (I < ncx) {
        T tot = T(0);
#pragma unroll
        for (int p = 0; p < MX; ++p) {
          const int i = I * MX + p;
          const T hxi = hx[c][p];
          const T su = suffix<T>(0, MX, p, [&](int q) { return cur.a[c][q]; });
          const T c0 = -su;
          const T cjm = zjm ? T(0) : -suffix<T>(0, MX, p, [&](int q) { return cur.bm[c][q]; });
          const T ckm = k > 0 ? -sprev[c][p] : T(0);
          vt[i] = cur.v[c][p] + cjm * hxi * ihym - c0 * hxi * ihy;
          wt[i] = cur.w[c][p] + ckm * hxi * ihzm - c0 * hxi * ihz;
          if (k == nz - 1) gwn[i] = gw[(size_t)nz * nxy + j * nx + i] + c0 * hxi * ihz;
          sprev[c][p] = su;
          tot += cur.a[c][p];
        }
        A.out0[orow + I] = tot;
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kRowCells; ++c) {
      const int I = t + c * nt;
      if (I < ncx) {
        A.out1[orow + I] = gather_row<T, MX>(A, G[c], vt, I);
        A.out2[orow + I] = gather_row<T, MX>(A, G[c], wt, I);
        if (k == nz - 1) A.out2[(size_t)nz * nyx + j * ncx + I] = gather_row<T, MX>(A, G[c], gwn, I);
      }
    }
    cur = nxt;
  }
}

template <typename T>
bool launch_tx_row(mr_ctx* c, const RefArgs<T>& a, hipStream_t s) {
  const size_t lds = sizeof(T) * 5 * (size_t)c->nx;
  if (lds > kFuseMaxLds || c->ncx > kRowCells * kRowThreads || c->mx > 4) return false;
  // levels per workgroup: about 16 workgroups per CU in all, at least 4 levels each
  const int64_t want = 256 * 16;
  int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(c->nz / 4, (want + c->ny - 1) / c->ny));
  const int kc = (c->nz + nchunk - 1) / nchunk;
  nchunk = (c->nz + kc - 1) / kc;
  const int threads = (c->ncx + kRowCells * kWave - 1) / (kRowCells * kWave) * kWave;
  const dim3 grid((unsigned)((int64_t)c->ny * nchunk)), block(threads);
  switch (c->mx) {
    case 1: hipLaunchKernelGGL((tx_row<T, 1>), grid, block, lds, s, a, kc); break;
    case 2: hipLaunchKernelGGL((tx_row<T, 2>), grid, block, lds, s, a, kc); break;
    case 3: hipLaunchKernelGGL((tx_row<T, 3>), grid, block, lds, s, a, kc); break;
    default: hipLaunchKernelGGL((tx_row<T, 4>), grid, block, lds, s, a, kc); break;
  }
  return true;
}

// Y^T in one kernel: a thread owns coarse column I on dense level k (cells k
// and bottom face k) and walks a range of coarse rows J.  Per row it forms the
// march adjoints of the row's dense y rows from gV_zy (its own column, the
// column I - 1 from the lane beside it, the level below from memory) as
// ty_march does, keeps them for the last five rows, and gathers every row
// whose R^T sources are complete (R_y stencils reach two rows at a wall), as
// ty_split does.  The per-row R_y entries are wave-uniform (scalar loads);
// the loads of a row are issued one row ahead of its use (13-17% faster).
constexpr int kYRows = 32;   // coarse rows per thread (plus two halo rows each side)

template <typename T, int MY>
__global__ void __launch_bounds__(256) ty_fused(RefArgs<T> A, int nrowc) {
  const int ncx = A.ncx, ncy = A.ncy, nz = A.nz, ny = A.ny;
  const int ncxy = ncx * ncy, nyx = ny * ncx;
  const int lane = threadIdx.x;
  const int ntx = (ncx + kWave - 1) / kWave;
  const int bid = blockIdx.x;
  const int xt = bid % ntx;
  const int k = (bid / ntx) % (nz + 1);             // cell level k (< nz) and face k
  const int rc = bid / (ntx * (nz + 1));            // range of output rows
  const int I_raw = xt * kWave + lane;
  const bool act = I_raw < ncx;
  const int I = min(I_raw, ncx - 1);
  const int Im = wrap(I - 1, ncx);
  const bool zim = A.wx && I == 0;
  const int J0 = rc * nrowc, J1 = min(ncy, J0 + nrowc);
  const bool cells = k < nz;   // the top face has no cell level of its own
  const T iHX = A.g.iHX[I], iHXm = A.g.iHX[Im];
  const T ihz = cells ? tab(A.g.ihz, k) : T(0);
  const T ihzm = k > 0 ? tab(A.g.ihz, k - 1) : T(0);
  const T* gUzy = A.in0;
  const T* gVzy = A.in1;
  const T* gWzy = A.in2;
  auto at = [&](const T* f, int kk, int j, int i) { return f[(size_t)kk * nyx + (size_t)j * ncx + i]; };
  // march adjoints of the last five coarse rows (window slot d holds row J - 4 + d)
  T wu[5][MY], ww[5][MY];
#pragma unroll
  for (int d = 0; d < 5; ++d)
#pragma unroll
    for (int q = 0; q < MY; ++q) wu[d][q] = ww[d][q] = T(0);
  // the output row Jo gathers from rows Jo-2 .. Jo+2 (window slots 0 .. 4)
  auto emit = [&](int Jo) {
    T au = T(0), aw = T(0);
    if (MY == 1) {   // R = [0 1 0]: the row itself
      au = wu[2][0];
      aw = ww[2][0];
    }
#pragma unroll
    for (int d = 0; d < 5 && MY > 1; ++d) {
      const int J = Jo - 2 + d;
      const int Jw = A.wy ? J : wrapm(J, ncy);
      if (A.wy && (J < 0 || J >= ncy)) continue;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        if (tab(A.g.sy, Jw * 3 + r) != Jo) continue;
        if (!A.wy && (J - Jo < -1 || J - Jo > 1)) continue;   // periodic: J - 1 .. J + 1 only
#pragma unroll
        for (int q = 0; q < MY; ++q) {
          const T R = tab(A.g.Ry, (Jw * MY + q) * 3 + r);
          au += R * wu[d][q];
          aw += R * ww[d][q];
        }
      }
    }
    if (act) {
      if (cells) A.out0[(size_t)k * ncxy + Jo * ncx + I] = au;
      A.out2[(size_t)k * ncxy + Jo * ncx + I] = aw;
    }
  };
  const int Ja = max(J0 - 2, A.wy ? 0 : J0 - 2), Jb = min(J1 + 2, A.wy ? ncy : J1 + 2);
  // the loads of a row, issued one row ahead of its use
  struct RowLd {
    T vc[MY], vl[MY], vb[MY], gu[MY], gw[MY];
  };
  auto load = [&](int Ju, RowLd& L) {
    const int J = wrapm(Ju, ncy);
#pragma unroll
    for (int q = 0; q < MY; ++q) {
      const int j = J * MY + q;
      L.vc[q] = cells ? at(gVzy, k, j, I) : T(0);
      L.vl[q] = cells ? at(gVzy, k, j, Im) : T(0);   // the lane beside it loads the same line
      L.vb[q] = k > 0 ? at(gVzy, k - 1, j, I) : T(0);
      L.gu[q] = cells ? at(gUzy, k, j, I) : T(0);
      L.gw[q] = at(gWzy, k, j, I);
    }
  };
  RowLd cur, nxt;
  if (Ja < Jb) load(Ja, cur);
  for (int Ju = Ja; Ju < Jb; ++Ju) {
    const int J = wrapm(Ju, ncy);
    if (Ju + 1 < Jb) load(Ju + 1, nxt);
    // shift the window
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int q = 0; q < MY; ++q) {
        wu[d][q] = wu[d + 1][q];
        ww[d][q] = ww[d + 1][q];
      }
    const T* vc = cur.vc;
    const T* vl = cur.vl;
    const T* vb = cur.vb;
    T tot = T(0);
#pragma unroll
    for (int q = 0; q < MY; ++q) {
      const int j = J * MY + q;
      const T hy = tab(A.g.hy, j);
      T s0 = T(0), sl = T(0), sb = T(0);
#pragma unroll
      for (int qq = q + 1; qq < MY; ++qq) {
        s0 += vc[qq];
        sl += vl[qq];
        sb += vb[qq];
      }
      const T c0 = -s0, cim = zim ? T(0) : -sl, ckm = k > 0 ? -sb : T(0);
      wu[4][q] = cells ? cur.gu[q] + cim * hy * iHXm - c0 * hy * iHX : T(0);
      T wv = cur.gw[q] + ckm * hy * ihzm;
      if (cells) wv -= c0 * hy * ihz;
      ww[4][q] = wv;
      tot += vc[q];
    }
    if (cells && act && Ju >= J0 && Ju < J1) A.out3[(size_t)k * ncxy + J * ncx + I] = tot;
    // the row two back now has every source row in the window
    const int Jo = Ju - 2;
    if (Jo >= J0 && Jo < J1) emit(Jo);
    cur = nxt;
  }
  // rows whose later sources lie beyond a wall
  for (int Jo = max(J0, Jb - 2); Jo < J1; ++Jo) {
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int q = 0; q < MY; ++q) {
        wu[d][q] = wu[d + 1][q];
        ww[d][q] = ww[d + 1][q];
      }
#pragma unroll
    for (int q = 0; q < MY; ++q) wu[4][q] = ww[4][q] = T(0);
    emit(Jo);
  }
}

// Z^T in one kernel: a thread owns coarse column (I, J) and walks a range of
// coarse layers K.  Per layer it forms the march adjoints of the layer's dense
// levels from gW_z (its own column, the columns I - 1 and J - 1) as tz_march
// does, writes gW, keeps the adjoints of the last five layers, and gathers
// every layer whose R_z^T sources are complete (R_z stencils reach two layers
// at a wall), as tz_split does.  The per-layer R_z entries are wave-uniform.
constexpr int kZLayers = 16;   // coarse layers per thread (plus two halo layers each side)

template <typename T, int MZ>
__global__ void __launch_bounds__(256) tz_fused(RefArgs<T> A, int nlayc) {
  const int ncx = A.ncx, ncy = A.ncy, ncz = A.ncz, nz = A.nz;
  const int ncxy = ncx * ncy;
  const int lane = threadIdx.x & (kWave - 1);
  const int row = threadIdx.x / kWave;                 // 4 rows J per workgroup
  const int ntx = (ncx + kWave - 1) / kWave, nty = (ncy + 3) / 4;
  const int bid = blockIdx.x;
  const int xt = bid % ntx, yt = (bid / ntx) % nty, lc = bid / (ntx * nty);
  const int I_raw = xt * kWave + lane, J_raw = yt * 4 + row;
  const bool act = I_raw < ncx && J_raw < ncy;
  const int I = min(I_raw, ncx - 1), J = min(J_raw, ncy - 1);
  const int Im = wrap(I - 1, ncx), Jm = wrap(J - 1, ncy);
  const bool zim = A.wx && I == 0, zjm = A.wy && J == 0;
  const T iHX = A.g.iHX[I], iHXm = A.g.iHX[Im], iHY = A.g.iHY[J], iHYm = A.g.iHY[Jm];
  const int K0 = lc * nlayc, K1 = min(ncz, K0 + nlayc);
  const T* gUz = A.in0;
  const T* gVz = A.in1;
  const T* gWz = A.in2;
  auto at = [&](const T* f, int k, int j, int i) { return f[(size_t)k * ncxy + (size_t)j * ncx + i]; };
  T wu[5][MZ], wv[5][MZ];   // window slot d holds layer K - 4 + d
#pragma unroll
  for (int d = 0; d < 5; ++d)
#pragma unroll
    for (int p = 0; p < MZ; ++p) wu[d][p] = wv[d][p] = T(0);
  auto emit = [&](int Ko) {
    T au = T(0), av = T(0);
    if (MZ == 1) {   // R = [0 1 0]: the layer itself
      au = wu[2][0];
      av = wv[2][0];
    }
#pragma unroll
    for (int d = 0; d < 5 && MZ > 1; ++d) {
      const int K = Ko - 2 + d;
      if (K < 0 || K >= ncz) continue;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        if (tab(A.g.sz, K * 3 + r) != Ko) continue;
#pragma unroll
        for (int p = 0; p < MZ; ++p) {
          const T R = tab(A.g.Rz, (K * MZ + p) * 3 + r);
          au += R * wu[d][p];
          av += R * wv[d][p];
        }
      }
    }
    if (act) {
      // a low wall face is taken as zero by the forward map: its gradient is zero
      A.out0[(size_t)Ko * ncxy + J * ncx + I] = zim ? T(0) : au;
      A.out1[(size_t)Ko * ncxy + J * ncx + I] = zjm ? T(0) : av;
    }
  };
  auto shift = [&]() {
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int p = 0; p < MZ; ++p) {
        wu[d][p] = wu[d + 1][p];
        wv[d][p] = wv[d + 1][p];
      }
  };
  const int Ka = max(K0 - 2, 0), Kb = min(K1 + 2, ncz);
  for (int K = Ka; K < Kb; ++K) {
    shift();
    T wc[MZ], wl[MZ], wb[MZ];
#pragma unroll
    for (int p = 0; p < MZ; ++p) {
      const int k = K * MZ + p;
      wc[p] = at(gWz, k, J, I);
      wl[p] = at(gWz, k, J, Im);   // the lane beside it loads the same line
      wb[p] = at(gWz, k, Jm, I);
    }
    T tot = T(0);
#pragma unroll
    for (int p = 0; p < MZ; ++p) {
      const int k = K * MZ + p;
      const T hz = tab(A.g.hz, k);
      T s0 = T(0), sl = T(0), sb = T(0);
#pragma unroll
      for (int q = p + 1; q < MZ; ++q) {
        s0 += wc[q];
        sl += wl[q];
        sb += wb[q];
      }
      const T c0 = -s0, cim = zim ? T(0) : -sl, cjm = zjm ? T(0) : -sb;
      wu[4][p] = at(gUz, k, J, I) + cim * hz * iHXm - c0 * hz * iHX;
      wv[4][p] = at(gVz, k, J, I) + cjm * hz * iHYm - c0 * hz * iHY;
      tot += wc[p];
    }
    if (act && K >= K0 && K < K1) {
      A.out2[(size_t)K * ncxy + J * ncx + I] = tot;
      if (K == ncz - 1) A.out2[(size_t)ncz * ncxy + J * ncx + I] = at(gWz, nz, J, I);
    }
    const int Ko = K - 2;
    if (Ko >= K0 && Ko < K1) emit(Ko);
  }
  for (int Ko = max(K0, Kb - 2); Ko < K1; ++Ko) {
    shift();
#pragma unroll
    for (int p = 0; p < MZ; ++p) wu[4][p] = wv[4][p] = T(0);
    emit(Ko);
  }
}

// Y1: thread per (coarse I, coarse J, dense k).  in1 = gVzy; out0 = gUzy (+=),
// out2 = gWzy (+=), out3 = gVz.
template <typename T>
__global__ void __launch_bounds__(256) ty_march(RefArgs<T> A) {
  const int ncx = A.ncx, ncy = A.ncy, nz = A.nz, my = A.my, ny = A.ny;
  const int ncxy = ncx * ncy, nyx = ny * ncx;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= ncxy * nz) return;
  const int I = tid % ncx, J = (tid / ncx) % ncy, k = tid / ncxy;
  const int Im = wrap(I - 1, ncx);
  const T* gV = A.in1;
  const T iHX = A.g.iHX[I], iHXm = A.g.iHX[Im], ihz = A.g.ihz[k];
  const T ihzm = k > 0 ? A.g.ihz[k - 1] : T(0);
  T tot = T(0);
  for (int p = 0; p < my; ++p) {
    const int j = J * my + p;
    const T hy = A.g.hy[j];
    tot += gV[k * nyx + j * ncx + I];
    const T c0 = -suffix<T>(J, my, p, [&](int q) { return gV[k * nyx + q * ncx + I]; });
    const T cim = A.wx && I == 0 ? T(0) : -suffix<T>(J, my, p, [&](int q) { return gV[k * nyx + q * ncx + Im]; });
    const T ckm = k > 0 ? -suffix<T>(J, my, p, [&](int q) { return gV[(k - 1) * nyx + q * ncx + I]; }) : T(0);
    A.out0[k * nyx + j * ncx + I] += cim * hy * iHXm - c0 * hy * iHX;
    A.out2[k * nyx + j * ncx + I] += ckm * hy * ihzm - c0 * hy * ihz;
    if (k == nz - 1) A.out2[nz * nyx + j * ncx + I] += c0 * hy * ihz;
  }
  A.out3[k * ncxy + J * ncx + I] = tot;
}

// Y2: thread per (coarse I, coarse J, dense level k <= nz).  in0 = gUzy,
// in2 = gWzy; out0 = gUz, out2 = gWz.
template <typename T>
__global__ void __launch_bounds__(256) ty_split(RefArgs<T> A) {
  const int ncx = A.ncx, ncy = A.ncy, nz = A.nz, my = A.my, ny = A.ny;
  const int ncxy = ncx * ncy, nyx = ny * ncx;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= ncxy * (nz + 1)) return;
  const int I = tid % ncx, J = (tid / ncx) % ncy, k = tid / ncxy;
  const T* gU = A.in0;
  const T* gW = A.in2;
  A.out2[k * ncxy + J * ncx + I] =
      gather<T>(A.g.Ry, A.g.sy, ncy, my, !A.wy, J, [&](int j) { return gW[k * nyx + j * ncx + I]; });
  if (k < nz)
    A.out0[k * ncxy + J * ncx + I] =
        gather<T>(A.g.Ry, A.g.sy, ncy, my, !A.wy, J, [&](int j) { return gU[k * nyx + j * ncx + I]; });
}

// Z1: thread per coarse cell (I, J, K).  in2 = gWz; out0 = gUz (+=),
// out1 = gVz (+=), out2 = gW (coarse, final).
template <typename T>
__global__ void __launch_bounds__(256) tz_march(RefArgs<T> A) {
  const int ncx = A.ncx, ncy = A.ncy, ncz = A.ncz, mz = A.mz;
  const int ncxy = ncx * ncy;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= ncxy * ncz) return;
  const int I = tid % ncx, J = (tid / ncx) % ncy, K = tid / ncxy;
  const int Im = wrap(I - 1, ncx), Jm = wrap(J - 1, ncy);
  const T* gWz = A.in2;
  const T iHX = A.g.iHX[I], iHXm = A.g.iHX[Im], iHY = A.g.iHY[J], iHYm = A.g.iHY[Jm];
  T tot = T(0);
  for (int p = 0; p < mz; ++p) {
    const int k = K * mz + p;
    const T hz = A.g.hz[k];
    tot += gWz[k * ncxy + J * ncx + I];
    const T c0 = -suffix<T>(K, mz, p, [&](int q) { return gWz[q * ncxy + J * ncx + I]; });
    const T cim = A.wx && I == 0 ? T(0) : -suffix<T>(K, mz, p, [&](int q) { return gWz[q * ncxy + J * ncx + Im]; });
    const T cjm = A.wy && J == 0 ? T(0) : -suffix<T>(K, mz, p, [&](int q) { return gWz[q * ncxy + Jm * ncx + I]; });
    A.out0[k * ncxy + J * ncx + I] += cim * hz * iHXm - c0 * hz * iHX;
    A.out1[k * ncxy + J * ncx + I] += cjm * hz * iHYm - c0 * hz * iHY;
  }
  A.out2[K * ncxy + J * ncx + I] = tot;
  if (K == ncz - 1) A.out2[ncz * ncxy + J * ncx + I] = gWz[A.nz * ncxy + J * ncx + I];
}

// Z2: thread per coarse cell (I, J, K).  in0 = gUz, in1 = gVz; out0 = gU, out1 = gV.
template <typename T>
__global__ void __launch_bounds__(256) tz_split(RefArgs<T> A) {
  const int ncx = A.ncx, ncy = A.ncy, ncz = A.ncz, mz = A.mz;
  const int ncxy = ncx * ncy;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= ncxy * ncz) return;
  const int I = tid % ncx, J = (tid / ncx) % ncy, K = tid / ncxy;
  const T* gU = A.in0;
  const T* gV = A.in1;
  // a low wall face is taken as zero by the forward map: its gradient is zero
  A.out0[K * ncxy + J * ncx + I] =
      A.wx && I == 0 ? T(0)
                     : gather<T>(A.g.Rz, A.g.sz, ncz, mz, false, K, [&](int k) { return gU[k * ncxy + J * ncx + I]; });
  A.out1[K * ncxy + J * ncx + I] =
      A.wy && J == 0 ? T(0)
                     : gather<T>(A.g.Rz, A.g.sz, ncz, mz, false, K, [&](int k) { return gV[k * ncxy + J * ncx + I]; });
}

// ---------------------------------------------------------------- launchers
inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename T>
RefArgs<T> ref_args(mr_ctx* c, const Geom<T>& g) {
  RefArgs<T> a;
  ::memset((void*)&a, 0, sizeof(a));
  a.g = g;
  a.nx = c->nx; a.ny = c->ny; a.nz = c->nz;
  a.ncx = c->ncx; a.ncy = c->ncy; a.ncz = c->ncz;
  a.mx = c->mx; a.my = c->my; a.mz = c->mz;
  a.wx = c->wx; a.wy = c->wy;
  return a;
}

hipError_t ensure(void** buf, size_t* have, size_t need) {
  if (*have >= need) return hipSuccess;
  if (*buf) (void)hipFree(*buf);
  *buf = nullptr;
  *have = 0;
  hipError_t e = hipMalloc(buf, need);
  if (e == hipSuccess) *have = need;
  return e;
}

constexpr int kFusedRows = 6;       // most coarse rows per tile
constexpr int kFusedWgs = 8192;     // workgroups the layer split aims for
constexpr int kFusedMinKc = 4;      // fewest coarse layers per workgroup

// LDS bytes of refine_fused for a tile of TI x TJ coarse cells.
template <typename T>
size_t fused_lds(int TI, int TJ, int mx, int my, int mz) {
  return sizeof(T) * (size_t)(fused_tables(TI, TJ, mx, my) + fused_fields(TI, TJ, my, mz));
}

// The time interpolation of the coarse velocity (Eq. 21, read as the linear
// interpolation (1 - s) level0 + s level1 between the two coarse levels) of
// U, V and W in one launch: n cells of U and V, nw of W.
template <typename T>
struct BlendArgs {
  const T* a[3];
  const T* b[3];
  T* out[3];
  int64_t n, nw;
  T s;
};

template <typename T>
__global__ void __launch_bounds__(256) blend_kernel(BlendArgs<T> A) {
  const int64_t tot = 2 * A.n + A.nw;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x) {
    const int f = q < A.n ? 0 : (q < 2 * A.n ? 1 : 2);
    const int64_t e = q - f * A.n;
    A.out[f][e] = (T(1) - A.s) * A.a[f][e] + A.s * A.b[f][e];
  }
}

// U1/V1/W1 null: refine (U, V, W); otherwise refine (1 - frac) (U, V, W) + frac (U1, V1, W1),
// the blend formed once in the context's buffer (at frac 0 or 1 the level itself).
// Timed at 256^3: the blend followed by the plain refinement took 0.177 ms in
// FP64 and 0.123 ms in FP32, against 0.190 and 0.131 ms for a refinement that
// blended on its coarse loads (those carried both levels' stencil values in
// registers: in FP64 three workgroups a CU instead of four).
template <typename T>
hipError_t refine_t(mr_ctx* c, const Geom<T>& g, const void* U, const void* V, const void* W,
                    const void* U1, const void* V1, const void* W1, double frac, void* u, void* v,
                    void* w, hipStream_t s) {
  if (U1 && frac == 0.0) U1 = V1 = W1 = nullptr;
  if (U1 && frac == 1.0) {
    U = U1; V = V1; W = W1;
    U1 = V1 = W1 = nullptr;
  }
  const int64_t ncl = (int64_t)c->ncx * c->ncy * c->ncz, ncw = ncl + (int64_t)c->ncx * c->ncy;
  const int64_t nbl = U1 ? 2 * ncl + ncw : 0;   // the blended coarse level, at the buffer's start
  int TI = kFuseCols / c->mx;
  int TJ = 0;
  // a walled axis needs every tile (the last one included) to hold at least
  // two cells along it, so that the one-sided stencils stay inside the halo
  while (c->wx && TI >= 2 && c->ncx % TI == 1) --TI;
  if (TI >= 1 && c->mz <= kFuseMaxMz && !(c->wx && TI < 2)) {
    // rows per tile: every stage-z item (one per halo column and row) on its own lane
    TJ = std::min(std::min(kFusedRows, 256 / (TI + 3) - 2), c->ncy);
    while (TJ >= 1 && fused_lds<T>(TI, TJ, c->mx, c->my, c->mz) > kFuseMaxLds) --TJ;
    if (c->wy) {
      while (TJ >= 2 && c->ncy % TJ == 1) --TJ;
      if (TJ < 2) TJ = 0;
    }
  }
  const int64_t zc = (int64_t)c->nz * c->ncy * c->ncx, zc1 = (int64_t)(c->nz + 1) * c->ncy * c->ncx;
  const int64_t yc = (int64_t)c->nz * c->ny * c->ncx, yc1 = (int64_t)(c->nz + 1) * c->ny * c->ncx;
  const size_t need = sizeof(T) * (size_t)(nbl + (TJ >= 1 ? 0 : 2 * zc + zc1 + 2 * yc + yc1));
  if (need > 0) {
    hipError_t e = ensure(&c->interp_tmp, &c->interp_tmp_bytes, need);
    if (e != hipSuccess) return e;
  }
  if (U1) {
    T* Ub = (T*)c->interp_tmp;
    T* Vb = Ub + ncl;
    T* Wb = Vb + ncl;
    BlendArgs<T> b;
    b.a[0] = (const T*)U; b.a[1] = (const T*)V; b.a[2] = (const T*)W;
    b.b[0] = (const T*)U1; b.b[1] = (const T*)V1; b.b[2] = (const T*)W1;
    b.out[0] = Ub; b.out[1] = Vb; b.out[2] = Wb;
    b.n = ncl;
    b.nw = ncw;
    b.s = (T)frac;
    const unsigned nbk = (unsigned)std::min<int64_t>(8192, (nbl + 255) / 256);
    hipLaunchKernelGGL(blend_kernel<T>, dim3(nbk), dim3(256), 0, s, b);
    U = Ub; V = Vb; W = Wb;
  }
  if (TJ >= 1) {
    RefArgs<T> a = ref_args<T>(c, g);
    a.in0 = (const T*)U; a.in1 = (const T*)V; a.in2 = (const T*)W;
    a.out0 = (T*)u; a.out1 = (T*)v; a.out2 = (T*)w;
    const int nbx = (c->ncx + TI - 1) / TI, nby = (c->ncy + TJ - 1) / TJ;
    const int64_t tiles = (int64_t)nbx * nby;
    // coarse layers per workgroup: enough workgroups to fill the chip
    // (at least kFusedMinKc layers each, so that the table set-up and the first
    // layer's loads are shared by a few layers)
    int nkc = (int)std::max<int64_t>(1, std::min<int64_t>(c->ncz, (kFusedWgs + tiles - 1) / tiles));
    nkc = std::min(nkc, std::max(1, c->ncz / kFusedMinKc));
    const int KC = (c->ncz + nkc - 1) / nkc;
    nkc = (c->ncz + KC - 1) / KC;
    const int64_t nb = tiles * nkc;
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    const size_t lds = fused_lds<T>(TI, TJ, c->mx, c->my, c->mz);
    const bool nt = (TI * c->mx * sizeof(T)) % 128 == 0 && (c->nx * sizeof(T)) % 128 == 0;
    const dim3 grid((unsigned)nb), block(256);
    if (nt)
      hipLaunchKernelGGL((refine_fused<T, true>), grid, block, lds, s, a, TI, TJ, nbx, nby, KC);
    else
      hipLaunchKernelGGL((refine_fused<T, false>), grid, block, lds, s, a, TI, TJ, nbx, nby, KC);
    return hipGetLastError();
  }
  T* Uz = (T*)c->interp_tmp + nbl;
  T* Vz = Uz + zc;
  T* Wz = Vz + zc;
  T* Uzy = Wz + zc1;
  T* Vzy = Uzy + yc;
  T* Wzy = Vzy + yc;
  RefArgs<T> a = ref_args<T>(c, g);
  a.in0 = (const T*)U; a.in1 = (const T*)V; a.in2 = (const T*)W;
  a.out0 = Uz; a.out1 = Vz; a.out2 = Wz;
  hipLaunchKernelGGL(stage_z<T>, dim3(nblk((int64_t)c->ncx * c->ncy * c->ncz)), dim3(256), 0, s, a);
  a.in0 = Uz; a.in1 = Vz; a.in2 = Wz;
  a.out0 = Uzy; a.out1 = Vzy; a.out2 = Wzy;
  hipLaunchKernelGGL(stage_y<T>, dim3(nblk(zc)), dim3(256), 0, s, a);
  a.in0 = Uzy; a.in1 = Vzy; a.in2 = Wzy;
  a.out0 = (T*)u; a.out1 = (T*)v; a.out2 = (T*)w;
  hipLaunchKernelGGL(stage_x<T>, dim3(nblk(yc)), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t refine_transpose_t(mr_ctx* c, const Geom<T>& g, const void* gu, const void* gv,
                              const void* gw, void* gU, void* gV, void* gW, hipStream_t s) {
  const int64_t d0 = (int64_t)c->nz * c->ny * c->nx, d1 = (int64_t)(c->nz + 1) * c->ny * c->nx;
  const int64_t zc = (int64_t)c->nz * c->ncy * c->ncx, zc1 = (int64_t)(c->nz + 1) * c->ncy * c->ncx;
  const int64_t yc = (int64_t)c->nz * c->ny * c->ncx, yc1 = (int64_t)(c->nz + 1) * c->ny * c->ncx;
  // stage x transposed in one kernel where a dense row fits (up to 512 coarse
  // cells of at most 4 columns, five dense rows within the LDS budget);
  // otherwise through two dense intermediates
  const bool fused_x = sizeof(T) * 5 * (size_t)c->nx <= kFuseMaxLds && c->ncx <= kRowCells * kRowThreads &&
                       c->mx <= 4;
  const size_t need = sizeof(T) * (size_t)((fused_x ? 0 : d0 + d1) + 2 * yc + yc1 + 2 * zc + zc1);
  hipError_t e = ensure(&c->interp_bwd_tmp, &c->interp_bwd_tmp_bytes, need);
  if (e != hipSuccess) return e;
  T* gv_tot = (T*)c->interp_bwd_tmp;
  T* gw_tot = gv_tot + d0;
  T* gUzy = fused_x ? (T*)c->interp_bwd_tmp : gw_tot + d1;
  T* gVzy = gUzy + yc;
  T* gWzy = gVzy + yc;
  T* gUz = gWzy + yc1;
  T* gVz = gUz + zc;
  T* gWz = gVz + zc;
  RefArgs<T> a = ref_args<T>(c, g);
  a.in0 = (const T*)gu; a.in1 = (const T*)gv; a.in2 = (const T*)gw;
  a.out0 = gUzy;
  if (fused_x) {
    a.out1 = gVzy; a.out2 = gWzy;
    launch_tx_row<T>(c, a, s);
  } else {
    a.out1 = gv_tot; a.out2 = gw_tot;
    hipLaunchKernelGGL(tx_march<T>, dim3(nblk(yc)), dim3(256), 0, s, a);
    a.in1 = gv_tot; a.in2 = gw_tot;
    a.out1 = gVzy; a.out2 = gWzy;
    hipLaunchKernelGGL(tx_split<T>, dim3(nblk(yc1)), dim3(256), 0, s, a);
  }
  // stage y transposed: one kernel for refinement factors up to 4
  a = ref_args<T>(c, g);
  if (c->my <= 4) {
    a.in0 = gUzy; a.in1 = gVzy; a.in2 = gWzy;
    a.out0 = gUz; a.out2 = gWz; a.out3 = gVz;
    const int nrc = (c->ncy + kYRows - 1) / kYRows;
    const int nrowc = (c->ncy + nrc - 1) / nrc;
    const int ntx = (c->ncx + kWave - 1) / kWave;
    const dim3 grid((unsigned)((int64_t)ntx * (c->nz + 1) * ((c->ncy + nrowc - 1) / nrowc))), block(kWave);
    switch (c->my) {
      case 1: hipLaunchKernelGGL((ty_fused<T, 1>), grid, block, 0, s, a, nrowc); break;
      case 2: hipLaunchKernelGGL((ty_fused<T, 2>), grid, block, 0, s, a, nrowc); break;
      case 3: hipLaunchKernelGGL((ty_fused<T, 3>), grid, block, 0, s, a, nrowc); break;
      default: hipLaunchKernelGGL((ty_fused<T, 4>), grid, block, 0, s, a, nrowc); break;
    }
  } else {
    a.in1 = gVzy;
    a.out0 = gUzy; a.out2 = gWzy; a.out3 = gVz;
    hipLaunchKernelGGL(ty_march<T>, dim3(nblk(zc)), dim3(256), 0, s, a);
    a = ref_args<T>(c, g);
    a.in0 = gUzy; a.in2 = gWzy;
    a.out0 = gUz; a.out2 = gWz;
    hipLaunchKernelGGL(ty_split<T>, dim3(nblk(zc1)), dim3(256), 0, s, a);
  }
  // stage z transposed: one kernel for refinement factors up to 4
  a = ref_args<T>(c, g);
  if (c->mz <= 4) {
    a.in0 = gUz; a.in1 = gVz; a.in2 = gWz;
    a.out0 = (T*)gU; a.out1 = (T*)gV; a.out2 = (T*)gW;
    const int nlc = (c->ncz + kZLayers - 1) / kZLayers;
    const int nlayc = (c->ncz + nlc - 1) / nlc;
    const int ntx = (c->ncx + kWave - 1) / kWave, nty = (c->ncy + 3) / 4;
    const dim3 grid((unsigned)((int64_t)ntx * nty * ((c->ncz + nlayc - 1) / nlayc))), block(256);
    switch (c->mz) {
      case 1: hipLaunchKernelGGL((tz_fused<T, 1>), grid, block, 0, s, a, nlayc); break;
      case 2: hipLaunchKernelGGL((tz_fused<T, 2>), grid, block, 0, s, a, nlayc); break;
      case 3: hipLaunchKernelGGL((tz_fused<T, 3>), grid, block, 0, s, a, nlayc); break;
      default: hipLaunchKernelGGL((tz_fused<T, 4>), grid, block, 0, s, a, nlayc); break;
    }
  } else {
    a.in2 = gWz;
    a.out0 = gUz; a.out1 = gVz; a.out2 = (T*)gW;
    hipLaunchKernelGGL(tz_march<T>, dim3(nblk((int64_t)c->ncx * c->ncy * c->ncz)), dim3(256), 0, s, a);
    a = ref_args<T>(c, g);
    a.in0 = gUz; a.in1 = gVz;
    a.out0 = (T*)gU; a.out1 = (T*)gV;
    hipLaunchKernelGGL(tz_split<T>, dim3(nblk((int64_t)c->ncx * c->ncy * c->ncz)), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_refine(mr_ctx* c, const void* U, const void* V, const void* W, void* u, void* v,
                         void* w, hipStream_t s) {
  if (c->precision == MR_FP64)
    return refine_t<double>(c, c->g64, U, V, W, nullptr, nullptr, nullptr, 0.0, u, v, w, s);
  return refine_t<float>(c, c->g32, U, V, W, nullptr, nullptr, nullptr, 0.0, u, v, w, s);
}

hipError_t launch_refine_time(mr_ctx* c, const void* U0, const void* V0, const void* W0,
                              const void* U1, const void* V1, const void* W1, double frac, void* u,
                              void* v, void* w, hipStream_t s) {
  if (c->precision == MR_FP64) return refine_t<double>(c, c->g64, U0, V0, W0, U1, V1, W1, frac, u, v, w, s);
  return refine_t<float>(c, c->g32, U0, V0, W0, U1, V1, W1, frac, u, v, w, s);
}

hipError_t launch_refine_transpose(mr_ctx* c, const void* gu, const void* gv, const void* gw,
                                   void* gU, void* gV, void* gW, hipStream_t s) {
  if (c->precision == MR_FP64) return refine_transpose_t<double>(c, c->g64, gu, gv, gw, gU, gV, gW, s);
  return refine_transpose_t<float>(c, c->g32, gu, gv, gw, gU, gV, gW, s);
}

}  // namespace mr
