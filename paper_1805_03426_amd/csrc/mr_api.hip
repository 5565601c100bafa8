// Host side of the C ABI: descriptor checks, grid tables, device uploads and
// the exported entry points.  Tables follow the paper's grid design (Sec. 3.1),
// the refinement matrices R = A_s A^-1 (Eqs. 12-19) and the implicit z
// diffusion of the scalar step (Eqs. 2, 5-7).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdlib>
#include <new>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "mr_internal.h"

namespace {

using std::vector;

struct Axis {
  int n = 0, m = 1, nc = 0;
  bool periodic = true;
  vector<double> f, h, c, dc;  // faces, widths, centres, centre distances across faces
};

int build_axis(const double* faces, int n, int m, bool periodic, Axis& ax) {
  if (!faces || n < 1 || m < 1 || n % m) return MR_EINVAL;
  ax.n = n;
  ax.m = m;
  ax.nc = n / m;
  ax.periodic = periodic;
  ax.f.assign(faces, faces + n + 1);
  for (int i = 0; i <= n; ++i)
    if (!std::isfinite(ax.f[i])) return MR_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!(ax.f[i + 1] > ax.f[i])) return MR_EINVAL;
  ax.h.resize(n);
  ax.c.resize(n);
  for (int i = 0; i < n; ++i) {
    ax.h[i] = ax.f[i + 1] - ax.f[i];
    ax.c[i] = 0.5 * (ax.f[i] + ax.f[i + 1]);
  }
  if (periodic) {
    const double len = ax.f[n] - ax.f[0];
    ax.dc.resize(n);
    for (int i = 0; i < n; ++i) ax.dc[i] = ax.c[i] - (i ? ax.c[i - 1] : ax.c[n - 1] - len);
  } else {
    ax.dc.resize(n + 1);
    ax.dc[0] = 0.5 * ax.h[0];
    ax.dc[n] = 0.5 * ax.h[n - 1];
    for (int i = 1; i < n; ++i) ax.dc[i] = ax.c[i] - ax.c[i - 1];
  }
  return MR_OK;
}

// True when the widths of the axis are equal to within 1e-13 relative.
bool uniform_axis(const Axis& ax) {
  const double h0 = ax.h[0];
  for (double h : ax.h)
    if (fabs(h - h0) > 1e-13 * h0) return false;
  return true;
}

// Fourth-order face weights of an axis (Sec. 2.2): the stencil of face f is
// the two cells on each side of it, cells f-2..f+1.  On a walled axis only the
// cells that exist take part (three next to a wall cell, two when the axis has
// two cells) and the wall faces get zero rows; on a periodic axis the stencil
// wraps around, the cells beyond an end taking the period added to (or
// subtracted from) their coordinates, and face n repeats face 0.  The face
// value of the polynomial whose cell means equal the cell values is the
// derivative at the face of the polynomial that interpolates the primitive
// P(e_j) = sum_{s<j} h_s theta_s at the stencil's edges e_0..e_m, so cell s
// gets h_s * sum_{j>s} L_j'(x_f), L_j the Lagrange basis on the edges.
// Returns (n+1)*4 weights, face f's for the cells f-2..f+1 in that order.
vector<double> face_weights4(const Axis& ax) {
  const int n = ax.n;
  const double len = ax.f[n] - ax.f[0];
  // left edge of stencil cell c (beyond the ends of a periodic axis: the
  // edge of the cell it wraps to, shifted by whole periods)
  auto edge = [&](int c) {
    if (c >= 0 && c <= n) return ax.f[c];
    const int r = ((c % n) + n) % n;
    return ax.f[r] + (double)((c - r) / n) * len;
  };
  vector<double> w((size_t)(n + 1) * 4, 0.0);
  for (int f = ax.periodic ? 0 : 1; f < n; ++f) {
    int lo = f - 2, hi = f + 1;
    if (!ax.periodic) lo = std::max(lo, 0), hi = std::min(hi, n - 1);
    const int m = hi - lo + 1;
    const double xf = ax.f[f], sc = ax.h[f];
    double e[5];
    for (int q = 0; q <= m; ++q) e[q] = (edge(lo + q) - xf) / sc;
    double dl[5];   // L_j'(0)
    for (int jj = 0; jj <= m; ++jj) {
      double sum = 0.0;
      for (int l = 0; l <= m; ++l) {
        if (l == jj) continue;
        double prod = 1.0 / (e[jj] - e[l]);
        for (int r = 0; r <= m; ++r)
          if (r != jj && r != l) prod *= (0.0 - e[r]) / (e[jj] - e[r]);
        sum += prod;
      }
      dl[jj] = sum;
    }
    for (int q = 0; q < m; ++q) {
      double acc = 0.0;
      for (int jj = q + 1; jj <= m; ++jj) acc += dl[jj];
      w[(size_t)f * 4 + (lo + q - (f - 2))] = (e[q + 1] - e[q]) * acc;
    }
  }
  if (ax.periodic)
    for (int q = 0; q < 4; ++q) w[(size_t)n * 4 + q] = w[q];
  return w;
}

// Means of 1, x, x^2 over [a, b]: a row of A (Eq. 15) or A_s (Eq. 18).
void interval_means(double a, double b, double* row) {
  row[0] = 1.0;
  row[1] = 0.5 * (a + b);
  row[2] = (a * a + a * b + b * b) / 3.0;
}

// Solve the 3x3 system M y = rhs by Gaussian elimination with partial pivoting.
bool solve3(double M[3][3], double rhs[3], double y[3]) {
  int p[3] = {0, 1, 2};
  double A[3][4];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) A[r][c] = M[r][c];
    A[r][3] = rhs[r];
  }
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (A[piv][col] == 0.0) return false;
    if (piv != col)
      for (int c = 0; c < 4; ++c) std::swap(A[piv][c], A[col][c]);
    for (int r = col + 1; r < 3; ++r) {
      const double f = A[r][col] / A[col][col];
      for (int c = col; c < 4; ++c) A[r][c] -= f * A[col][c];
    }
  }
  (void)p;
  for (int r = 2; r >= 0; --r) {
    double s = A[r][3];
    for (int c = r + 1; c < 3; ++c) s -= A[r][c] * y[c];
    y[r] = s / A[r][r];
  }
  return true;
}

int stencil_start(const Axis& ax, int I) {
  if (ax.periodic) return I - 1;
  return std::min(std::max(I - 1, 0), ax.nc - 3);
}

// R_I = A_s A^-1 for every coarse cell (local coordinate (x - centre)/H), and
// the wrapped stencil cell indices.  m = 1 gives R = [0 1 0] on the cell itself.
int refinement_table(const Axis& ax, vector<double>& R, vector<int>& idx, vector<int>& start) {
  const int nc = ax.nc, m = ax.m;
  R.assign((size_t)nc * m * 3, 0.0);
  idx.assign((size_t)nc * 3, 0);
  start.assign(nc, 0);
  if (m == 1) {
    for (int I = 0; I < nc; ++I) {
      R[(size_t)I * 3 + 1] = 1.0;
      for (int r = 0; r < 3; ++r) idx[I * 3 + r] = ((I - 1 + r) % nc + nc) % nc;
      start[I] = I - 1;
    }
    return MR_OK;
  }
  if (nc < 3) return MR_EINVAL;
  const double len = ax.f[ax.n] - ax.f[0];
  for (int I = 0; I < nc; ++I) {
    const double X0 = ax.f[(size_t)I * m], X1 = ax.f[(size_t)(I + 1) * m];
    const double centre = 0.5 * (X0 + X1), H = X1 - X0;
    const int s = stencil_start(ax, I);
    start[I] = s;
    double A[3][3];
    for (int r = 0; r < 3; ++r) {
      int cell = s + r;
      double shift = 0.0;
      if (ax.periodic) {
        if (cell < 0) { cell += nc; shift = -len; }
        if (cell >= nc) { cell -= nc; shift = len; }
      }
      idx[I * 3 + r] = cell;
      const double a = (ax.f[(size_t)cell * m] + shift - centre) / H;
      const double b = (ax.f[(size_t)(cell + 1) * m] + shift - centre) / H;
      interval_means(a, b, A[r]);
    }
    // R A = A_s  <=>  A^T R^T = A_s^T : one 3x3 solve per sub-interval row
    double At[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) At[r][c] = A[c][r];
    for (int q = 0; q < m; ++q) {
      const double a = (ax.f[(size_t)I * m + q] - centre) / H;
      const double b = (ax.f[(size_t)I * m + q + 1] - centre) / H;
      double row[3], y[3];
      interval_means(a, b, row);
      double Mt[3][3];
      memcpy(Mt, At, sizeof(Mt));
      if (!solve3(Mt, row, y)) return MR_EINVAL;
      for (int r = 0; r < 3; ++r) R[((size_t)I * m + q) * 3 + r] = y[r];
    }
  }
  return MR_OK;
}

struct Problem {
  Axis x, y, z;
  double kappa = 0.0;
  bool sweep_ok = false;   // the column-sweep step applies
};

int check_desc(const mr_desc* d, Problem& P) {
  if (!d) return MR_EINVAL;
  if (d->ncx < 1 || d->ncy < 1 || d->ncz < 1 || d->mx < 1 || d->my < 1 || d->mz < 1) return MR_EINVAL;
  const int64_t nx = (int64_t)d->ncx * d->mx, ny = (int64_t)d->ncy * d->my, nz = (int64_t)d->ncz * d->mz;
  if (nx > (1 << 20) || ny > (1 << 20) || nz > (1 << 20)) return MR_ESHAPE;
  if (nx * ny * (nz + 1) > (int64_t)INT32_MAX) return MR_ESHAPE;   // kernels index with int32
  if ((d->mx > 1 && d->ncx < 3) || (d->my > 1 && d->ncy < 3) || (d->mz > 1 && d->ncz < 3)) return MR_EINVAL;
  if (d->bc_bot != MR_DIRICHLET && d->bc_bot != MR_ADIABATIC) return MR_EINVAL;
  if (d->bc_top != MR_DIRICHLET && d->bc_top != MR_ADIABATIC) return MR_EINVAL;
  if (d->precision != MR_FP64 && d->precision != MR_FP32) return MR_EINVAL;
  // the step kernels address a z level with 32-bit byte offsets
  if (nx * ny * (d->precision == MR_FP64 ? 8 : 4) > (int64_t)UINT32_MAX) return MR_ESHAPE;
  if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return MR_EINVAL;
  if (!(d->ra > 0.0) || !(d->pr > 0.0) || !std::isfinite(d->ra * d->pr)) return MR_EINVAL;
  if (d->n_avg < 0) return MR_EINVAL;
  if (!std::isfinite(d->t_bot) || !std::isfinite(d->t_top)) return MR_EINVAL;
  if ((d->side_x != MR_PERIODIC && d->side_x != MR_WALLS) || (d->side_y != MR_PERIODIC && d->side_y != MR_WALLS))
    return MR_EINVAL;
  // explicit z share: up to 1/2 the z part stays unconditionally stable
  if (!(d->z_explicit >= 0.0 && d->z_explicit <= 0.5)) return MR_EINVAL;
  if (d->face_order != 0 && d->face_order != 2 && d->face_order != 4) return MR_EINVAL;
  if (d->step_method < 0 || d->step_method > 2) return MR_EINVAL;
  if (d->sweep_tile < 0 || d->sweep_tile > mr::kSweepShapes) return MR_EINVAL;
  if (d->sweep_tile == 1 && d->precision != MR_FP64) return MR_EINVAL;   // 256 x 4 is FP64 only
  int st;
  if ((st = build_axis(d->xf, (int)nx, d->mx, d->side_x == MR_PERIODIC, P.x)) != MR_OK) return st;
  if ((st = build_axis(d->yf, (int)ny, d->my, d->side_y == MR_PERIODIC, P.y)) != MR_OK) return st;
  if ((st = build_axis(d->zf, (int)nz, d->mz, false, P.z)) != MR_OK) return st;
  P.kappa = 1.0 / sqrt(d->ra * d->pr);
  // explicit x/y diffusion: the leapfrog step is forward Euler over 2 dt
  const double hxm = *std::min_element(P.x.h.begin(), P.x.h.end());
  const double hym = *std::min_element(P.y.h.begin(), P.y.h.end());
  const double num = 2.0 * d->dt * P.kappa * (4.0 / (hxm * hxm) + 4.0 / (hym * hym));
  if (!(num <= 1.0)) return MR_EINVAL;
  // column sweeps: x and y periodic with uniform widths, the plain method
  P.sweep_ok = d->side_x == MR_PERIODIC && d->side_y == MR_PERIODIC && uniform_axis(P.x) &&
               uniform_axis(P.y) && d->z_explicit == 0.0 && d->face_order != 4;
  if (d->step_method == 2 && !P.sweep_ok) return MR_EINVAL;
  // columns beyond the line solver's chunks need the sweeps
  if (nz > (int64_t)mr::kMaxChunks * mr::kChunkLens[2] && (!P.sweep_ok || d->step_method == 1))
    return MR_ESHAPE;
  return MR_OK;
}

double kind_tau(int kind, double dt) {
  return kind == mr::KIND_STARTUP ? dt : (kind == mr::KIND_AVERAGE ? 1.5 * dt : 2.0 * dt);
}

// Tridiagonal I - tk Lz (rows k: sub couples k-1, sup couples k+1) and the
// Dirichlet wall source b_z with Lz theta = Lz0 theta + b_z.
void z_system(const Axis& z, const mr_desc* d, double tk, double* sub, double* diag, double* sup,
              double* bz) {
  const int nz = z.n;
  for (int k = 0; k < nz; ++k) {
    const double lo = k > 0 ? -tk / (z.h[k] * z.dc[k]) : 0.0;
    const double hi = k < nz - 1 ? -tk / (z.h[k] * z.dc[k + 1]) : 0.0;
    if (sub) sub[k] = lo;
    if (sup) sup[k] = hi;
    double dg = 1.0 - lo - hi;
    double b = 0.0;
    if (k == 0 && d->bc_bot == MR_DIRICHLET) {
      dg += tk / (z.h[0] * z.dc[0]);
      b += d->t_bot / (z.h[0] * z.dc[0]);
    }
    if (k == nz - 1 && d->bc_top == MR_DIRICHLET) {
      dg += tk / (z.h[nz - 1] * z.dc[nz]);
      b += d->t_top / (z.h[nz - 1] * z.dc[nz]);
    }
    if (diag) diag[k] = dg;
    if (bz) bz[k] = b;
  }
}

// Host image of one ZSys.
struct ZHost {
  vector<double> m, a, cp, G, B, Fe, Gs, Bs, tkb;
};

// Thomas factors and chunk coupling vectors of the system (sub, diag, sup),
// for chunks [c L, (c+1) L).  The tables are padded to nch*L rows: rows k >= nz
// are identity rows decoupled from the system (m = 1, a = cp = 0), so every
// chunk has exactly L rows.  With the forward sweep d_k = m_k r_k + a_k d_{k-1}
// and back substitution x_k = d_k - cp_k x_{k+1}, a chunk that starts its
// sweeps from zero gets x_hat; the true solution is x_k = x_hat_k + D G_k + X B_k
// with D = d at the level below the chunk and X = x at the level above it.
bool z_factors(int nz, int L, const double* sub, const double* diag, const double* sup, ZHost& z) {
  const int nch = (nz + L - 1) / L;
  const int np = nch * L;
  z.m.assign(np, 1.0); z.a.assign(np, 0.0); z.cp.assign(np, 0.0); z.G.assign(np, 0.0); z.B.assign(np, 0.0);
  z.Fe.resize(nch); z.Gs.resize(nch); z.Bs.resize(nch);
  double cprev = 0.0;
  for (int k = 0; k < nz; ++k) {
    const double den = diag[k] - (k ? sub[k] * cprev : 0.0);
    if (den == 0.0 || !std::isfinite(den)) return false;
    z.m[k] = 1.0 / den;
    z.a[k] = k ? -sub[k] * z.m[k] : 0.0;
    z.cp[k] = k < nz - 1 ? sup[k] * z.m[k] : 0.0;
    cprev = z.cp[k];
  }
  vector<double> F(np);
  for (int c = 0; c < nch; ++c) {
    const int k0 = c * L, k1 = k0 + L;
    double f = 1.0;
    for (int k = k0; k < k1; ++k) { f *= z.a[k]; F[k] = f; }
    double g = 0.0, b = 1.0;
    for (int k = k1 - 1; k >= k0; --k) {
      g = F[k] - z.cp[k] * g;
      z.G[k] = g;
      b *= -z.cp[k];
      z.B[k] = b;
    }
    z.Fe[c] = F[k1 - 1];
    z.Gs[c] = z.G[k0];
    z.Bs[c] = z.B[k0];
  }
  return true;
}

// Factors of the column-sweep steps for the system (sub, diag, sup), both
// elimination directions: upward (the Thomas factors above, back substitution
// downward) and downward (the mirrored recurrences, back substitution upward).
struct SweepHost {
  vector<double> up_m, up_a, up_cb, dn_m, dn_a, dn_cb, tkb;
};

bool sweep_factors(int nz, const double* sub, const double* diag, const double* sup, SweepHost& z) {
  z.up_m.assign(nz, 0.0); z.up_a.assign(nz, 0.0); z.up_cb.assign(nz, 0.0);
  z.dn_m.assign(nz, 0.0); z.dn_a.assign(nz, 0.0); z.dn_cb.assign(nz, 0.0);
  double c = 0.0;
  for (int k = 0; k < nz; ++k) {
    const double den = diag[k] - (k ? sub[k] * c : 0.0);
    if (den == 0.0 || !std::isfinite(den)) return false;
    z.up_m[k] = 1.0 / den;
    z.up_a[k] = k ? -sub[k] * z.up_m[k] : 0.0;
    z.up_cb[k] = k < nz - 1 ? sup[k] * z.up_m[k] : 0.0;
    c = z.up_cb[k];
  }
  c = 0.0;
  for (int k = nz - 1; k >= 0; --k) {
    const double den = diag[k] - (k < nz - 1 ? sup[k] * c : 0.0);
    if (den == 0.0 || !std::isfinite(den)) return false;
    z.dn_m[k] = 1.0 / den;
    z.dn_a[k] = k < nz - 1 ? -sup[k] * z.dn_m[k] : 0.0;
    z.dn_cb[k] = k > 0 ? sub[k] * z.dn_m[k] : 0.0;
    c = z.dn_cb[k];
  }
  return true;
}

// Shortest chunk length that splits nz levels into at most
// kMaxChunks chunks.
int choose_chunks(int nz, int& L, int& nch) {
  for (int l : mr::kChunkLens) {
    if ((nz + l - 1) / l <= mr::kMaxChunks) {
      L = l;
      nch = (nz + l - 1) / l;
      return MR_OK;
    }
  }
  return MR_ESHAPE;
}

// Byte buffer that hands out 256-byte aligned slots.
struct Packer {
  vector<char> buf;
  size_t put(const void* p, size_t bytes) {
    size_t off = (buf.size() + 255) & ~(size_t)255;
    buf.resize(off + bytes);
    if (bytes) memcpy(buf.data() + off, p, bytes);
    return off;
  }
  template <typename T>
  size_t put(const vector<T>& v) { return put(v.data(), v.size() * sizeof(T)); }
};

template <typename T>
vector<T> cast(const vector<double>& v) { return vector<T>(v.begin(), v.end()); }

vector<double> inv(const vector<double>& v) {
  vector<double> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = 1.0 / v[i];
  return o;
}

struct GeomOffsets {
  size_t hx, ihx, idxc, hy, ihy, idyc, hz, ihz, iHX, iHY, Rx, Ry, Rz, sx, sy, sz, zlo, zhi;
  size_t lzl, lzd, lzh, lztl, lzth, c4z, c4zt, c4x, c4y;
};

template <typename T>
GeomOffsets pack_geom(Packer& pk, const Problem& P, const mr_desc* d, const vector<double>* R,
                      const vector<int>* idx, int npad) {
  GeomOffsets o;
  o.hx = pk.put(cast<T>(P.x.h));
  o.ihx = pk.put(cast<T>(inv(P.x.h)));
  o.idxc = pk.put(cast<T>(inv(P.x.dc)));
  o.hy = pk.put(cast<T>(P.y.h));
  o.ihy = pk.put(cast<T>(inv(P.y.h)));
  o.idyc = pk.put(cast<T>(inv(P.y.dc)));
  o.hz = pk.put(cast<T>(P.z.h));
  o.ihz = pk.put(cast<T>(inv(P.z.h)));
  vector<double> HX(P.x.nc), HY(P.y.nc);
  for (int I = 0; I < P.x.nc; ++I) HX[I] = 1.0 / (P.x.f[(size_t)(I + 1) * P.x.m] - P.x.f[(size_t)I * P.x.m]);
  for (int J = 0; J < P.y.nc; ++J) HY[J] = 1.0 / (P.y.f[(size_t)(J + 1) * P.y.m] - P.y.f[(size_t)J * P.y.m]);
  o.iHX = pk.put(cast<T>(HX));
  o.iHY = pk.put(cast<T>(HY));
  o.Rx = pk.put(cast<T>(R[0]));
  o.Ry = pk.put(cast<T>(R[1]));
  o.Rz = pk.put(cast<T>(R[2]));
  o.sx = pk.put(idx[0]);
  o.sy = pk.put(idx[1]);
  o.sz = pk.put(idx[2]);
  // interior-face masks of the z levels (the walls carry no advective flux),
  // zero on the padding rows of the line solver
  vector<double> lo(npad, 0.0), hi(npad, 0.0);
  for (int k = 0; k < P.z.n; ++k) {
    lo[k] = k > 0 ? 1.0 : 0.0;
    hi[k] = k < P.z.n - 1 ? 1.0 : 0.0;
  }
  o.zlo = pk.put(cast<T>(lo));
  o.zhi = pk.put(cast<T>(hi));
  // Lz0 rows and their transpose (a Dirichlet wall adds to the diagonal; its
  // wall value is the separate source b_z)
  const int nz = P.z.n;
  const vector<double>& h = P.z.h;
  const vector<double>& dc = P.z.dc;
  vector<double> zl(npad, 0.0), zd(npad, 0.0), zh(npad, 0.0), ztl(npad, 0.0), zth(npad, 0.0);
  for (int k = 0; k < nz; ++k) {
    zl[k] = k > 0 ? 1.0 / (h[k] * dc[k]) : 0.0;
    zh[k] = k < nz - 1 ? 1.0 / (h[k] * dc[k + 1]) : 0.0;
    double dg = -(zl[k] + zh[k]);
    if (k == 0 && d->bc_bot == MR_DIRICHLET) dg -= 1.0 / (h[0] * dc[0]);
    if (k == nz - 1 && d->bc_top == MR_DIRICHLET) dg -= 1.0 / (h[nz - 1] * dc[nz]);
    zd[k] = dg;
  }
  for (int k = 0; k < nz; ++k) {
    ztl[k] = k > 0 ? zh[k - 1] : 0.0;
    zth[k] = k < nz - 1 ? zl[k + 1] : 0.0;
  }
  o.lzl = pk.put(cast<T>(zl));
  o.lzd = pk.put(cast<T>(zd));
  o.lzh = pk.put(cast<T>(zh));
  o.lztl = pk.put(cast<T>(ztl));
  o.lzth = pk.put(cast<T>(zth));
  // fourth-order z faces, padded: faces 0..npad, cells per level 0..npad-1
  const vector<double> w4 = face_weights4(P.z);
  vector<double> c4((size_t)(npad + 1) * 4, 0.0), c4t((size_t)npad * 4, 0.0);
  for (int f = 0; f <= nz; ++f)
    for (int q = 0; q < 4; ++q) c4[(size_t)f * 4 + q] = w4[(size_t)f * 4 + q];
  for (int k = 0; k < nz; ++k)
    for (int q = 0; q < 4; ++q) {
      const int f = k - 1 + q;   // cell k is slot 3 - q of face k - 1 + q
      if (f >= 0 && f <= nz) c4t[(size_t)k * 4 + q] = w4[(size_t)f * 4 + (3 - q)];
    }
  o.c4z = pk.put(cast<T>(c4));
  o.c4zt = pk.put(cast<T>(c4t));
  o.c4x = pk.put(cast<T>(face_weights4(P.x)));
  o.c4y = pk.put(cast<T>(face_weights4(P.y)));
  return o;
}

template <typename T>
mr::Geom<T> geom_ptrs(char* base, const GeomOffsets& o) {
  mr::Geom<T> g;
  g.hx = (const T*)(base + o.hx); g.ihx = (const T*)(base + o.ihx); g.idxc = (const T*)(base + o.idxc);
  g.hy = (const T*)(base + o.hy); g.ihy = (const T*)(base + o.ihy); g.idyc = (const T*)(base + o.idyc);
  g.hz = (const T*)(base + o.hz); g.ihz = (const T*)(base + o.ihz);
  g.iHX = (const T*)(base + o.iHX); g.iHY = (const T*)(base + o.iHY);
  g.Rx = (const T*)(base + o.Rx); g.Ry = (const T*)(base + o.Ry); g.Rz = (const T*)(base + o.Rz);
  g.sx = (const int*)(base + o.sx); g.sy = (const int*)(base + o.sy); g.sz = (const int*)(base + o.sz);
  g.zlo = (const T*)(base + o.zlo); g.zhi = (const T*)(base + o.zhi);
  g.lzl = (const T*)(base + o.lzl); g.lzd = (const T*)(base + o.lzd); g.lzh = (const T*)(base + o.lzh);
  g.lztl = (const T*)(base + o.lztl); g.lzth = (const T*)(base + o.lzth);
  g.c4z = (const T*)(base + o.c4z); g.c4zt = (const T*)(base + o.c4zt);
  g.c4x = (const T*)(base + o.c4x); g.c4y = (const T*)(base + o.c4y);
  return g;
}

struct ZOffsets {
  size_t m, a, cp, G, B, Fe, Gs, Bs, tkb;
};

ZOffsets pack_z(Packer& pk, const ZHost& z) {
  ZOffsets o;
  o.m = pk.put(z.m); o.a = pk.put(z.a); o.cp = pk.put(z.cp); o.G = pk.put(z.G); o.B = pk.put(z.B);
  o.Fe = pk.put(z.Fe); o.Gs = pk.put(z.Gs); o.Bs = pk.put(z.Bs); o.tkb = pk.put(z.tkb);
  return o;
}

struct SweepOffsets {
  size_t up_m, up_a, up_cb, dn_m, dn_a, dn_cb, tkb;
};

SweepOffsets pack_sweep(Packer& pk, const SweepHost& z) {
  SweepOffsets o;
  o.up_m = pk.put(z.up_m); o.up_a = pk.put(z.up_a); o.up_cb = pk.put(z.up_cb);
  o.dn_m = pk.put(z.dn_m); o.dn_a = pk.put(z.dn_a); o.dn_cb = pk.put(z.dn_cb);
  o.tkb = pk.put(z.tkb);
  return o;
}

mr::SweepSys sweep_ptrs(char* base, const SweepOffsets& o) {
  mr::SweepSys z;
  z.up_m = (const double*)(base + o.up_m); z.up_a = (const double*)(base + o.up_a);
  z.up_cb = (const double*)(base + o.up_cb); z.dn_m = (const double*)(base + o.dn_m);
  z.dn_a = (const double*)(base + o.dn_a); z.dn_cb = (const double*)(base + o.dn_cb);
  z.tkb = (const double*)(base + o.tkb);
  return z;
}

mr::ZSys z_ptrs(char* base, const ZOffsets& o) {
  mr::ZSys z;
  z.m = (const double*)(base + o.m); z.a = (const double*)(base + o.a); z.cp = (const double*)(base + o.cp);
  z.G = (const double*)(base + o.G); z.B = (const double*)(base + o.B);
  z.Fe = (const double*)(base + o.Fe); z.Gs = (const double*)(base + o.Gs); z.Bs = (const double*)(base + o.Bs);
  z.tkb = (const double*)(base + o.tkb);
  return z;
}

int hip_fail(mr_ctx* c, hipError_t e) {
  if (c) c->last_err = (int)e;
  (void)hipGetLastError();
  return MR_EHIP;
}

inline hipStream_t as_stream(void* s) { return (hipStream_t)s; }

size_t elem_size(const mr_ctx* c) { return c->precision == MR_FP64 ? 8 : 4; }

// A roctx range named after an entry point, around its host work and its
// launches, so that a marker trace (rocprofv3 --marker-trace) shows each call
// beside the kernels it enqueued.
struct CallRange {
  explicit CallRange(const char* name) { roctxRangePushA(name); }
  ~CallRange() { roctxRangePop(); }
  CallRange(const CallRange&) = delete;
  CallRange& operator=(const CallRange&) = delete;
};

}  // namespace

#define MR_CALL_RANGE() CallRange mr_call_range_(__func__)

// ===================================================================== C ABI
extern "C" {

const char* mr_status_string(int status) {
  switch (status) {
    case MR_OK: return "ok";
    case MR_EINVAL: return "invalid argument";
    case MR_ESHAPE: return "unsupported size";
    case MR_EHIP: return "HIP runtime error";
    case MR_ENOMEM: return "out of device memory";
    case MR_ENONFINITE: return "non-finite value in reduction";
    default: return "unknown status";
  }
}

int mr_last_hip_error(const mr_ctx* ctx) { return ctx ? ctx->last_err : 0; }

int mr_get_step_method(const mr_ctx* ctx, int32_t* method) {
  if (!ctx || !method) return MR_EINVAL;
  *method = ctx->sweep_pref ? 2 : 1;
  return MR_OK;
}

int mr_get_dims(const mr_ctx* ctx, int32_t* nx, int32_t* ny, int32_t* nz, int32_t* precision) {
  if (!ctx) return MR_EINVAL;
  if (nx) *nx = ctx->nx;
  if (ny) *ny = ctx->ny;
  if (nz) *nz = ctx->nz;
  if (precision) *precision = ctx->precision;
  return MR_OK;
}

int mr_host_refinement_table(const mr_desc* desc, int32_t axis, double* R_out, int32_t* start_out) {
  Problem P;
  int st = check_desc(desc, P);
  if (st != MR_OK) return st;
  if (axis < 0 || axis > 2) return MR_EINVAL;
  const Axis& ax = axis == 0 ? P.x : (axis == 1 ? P.y : P.z);
  vector<double> R;
  vector<int> idx, start;
  if ((st = refinement_table(ax, R, idx, start)) != MR_OK) return st;
  if (R_out) memcpy(R_out, R.data(), R.size() * sizeof(double));
  if (start_out)
    for (int I = 0; I < ax.nc; ++I) start_out[I] = start[I];
  return MR_OK;
}

int mr_host_z_system(const mr_desc* desc, int64_t n, double* sub, double* diag, double* sup,
                     double* bz, double* tau_out) {
  Problem P;
  int st = check_desc(desc, P);
  if (st != MR_OK) return st;
  if (n < 0) return MR_EINVAL;
  const double tau = kind_tau(mr::step_kind(n, desc->n_avg), desc->dt);
  z_system(P.z, desc, tau * P.kappa * (1.0 - desc->z_explicit), sub, diag, sup, bz);
  if (tau_out) *tau_out = tau;
  return MR_OK;
}

int mr_host_z_face_weights(const mr_desc* desc, double* w_out) {
  Problem P;
  int st = check_desc(desc, P);
  if (st != MR_OK) return st;
  if (!w_out) return MR_EINVAL;
  const vector<double> w = face_weights4(P.z);
  memcpy(w_out, w.data(), w.size() * sizeof(double));
  return MR_OK;
}

int mr_host_face_weights(const mr_desc* desc, int32_t axis, double* w_out) {
  Problem P;
  int st = check_desc(desc, P);
  if (st != MR_OK) return st;
  if (!w_out || axis < 0 || axis > 2) return MR_EINVAL;
  const vector<double> w = face_weights4(axis == 0 ? P.x : (axis == 1 ? P.y : P.z));
  memcpy(w_out, w.data(), w.size() * sizeof(double));
  return MR_OK;
}

int mr_init(const mr_desc* desc, mr_ctx** out) {
  MR_CALL_RANGE();
  if (!out) return MR_EINVAL;
  Problem P;
  int st = check_desc(desc, P);
  if (st != MR_OK) return st;
  int L = 0, nch = 0;
  // columns taller than the line solver's chunks: only the column-sweep step
  // (check_desc has made sure that it applies)
  if (choose_chunks(P.z.n, L, nch) != MR_OK) L = nch = 0;
  const int npad = std::max(nch * L, P.z.n);

  vector<double> R[3];
  vector<int> idx[3], start[3];
  const Axis* axes[3] = {&P.x, &P.y, &P.z};
  for (int a = 0; a < 3; ++a)
    if ((st = refinement_table(*axes[a], R[a], idx[a], start[a])) != MR_OK) return st;

  Packer pk;
  GeomOffsets o64 = pack_geom<double>(pk, P, desc, R, idx, npad);
  GeomOffsets o32 = pack_geom<float>(pk, P, desc, R, idx, npad);
  ZOffsets zfo[mr::NKINDS], zto[mr::NKINDS];
  SweepOffsets swo[mr::NKINDS], swto[mr::NKINDS];
  double taus[mr::NKINDS];
  const int nz = P.z.n;
  vector<double> sub(nz), diag(nz), sup(nz), bz(nz), tsub(nz), tsup(nz);
  for (int kind = 0; kind < mr::NKINDS; ++kind) {
    const double tau = kind_tau(kind, desc->dt);
    taus[kind] = tau;
    const double tk = tau * P.kappa;
    // the implicit share (1 - w) of the z diffusion; the wall source stays whole
    z_system(P.z, desc, tk * (1.0 - desc->z_explicit), sub.data(), diag.data(), sup.data(), bz.data());
    SweepHost sh;
    if (!sweep_factors(nz, sub.data(), diag.data(), sup.data(), sh)) return MR_EINVAL;
    sh.tkb.assign(nz, 0.0);
    for (int k = 0; k < nz; ++k) sh.tkb[k] = tk * bz[k];
    swo[kind] = pack_sweep(pk, sh);
    // transpose: sub^T_k = sup_{k-1}, sup^T_k = sub_{k+1}
    for (int k = 0; k < nz; ++k) {
      tsub[k] = k > 0 ? sup[k - 1] : 0.0;
      tsup[k] = k < nz - 1 ? sub[k + 1] : 0.0;
    }
    SweepHost sht;   // the reverse steps' systems: no wall source
    if (!sweep_factors(nz, tsub.data(), diag.data(), tsup.data(), sht)) return MR_EINVAL;
    sht.tkb.assign(nz, 0.0);
    swto[kind] = pack_sweep(pk, sht);
    if (nch == 0) continue;
    ZHost zh, th;
    if (!z_factors(nz, L, sub.data(), diag.data(), sup.data(), zh)) return MR_EINVAL;
    zh.tkb.assign((size_t)nch * L, 0.0);
    for (int k = 0; k < nz; ++k) zh.tkb[k] = tk * bz[k];
    if (!z_factors(nz, L, tsub.data(), diag.data(), tsup.data(), th)) return MR_EINVAL;
    th.tkb.assign((size_t)nch * L, 0.0);
    zfo[kind] = pack_z(pk, zh);
    zto[kind] = pack_z(pk, th);
  }
  // identity factors for the start-up step's reverse sweep (no solve)
  SweepHost shid;
  shid.up_m.assign(nz, 1.0); shid.dn_m.assign(nz, 1.0);
  shid.up_a.assign(nz, 0.0); shid.dn_a.assign(nz, 0.0);
  shid.up_cb.assign(nz, 0.0); shid.dn_cb.assign(nz, 0.0);
  shid.tkb.assign(nz, 0.0);
  const SweepOffsets swido = pack_sweep(pk, shid);
  vector<double> dcz(P.z.dc);
  size_t o_hx64 = pk.put(P.x.h), o_hy64 = pk.put(P.y.h), o_dcz = pk.put(dcz), o_hz64 = pk.put(P.z.h);

  mr_ctx* c = new (std::nothrow) mr_ctx();
  if (!c) return MR_ENOMEM;
  memset((void*)c, 0, sizeof(mr_ctx));
  c->nx = P.x.n; c->ny = P.y.n; c->nz = P.z.n;
  c->ncx = P.x.nc; c->ncy = P.y.nc; c->ncz = P.z.nc;
  c->mx = desc->mx; c->my = desc->my; c->mz = desc->mz;
  c->precision = desc->precision;
  c->kappa = P.kappa; c->dt = desc->dt; c->ra = desc->ra; c->pr = desc->pr;
  c->t_bot = desc->t_bot; c->t_top = desc->t_top;
  c->bc_bot = desc->bc_bot; c->bc_top = desc->bc_top; c->n_avg = desc->n_avg;
  c->wx = desc->side_x == MR_WALLS;
  c->wy = desc->side_y == MR_WALLS;
  c->z_explicit = desc->z_explicit;
  c->face_order = desc->face_order == 4 ? 4 : 2;
  c->uniform_xy = !c->wx && !c->wy && uniform_axis(P.x) && uniform_axis(P.y);
  c->uhx = P.x.n / (P.x.f[P.x.n] - P.x.f[0]);
  c->uhy = P.y.n / (P.y.f[P.y.n] - P.y.f[0]);
  c->L = L; c->nch = nch;
  for (int k = 0; k < mr::NKINDS; ++k) c->tau[k] = taus[k];
  {
    // total horizontal area, compensated
    double s = 0.0, comp = 0.0;
    for (int j = 0; j < P.y.n; ++j)
      for (int i = 0; i < P.x.n; ++i) {
        const double v = P.x.h[i] * P.y.h[j];
        const double t = s + v;
        comp += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
        s = t;
      }
    c->atot = s + comp;
    c->vtot = c->atot * (P.z.f[P.z.n] - P.z.f[0]);
  }
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) { int r = hip_fail(c, e); delete c; return r; }
  // the allocation-free entry point's fixed memory on this device
  e = mr::scratch_init(c->device);
  if (e != hipSuccess) { int r = hip_fail(c, e); delete c; return r; }
  e = hipMalloc(&c->tables, pk.buf.size());
  if (e != hipSuccess) { delete c; (void)hipGetLastError(); return MR_ENOMEM; }
  e = hipMemcpy(c->tables, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { (void)hipFree(c->tables); int r = hip_fail(c, e); delete c; return r; }
  char* base = (char*)c->tables;
  c->g64 = geom_ptrs<double>(base, o64);
  c->g32 = geom_ptrs<float>(base, o32);
  for (int k = 0; k < mr::NKINDS; ++k) {
    if (nch > 0) {
      c->zf[k] = z_ptrs(base, zfo[k]);
      c->zt[k] = z_ptrs(base, zto[k]);
    }
    c->sw[k] = sweep_ptrs(base, swo[k]);
    c->swt[k] = sweep_ptrs(base, swto[k]);
  }
  c->swid = sweep_ptrs(base, swido);
  // step sequences run as column sweeps where the line solver cannot take the
  // columns, and where the sweep's tiles keep the GPU full: at least 16
  // wavefronts per CU in all, and either one round of tiles (one workgroup
  // per CU: the sweep kernels run 4 wavefronts per SIMD) or rounds at least
  // 3/4 full.  Measured in one run: at 256^3 (64 tiles of 256 x 4 columns)
  // the line solver is 2.7x (FP64) and 2.5x (FP32) faster; at 576^3 (432
  // tiles of 192 x 4) the sweeps are 10% and 20% faster; at 1024 x 1024 x 512
  // (1024 tiles) 27% and 25% faster.
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1)
    cus = 256;
  const bool f64 = c->precision == MR_FP64;
  c->sweep_shape = desc->sweep_tile > 0 ? desc->sweep_tile - 1 : mr::sweep_pick_shape(c->nx, f64);
  const mr::SweepShape sh = mr::kSweepShape[c->sweep_shape];
  const int tw = 64 * sh.segs;
  const int64_t tiles = (int64_t)((c->nx + tw - 1) / tw) * ((c->ny + sh.rows - 1) / sh.rows);
  const int64_t slots = cus, rounds = (tiles + slots - 1) / slots;
  const bool fills = tiles * sh.segs * sh.rows >= 16 * (int64_t)cus && (rounds == 1 || 4 * tiles >= 3 * rounds * slots);
  c->sweep_pref = desc->step_method == 2 || (desc->step_method == 0 && P.sweep_ok && (nch == 0 || fills));
  c->sweep_single = nch == 0 || desc->step_method == 2;
  c->hx64 = (const double*)(base + o_hx64);
  c->areaw = (const double*)(base + o_hy64);
  c->dcz = (const double*)(base + o_dcz);
  c->hz64 = (const double*)(base + o_hz64);
  *out = c;
  return MR_OK;
}

int mr_destroy(mr_ctx* ctx) {
  if (!ctx) return MR_OK;
  if (ctx->tables) (void)hipFree(ctx->tables);
  if (ctx->interp_tmp) (void)hipFree(ctx->interp_tmp);
  if (ctx->interp_bwd_tmp) (void)hipFree(ctx->interp_bwd_tmp);
  if (ctx->red) (void)hipFree(ctx->red);
  for (void* p : ctx->sweep_e)
    if (p) (void)hipFree(p);
  delete ctx;
  return MR_OK;
}

#define MR_LAUNCH(call)                              \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(ctx, e_);  \
  } while (0)

int mr_interpolate_velocity(mr_ctx* ctx, const void* U, const void* V, const void* W, void* u,
                            void* v, void* w, void* stream) {
  MR_CALL_RANGE();
  if (!ctx || !U || !V || !W || !u || !v || !w) return MR_EINVAL;
  MR_LAUNCH(mr::launch_refine(ctx, U, V, W, u, v, w, as_stream(stream)));
  return MR_OK;
}

int mr_interpolate_velocity_backward(mr_ctx* ctx, const void* gu, const void* gv, const void* gw,
                                     void* gU, void* gV, void* gW, void* stream) {
  MR_CALL_RANGE();
  if (!ctx || !gu || !gv || !gw || !gU || !gV || !gW) return MR_EINVAL;
  MR_LAUNCH(mr::launch_refine_transpose(ctx, gu, gv, gw, gU, gV, gW, as_stream(stream)));
  return MR_OK;
}

int mr_divergence(mr_ctx* ctx, const void* u, const void* v, const void* w, double* dev_out,
                  void* stream) {
  MR_CALL_RANGE();
  if (!ctx || !u || !v || !w || !dev_out) return MR_EINVAL;
  MR_LAUNCH(mr::launch_divergence(ctx, u, v, w, dev_out, as_stream(stream)));
  return MR_OK;
}

int mr_scalar_step(mr_ctx* ctx, int64_t n, const void* th_prev, const void* th_cur, void* th_next,
                   const void* u, const void* v, const void* w, void* stream) {
  MR_CALL_RANGE();
  if (!ctx || n < 0 || !th_cur || !th_next || !u || !v || !w) return MR_EINVAL;
  if (n > 0 && !th_prev) return MR_EINVAL;
  if (th_next == th_cur || th_next == th_prev) return MR_EINVAL;
  const void* thp = n > 0 ? th_prev : th_cur;
  if (ctx->sweep_single) {
    // one column sweep and its back substitution
    void* outs[1] = {th_next};
    MR_LAUNCH(mr::launch_sweep_steps(ctx, n, 1, thp, th_cur, outs, u, v, w, as_stream(stream)));
    return MR_OK;
  }
  MR_LAUNCH(mr::launch_step(ctx, n, thp, th_cur, th_next, u, v, w, as_stream(stream)));
  return MR_OK;
}

int mr_scalar_steps(mr_ctx* ctx, int64_t n0, int32_t count, const void* th_prev, const void* th_cur,
                    void* const* outs, const void* u, const void* v, const void* w, void* stream) {
  MR_CALL_RANGE();
  if (!ctx || n0 < 0 || count < 1 || !th_cur || !outs || !u || !v || !w) return MR_EINVAL;
  if (n0 > 0 && !th_prev) return MR_EINVAL;
  const void* thp = n0 > 0 ? th_prev : th_cur;
  // every output differs from the two levels before it
  for (int32_t q = 0; q < count; ++q) {
    const void* l1 = q >= 1 ? outs[q - 1] : th_cur;
    const void* l2 = q >= 2 ? outs[q - 2] : (q == 1 ? th_cur : thp);
    if (!outs[q] || outs[q] == l1 || outs[q] == l2) return MR_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  if (ctx->sweep_pref) {
    MR_LAUNCH(mr::launch_sweep_steps(ctx, n0, count, thp, th_cur, outs, u, v, w, s));
    return MR_OK;
  }
  for (int32_t q = 0; q < count; ++q) {
    const void* a = q >= 2 ? outs[q - 2] : (q == 1 ? th_cur : thp);
    const void* b = q >= 1 ? outs[q - 1] : th_cur;
    MR_LAUNCH(mr::launch_step(ctx, n0 + q, a, b, outs[q], u, v, w, s));
  }
  return MR_OK;
}

int mr_adjoint_seed(mr_ctx* ctx, int64_t n, const void* lam, void* mu_out, void* stream) {
  MR_CALL_RANGE();
  if (!ctx || n < 0 || !lam || !mu_out || lam == mu_out) return MR_EINVAL;
  if (ctx->nch == 0) {
    // columns beyond the line solver: a column-by-column solve
    MR_LAUNCH(mr::launch_sweep_seed(ctx, n, lam, mu_out, as_stream(stream)));
    return MR_OK;
  }
  MR_LAUNCH(mr::launch_seed(ctx, n, lam, mu_out, as_stream(stream)));
  return MR_OK;
}

int mr_scalar_step_backward(mr_ctx* ctx, int64_t n, const void* mu_next, const void* mu_cur,
                            const void* lam_add, void* out, const void* u, const void* v,
                            const void* w, void* stream) {
  MR_CALL_RANGE();
  if (!ctx || n < 0 || !mu_cur || !out || !u || !v || !w) return MR_EINVAL;
  if (out == mu_cur || (mu_next && out == mu_next) || (lam_add && out == lam_add)) return MR_EINVAL;
  if (ctx->nch == 0) {
    // columns beyond the line solver: the reverse step as a column sweep
    // and its back substitution (no lam_add there)
    if (lam_add) return MR_ESHAPE;
    hipStream_t s = as_stream(stream);
    if (n == 0) {
      MR_LAUNCH(mr::launch_sweep_bwd0(ctx, mu_next, mu_cur, out, u, v, w, s));
    } else {
      void* outs[1] = {out};
      MR_LAUNCH(mr::launch_sweep_bwd_steps(ctx, n, 1, mu_next, mu_cur, outs, u, v, w, s));
    }
    return MR_OK;
  }
  MR_LAUNCH(mr::launch_step_backward(ctx, n, mu_next, mu_cur, lam_add, out, u, v, w,
                                     as_stream(stream)));
  return MR_OK;
}

int mr_scalar_steps_backward(mr_ctx* ctx, int64_t n0, int32_t count, const void* mu_next, const void* mu_cur,
                             void* const* outs, const void* u, const void* v, const void* w, void* stream) {
  MR_CALL_RANGE();
  if (!ctx || count < 1 || n0 - count + 1 < 1 || !mu_cur || !outs || !u || !v || !w) return MR_EINVAL;
  // every output differs from the two levels before it
  for (int32_t q = 0; q < count; ++q) {
    const void* l1 = q >= 1 ? outs[q - 1] : mu_cur;
    const void* l2 = q >= 2 ? outs[q - 2] : (q == 1 ? mu_cur : mu_next);
    if (!outs[q] || outs[q] == l1 || outs[q] == l2) return MR_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  if (ctx->sweep_pref) {
    MR_LAUNCH(mr::launch_sweep_bwd_steps(ctx, n0, count, mu_next, mu_cur, outs, u, v, w, s));
    return MR_OK;
  }
  if (ctx->nch == 0) return MR_ESHAPE;
  for (int32_t q = 0; q < count; ++q) {
    const void* nxt = q >= 2 ? outs[q - 2] : (q == 1 ? mu_cur : mu_next);
    const void* cur = q >= 1 ? outs[q - 1] : mu_cur;
    MR_LAUNCH(mr::launch_step_backward(ctx, n0 - q, nxt, cur, nullptr, outs[q], u, v, w, s));
  }
  return MR_OK;
}

int mr_velocity_grad(mr_ctx* ctx, int32_t count, const int64_t* steps, const void* const* thetas,
                     const void* const* mus, void* gu, void* gv, void* gw, void* stream) {
  MR_CALL_RANGE();
  if (!ctx || count < 1 || count > 16 || !steps || !thetas || !mus || !gu || !gv || !gw)
    return MR_EINVAL;
  for (int s = 0; s < count; ++s)
    if (steps[s] < 0 || !thetas[s] || !mus[s]) return MR_EINVAL;
  MR_LAUNCH(mr::launch_velocity_grad(ctx, count, steps, thetas, mus, gu, gv, gw, as_stream(stream)));
  return MR_OK;
}

int mr_nusselt(mr_ctx* ctx, const void* theta, const void* w, double* dev_profile, mr_nu* host_out,
               void* stream) {
  MR_CALL_RANGE();
  if (!ctx || !theta || !w || !dev_profile) return MR_EINVAL;
  hipStream_t s = as_stream(stream);
  MR_LAUNCH(mr::launch_nusselt(ctx, theta, w, dev_profile, s));
  if (host_out) {
    double tmp[5];
    MR_LAUNCH(hipMemcpyAsync(tmp, dev_profile + ctx->nz + 1, sizeof(tmp), hipMemcpyDeviceToHost, s));
    MR_LAUNCH(hipStreamSynchronize(s));
    host_out->nu_bot = tmp[0];
    host_out->nu_top = tmp[1];
    host_out->nu_vol = tmp[2];
    host_out->nu_paper = tmp[3];
    host_out->mean_theta = tmp[4];
    for (double t : tmp)
      if (!std::isfinite(t)) return MR_ENONFINITE;
  }
  return MR_OK;
}

int mr_nusselt_noalloc(mr_ctx* ctx, const void* theta, const void* w, double* dev_profile,
                       void* stream) {
  MR_CALL_RANGE();
  if (!ctx || !theta || !w || !dev_profile) return MR_EINVAL;
  return mr::nusselt_fixed(ctx, theta, w, dev_profile, as_stream(stream));
}

int mr_thermal_dissipation(mr_ctx* ctx, const void* theta, double* dev_out, double* host_out,
                           void* stream) {
  MR_CALL_RANGE();
  if (!ctx || !theta || !dev_out) return MR_EINVAL;
  hipStream_t s = as_stream(stream);
  MR_LAUNCH(mr::launch_dissipation(ctx, theta, dev_out, s));
  if (host_out) {
    MR_LAUNCH(hipMemcpyAsync(host_out, dev_out, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    MR_LAUNCH(hipStreamSynchronize(s));
    for (int q = 0; q < 4; ++q)
      if (!std::isfinite(host_out[q])) return MR_ENONFINITE;
  }
  return MR_OK;
}

int mr_interpolate_velocity_time(mr_ctx* ctx, const void* U0, const void* V0, const void* W0,
                                 const void* U1, const void* V1, const void* W1, int64_t i,
                                 int64_t mt, void* u, void* v, void* w, void* stream) {
  MR_CALL_RANGE();
  if (!ctx || !U0 || !V0 || !W0 || !U1 || !V1 || !W1 || !u || !v || !w) return MR_EINVAL;
  if (mt < 1 || i < 0 || i > mt) return MR_EINVAL;
  MR_LAUNCH(mr::launch_refine_time(ctx, U0, V0, W0, U1, V1, W1, (double)i / (double)mt, u, v, w,
                                   as_stream(stream)));
  return MR_OK;
}

int mr_integrate_scalar(mr_ctx* ctx, const void* theta, void* theta_c, void* stream) {
  MR_CALL_RANGE();
  if (!ctx || !theta || !theta_c || theta == theta_c) return MR_EINVAL;
  MR_LAUNCH(mr::launch_integrate(ctx, theta, theta_c, as_stream(stream)));
  return MR_OK;
}

int mr_coarse_step(mr_ctx* ctx, int64_t n0, int32_t mt, const void* U0, const void* V0,
                   const void* W0, const void* U1, const void* V1, const void* W1, void* u, void* v,
                   void* w, void* const* ring, int32_t* prev, int32_t* cur, void* theta_c,
                   void* stream) {
  MR_CALL_RANGE();
  if (!ctx || n0 < 0 || mt < 1 || !U0 || !V0 || !W0 || !U1 || !V1 || !W1 || !u || !v || !w)
    return MR_EINVAL;
  if (!ring || !prev || !cur) return MR_EINVAL;
  int p = *prev, c = *cur;
  if (c < 0 || c > 2 || (n0 > 0 && (p < 0 || p > 2 || p == c))) return MR_EINVAL;
  if (!ring[0] || !ring[1] || !ring[2] || ring[0] == ring[1] || ring[0] == ring[2] ||
      ring[1] == ring[2])
    return MR_EINVAL;
  if (n0 == 0) p = c;
  hipStream_t s = as_stream(stream);
  if (ctx->sweep_pref) {
    // column sweeps: the kernel of sub-step i finishes theta^{n0+i-1} and
    // starts sub-step i on the velocity refined just before it (the velocity
    // at the start of the sub-step, fraction (i-1)/mt)
    const int c0 = c;
    for (int32_t i = 1; i <= mt; ++i) {
      MR_LAUNCH(mr::launch_refine_time(ctx, U0, V0, W0, U1, V1, W1, (double)(i - 1) / (double)mt, u, v, w, s));
      const int q = i - 1;
      int o = 0;
      while (o == c || o == p) ++o;
      // q = 0 reads theta^{n0} itself; q > 0 writes theta^{n0+q} into the free buffer
      MR_LAUNCH(mr::launch_sweep_step(ctx, n0, q, q == 0 ? ring[p] : ring[c], ring[c0],
                                      q == 0 ? nullptr : ring[o], u, v, w, s));
      if (q > 0) {
        p = c;
        c = o;
      }
    }
    int o = 0;
    while (o == c || o == p) ++o;
    MR_LAUNCH(mr::launch_sweep_finish(ctx, n0, mt, ring[o], s));
    p = c;
    c = o;
  } else {
    for (int32_t i = 1; i <= mt; ++i) {
      MR_LAUNCH(mr::launch_refine_time(ctx, U0, V0, W0, U1, V1, W1, (double)(i - 1) / (double)mt, u, v, w, s));
      const int64_t n = n0 + i - 1;
      int o = 0;
      while (o == c || o == p) ++o;   // the buffer holding neither level
      MR_LAUNCH(mr::launch_step(ctx, n, ring[p], ring[c], ring[o], u, v, w, s));
      p = c;
      c = o;
    }
  }
  if (theta_c) MR_LAUNCH(mr::launch_integrate(ctx, ring[c], theta_c, s));
  *prev = p;
  *cur = c;
  return MR_OK;
}

int mr_copy_probe(const void* src, void* dst, int64_t nbytes, void* stream) {
  if (!src || !dst || nbytes < 0 || (nbytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
    return MR_EINVAL;
  hipError_t e = mr::launch_copy(src, dst, nbytes, as_stream(stream));
  if (e != hipSuccess) { (void)hipGetLastError(); return MR_EHIP; }
  return MR_OK;
}

}  // extern "C"
