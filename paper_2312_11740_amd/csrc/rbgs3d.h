// Red-black Gauss-Seidel sweep, one pass over memory, on 3D tiles loaded at once.
//
// Same semantics as the z-marching sweep (two one-colour half sweeps, out of place):
//   x1  = x_in with every c1 cell set to (sum_f w_f x_in[nb] - h^2 b) / sum_f w_f,
//   out = x1  with every c2 cell set to (sum_f w_f x1[nb]  - h^2 b) / sum_f w_f.
// A block owns a tile of SX x SY x SZ cells (32 x 8 x 8 with 512 threads; on small
// grids, where the sweep is latency-bound, 16 x 8 x 4 with 256 threads or 8 x 8 x 4 with
// 128 give more blocks).  It issues every load of its inputs together (x_in on the tile
// and a two-cell ring, b and the finest-level code on the tile and a one-cell ring), so
// each block has its whole input in flight instead of one plane; then the c1 values on
// tile + ring, a barrier, the c2 values on the tile.  The ring reads of neighbouring
// tiles hit L2 (tiles are handed out in x-fastest order per XCD).
#pragma once

#include "rbgs.h"

namespace mpp {

// tile shapes: 0 = 32 x 8 x 8 / 512 threads, 1 = 16 x 8 x 4 / 256, 2 = 8 x 8 x 4 / 128
template <int SHAPE>
struct Shape3;
template <>
struct Shape3<0> {
  static constexpr int X = 32, Y = 8, Z = 8, Threads = 512;
};
template <>
struct Shape3<1> {
  static constexpr int X = 16, Y = 8, Z = 4, Threads = 256;
};
template <>
struct Shape3<2> {
  static constexpr int X = 8, Y = 8, Z = 4, Threads = 128;
};
constexpr int k3Shapes = 3;

struct Tiles3 {
  int tx, ty, tz, ntiles;
};

inline Tiles3 tiles3(int n, int shape = 0) {
  const int X = shape == 0 ? Shape3<0>::X : (shape == 1 ? Shape3<1>::X : Shape3<2>::X);
  const int Y = shape == 0 ? Shape3<0>::Y : (shape == 1 ? Shape3<1>::Y : Shape3<2>::Y);
  const int Z = shape == 0 ? Shape3<0>::Z : (shape == 1 ? Shape3<1>::Z : Shape3<2>::Z);
  Tiles3 t;
  t.tx = (n + X - 1) / X;
  t.ty = (n + Y - 1) / Y;
  t.tz = (n + Z - 1) / Z;
  t.ntiles = t.tx * t.ty * t.tz;
  return t;
}

inline int grid3(const Tiles3& t) { return 8 * ((t.ntiles + 7) / 8); }

template <typename T, int SHAPE>
struct Lds3 {
  static constexpr int XX = Shape3<SHAPE>::X + 4, XY = Shape3<SHAPE>::Y + 4,
                       XZ = Shape3<SHAPE>::Z + 4;   // x_in tile, 2-cell ring
  static constexpr int BX = Shape3<SHAPE>::X + 2, BY = Shape3<SHAPE>::Y + 2,
                       BZ = Shape3<SHAPE>::Z + 2;   // b / c1 tile, 1-cell ring
  static constexpr int NX = XX * XY * XZ, NB = BX * BY * BZ;
  T x[NX];
  T c1[NB];
  T b[NB];
  uint8_t code[NB];
};

template <typename T, int MODE, bool FINE, int SHAPE>
__global__ void __launch_bounds__(Shape3<SHAPE>::Threads)
    k_rb_sweep3d(Faces<T> F, int n, Tiles3 tl, const T* __restrict__ rhs,
                 const T* __restrict__ xin, const T* __restrict__ ec, T* __restrict__ xout,
                 int c1, Ctl ctl, int dot, Sel sel) {
  using Sh = Shape3<SHAPE>;
  using Ld = Lds3<T, SHAPE>;
  constexpr int k3X = Sh::X, k3Y = Sh::Y, k3Z = Sh::Z, k3Threads = Sh::Threads;
  constexpr int k3XX = Ld::XX, k3XY = Ld::XY;
  constexpr int k3BX = Ld::BX, k3BY = Ld::BY, k3BZ = Ld::BZ;
  constexpr int k3NX = Ld::NX, k3NB = Ld::NB;
  const int b = sel_problem(sel, blockIdx.y);
  if (b < 0) return;
  const int tile = xcd_tile(blockIdx.x, tl.ntiles);
  if (tile < 0) {
    if (dot && threadIdx.x == 0) ctl.partials[(size_t)b * ctl.pstride + blockIdx.x] = 0.0;
    return;
  }
  __shared__ Ld S;
  const int tid = threadIdx.x;
  const int i0 = (tile % tl.tx) * k3X;
  const int j0 = ((tile / tl.tx) % tl.ty) * k3Y;
  const int k0 = (tile / (tl.tx * tl.ty)) * k3Z;
  const size_t nn = (size_t)n * n;
  const size_t base = (size_t)b * nn * n;
  const int nc = n >> 1;
  const size_t basec = (size_t)b * (size_t)nc * nc * nc;
  const T h2 = (T)(1.0 / ((double)n * (double)n));
  const T ir0 = FINE ? F.inv_rho[2 * b] : T(0), ir1 = FINE ? F.inv_rho[2 * b + 1] : T(0);
  const T hr0 = FINE ? h2 / ir0 : T(0), hr1 = FINE ? h2 / ir1 : T(0);
  // diagonal shift times h^2; with a shift every cell takes the general update
  const T sh2 = F.sig * h2;
  const bool plain = sh2 == T(0);
  // shifted operator, cell without a crossed face: x = (sum - hr b) / (faces + sig hr)
  const T shr0 = FINE ? F.sig * hr0 : T(0), shr1 = FINE ? F.sig * hr1 : T(0);

  // ---- every load of the block at once ----
  constexpr int PX = (k3NX + k3Threads - 1) / k3Threads;
  constexpr int PB = (k3NB + k3Threads - 1) / k3Threads;
  if (MODE != 1) {
    T rx[PX];
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + u * k3Threads;
      const int i = i0 - 2 + e % k3XX, j = j0 - 2 + (e / k3XX) % k3XY, k = k0 - 2 + e / (k3XX * k3XY);
      T v = T(0);
      if (e < k3NX && i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n) {
        v = xin[base + (size_t)k * nn + (size_t)j * n + i];
        if (MODE == 2) v += ec[basec + ((size_t)(k >> 1) * nc + (j >> 1)) * nc + (i >> 1)];
      }
      rx[u] = v;
    }
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int e = tid + u * k3Threads;
      if (e < k3NX) S.x[e] = rx[u];
    }
  }
  {
    T rb[PB];
    uint8_t rc[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int e = tid + u * k3Threads;
      const int i = i0 - 1 + e % k3BX, j = j0 - 1 + (e / k3BX) % k3BY, k = k0 - 1 + e / (k3BX * k3BY);
      T v = T(0);
      uint8_t cd = 0;
      if (e < k3NB && i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n) {
        const size_t c = base + (size_t)k * nn + (size_t)j * n + i;
        v = rhs[c];
        if (FINE) cd = F.code[c];
      }
      rb[u] = v;
      rc[u] = cd;
    }
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int e = tid + u * k3Threads;
      if (e < k3NB) {
        S.b[e] = rb[u];
        if (FINE) S.code[e] = rc[u];
      }
    }
  }
  lds_barrier();

  // Gauss-Seidel update of one cell from its six neighbour values (walls masked);
  // nb = false when every neighbour value is zero (first colour of a sweep from zero)
  auto update = [&](bool nb, unsigned cd, size_t cell, int i, int j, int k, T xw, T xe, T xs,
                    T xn, T xd, T xu, T bb) -> T {
    const bool wl = i > 0, wr = i < n - 1, ws = j > 0, wn = j < n - 1, wd = k > 0, wu = k < n - 1;
    if (FINE && (cd & 63u) == 0u) {
      T sum = T(0);
      if (nb) {
        sum = (wl ? xw : T(0)) + (wr ? xe : T(0));
        sum += (ws ? xs : T(0)) + (wn ? xn : T(0));
        sum += (wd ? xd : T(0)) + (wu ? xu : T(0));
      }
      const int cnt = (int)wl + (int)wr + (int)ws + (int)wn + (int)wd + (int)wu;
      const T hr = (cd & 64u) ? hr1 : hr0;
      if (!plain) return (sum - hr * bb) / (T(cnt) + ((cd & 64u) ? shr1 : shr0));
      const T inv = cnt == 6 ? T(1) / T(6) : (cnt == 5 ? T(1) / T(5) : (cnt == 4 ? T(0.25) : T(1) / T(3)));
      return (sum - hr * bb) * inv;
    }
    T w[6];
    sweep_faces<T, FINE>(F, cell, cd, i, j, k, n, nn, ir0, ir1, w);
    T num = T(0);
    if (nb) {
      if (wl) num += w[0] * xw;
      if (wr) num += w[1] * xe;
      if (ws) num += w[2] * xs;
      if (wn) num += w[3] * xn;
      if (wd) num += w[4] * xd;
      if (wu) num += w[5] * xu;
    }
    const T den = w[0] + w[1] + w[2] + w[3] + w[4] + w[5] + sh2;
    return (num - h2 * bb) / den;
  };

  // ---- c1 values on the tile and its one-cell ring (17 per ring row) ----
  constexpr int kRowC1 = k3BX / 2;
  constexpr int kNC1 = kRowC1 * k3BY * k3BZ;
  for (int q = tid; q < kNC1; q += k3Threads) {
    const int row = q / kRowC1;
    const int ey = row % k3BY, ez = row / k3BY;
    const int j = j0 - 1 + ey, k = k0 - 1 + ez;
    const int par = ((c1 - (i0 - 1) - j - k) % 2 + 2) % 2;
    const int ex = 2 * (q % kRowC1) + par;
    const int i = i0 - 1 + ex;
    if (i < 0 || i >= n || j < 0 || j >= n || k < 0 || k >= n) continue;
    const int lb = (ez * k3BY + ey) * k3BX + ex;
    const int lx = ((ez + 1) * k3XY + ey + 1) * k3XX + ex + 1;
    T xw = T(0), xe = T(0), xs = T(0), xn = T(0), xd = T(0), xu = T(0);
    if (MODE != 1) {
      xw = S.x[lx - 1];
      xe = S.x[lx + 1];
      xs = S.x[lx - k3XX];
      xn = S.x[lx + k3XX];
      xd = S.x[lx - k3XX * k3XY];
      xu = S.x[lx + k3XX * k3XY];
    }
    const unsigned cd = FINE ? S.code[lb] : 0u;
    S.c1[lb] = update(MODE != 1, cd, base + (size_t)k * nn + (size_t)j * n + i, i, j, k, xw, xe,
                      xs, xn, xd, xu, S.b[lb]);
  }
  lds_barrier();

  // ---- c2 values (and the c1 copies) on the tile ----
  double acc = 0.0;
  constexpr int kCells = k3X * k3Y * k3Z;
  for (int t = tid; t < kCells; t += k3Threads) {
    const int tx = t % k3X, ty = (t / k3X) % k3Y, tz = t / (k3X * k3Y);
    const int i = i0 + tx, j = j0 + ty, k = k0 + tz;
    if (i >= n || j >= n || k >= n) continue;
    const int q = ((tz + 1) * k3BY + ty + 1) * k3BX + tx + 1;
    const size_t cell = base + (size_t)k * nn + (size_t)j * n + i;
    const T bb = S.b[q];
    T out;
    if (((i + j + k) & 1) == c1) {
      out = S.c1[q];
    } else {
      // c1 entries outside the domain were never written: the wall masks skip them
      const unsigned cd = FINE ? S.code[q] : 0u;
      out = update(true, cd, cell, i, j, k, S.c1[q - 1], S.c1[q + 1], S.c1[q - k3BX],
                   S.c1[q + k3BX], S.c1[q - k3BX * k3BY], S.c1[q + k3BX * k3BY], bb);
    }
    xout[cell] = out;
    if (dot) acc += (double)bb * (double)out;
  }
  if (dot) block_partial(acc, ctl, b);
}

}  // namespace mpp
