// Fused red-black Gauss-Seidel sweep on the finest level, one pass over memory.
//
// Semantics (identical to two one-colour half sweeps): with c1 the first colour,
//   x1  = x_in with every c1 cell set to (sum_f w_f x_in[nb] - h^2 b) / sum_f w_f,
//   out = x1  with every c2 cell set to (sum_f w_f x1[nb]  - h^2 b) / sum_f w_f.
// Out of place (x_in and out are different arrays), so blocks never see each other's
// results: every block recomputes the c1 values on a one-cell ring around its tile
// from x_in loaded with a two-cell ring.
//
// Layout of the work: a block owns a TX x TY column of cells (x fastest, one thread
// per cell) and marches up a chunk of KZ planes.  At lead plane L it loads x_in of
// plane L+1 (tile + 2-cell ring) and b / code of plane L (tile + 1-cell ring) into
// LDS, computes the c1 values of plane L on tile + ring, then the c2 values of plane
// L-1 on the tile, which need c1 values of planes L-2, L-1 and L.  Three-plane ring
// buffers in LDS; two barriers per plane.
//
// Variants: MODE 0 reads x_in, MODE 1 takes x_in = 0 (first sweep of a V-cycle),
// MODE 2 reads x_in = x_prev + (coarse correction of the parent cell).  With `dot`
// set the block also stores its partial sum of b * out (r.z in the CG).
#pragma once

#include "kernels.h"

namespace mpp {

constexpr int kRbTX = 64;
constexpr int kRbTY = 8;
constexpr int kRbKZ = 16;
constexpr int kRbThreads = kRbTX * kRbTY;

struct RbTiles {
  int ntx, nty, nkz;   // tiles along x, y and z-chunks along z
  int ntiles;          // ntx * nty * nkz
  int kz;              // planes per z-chunk
};

// Tiles for z-chunks of kz planes.  kz = 0 picks the default: chunks of kRbKZ planes,
// shortened (down to 4) while the grid would not give every compute unit a few blocks.
inline RbTiles rb_tiles(int n, int batch = 1, int kz = 0) {
  RbTiles t;
  t.ntx = (n + kRbTX - 1) / kRbTX;
  t.nty = (n + kRbTY - 1) / kRbTY;
  if (kz > 0) {
    t.kz = kz;
  } else {
    t.kz = kRbKZ;
    while (t.kz > 4 && (long)t.ntx * t.nty * ((n + t.kz - 1) / t.kz) * batch < 1536) t.kz /= 2;
  }
  t.nkz = (n + t.kz - 1) / t.kz;
  t.ntiles = t.ntx * t.nty * t.nkz;
  return t;
}


inline int rb_grid(const RbTiles& t) { return 8 * ((t.ntiles + 7) / 8); }

constexpr int kRbXW = kRbTX + 4;                 // row length of the x_in tile (2-cell ring)
constexpr int kRbBW = kRbTX + 2;                 // row length of the b / c1 tiles (1-cell ring)
constexpr int kRbNX = (kRbTY + 4) * kRbXW;
constexpr int kRbNB = (kRbTY + 2) * kRbBW;

template <typename T>
struct RbLds {
  T x[3][kRbNX];
  T c1[3][kRbNB];
  T b[3][kRbNB];
  uint8_t code[3][kRbNB];
};

// Face coefficients of a cell from its code byte (finest level); p points at the
// cell in each face array, plane-offset already applied.
template <typename T>
__device__ inline void coded_faces_at(const T* px, const T* py, const T* pz, unsigned cd, int i,
                                      int j, int k, int n, size_t nn, T ir, T w[6]) {
  w[0] = i > 0 ? ((cd & 1u) ? px[0] : ir) : T(0);
  w[1] = i < n - 1 ? ((cd & 2u) ? px[1] : ir) : T(0);
  w[2] = j > 0 ? ((cd & 4u) ? py[0] : ir) : T(0);
  w[3] = j < n - 1 ? ((cd & 8u) ? py[n] : ir) : T(0);
  w[4] = k > 0 ? ((cd & 16u) ? pz[0] : ir) : T(0);
  w[5] = k < n - 1 ? ((cd & 32u) ? pz[nn] : ir) : T(0);
}

// Face coefficients of a cell on a coarse level: every face from the arrays.
template <typename T>
__device__ inline void full_faces_at(const T* px, const T* py, const T* pz, int i, int j, int k,
                                     int n, size_t nn, T w[6]) {
  w[0] = i > 0 ? px[0] : T(0);
  w[1] = i < n - 1 ? px[1] : T(0);
  w[2] = j > 0 ? py[0] : T(0);
  w[3] = j < n - 1 ? py[n] : T(0);
  w[4] = k > 0 ? pz[0] : T(0);
  w[5] = k < n - 1 ? pz[nn] : T(0);
}

template <typename T, bool FINE>
__device__ inline void sweep_faces(const Faces<T>& F, size_t cell, unsigned cd, int i, int j, int k,
                                   int n, size_t nn, T ir0, T ir1, T w[6]) {
  if (FINE)
    coded_faces_at(F.bx + cell, F.by + cell, F.bz + cell, cd, i, j, k, n, nn,
                   (cd & 64u) ? ir1 : ir0, w);
  else
    full_faces_at(F.bx + cell, F.by + cell, F.bz + cell, i, j, k, n, nn, w);
}

// p[byte offset] with a 32-bit offset from a wave-uniform base (lets the compiler use
// the scalar-base addressing form)
template <typename T>
__device__ inline T ld_off(const T* p, unsigned byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + byte_off);
}

template <typename T, int MODE, bool FINE>
__global__ void __launch_bounds__(kRbThreads)
    k_rb_sweep(Faces<T> F, int n, RbTiles tl, const T* __restrict__ rhs,
               const T* __restrict__ xin, const T* __restrict__ ec, T* __restrict__ xout, int c1,
               Ctl ctl, int dot, Sel sel) {
  const int b = sel_problem(sel, blockIdx.y);
  if (b < 0) return;
  const int tile = xcd_tile(blockIdx.x, tl.ntiles);
  if (tile < 0) {
    if (dot && threadIdx.x == 0) ctl.partials[(size_t)b * ctl.pstride + blockIdx.x] = 0.0;
    return;
  }
  __shared__ RbLds<T> S;
  const int tid = threadIdx.x;
  const int ti = tile % tl.ntx;
  const int tj = (tile / tl.ntx) % tl.nty;
  const int tk = tile / (tl.ntx * tl.nty);
  const int i0 = ti * kRbTX, j0 = tj * kRbTY, k0 = tk * tl.kz;
  const int k1 = min(k0 + tl.kz, n);
  const size_t nn = (size_t)n * n;
  const size_t base = (size_t)b * nn * n;
  const int nc = n >> 1;
  const size_t ncc = (size_t)nc * nc;
  const size_t basec = (size_t)b * ncc * nc;
  const T h2 = (T)(1.0 / ((double)n * (double)n));
  // finest level, cells without a crossed face: every interior face carries 1/rho of
  // the cell's side, so x = (sum of interior neighbours - h^2 rho b) / (their count)
  const T ir0 = FINE ? F.inv_rho[2 * b] : T(0), ir1 = FINE ? F.inv_rho[2 * b + 1] : T(0);
  const T hr0 = FINE ? h2 / ir0 : T(0), hr1 = FINE ? h2 / ir1 : T(0);
  // diagonal shift times h^2; with a shift every cell takes the general update
  const T sh2 = F.sig * h2;
  const bool plain = sh2 == T(0);
  // shifted operator, cell without a crossed face: x = (sum - hr b) / (faces + sig hr)
  const T shr0 = FINE ? F.sig * hr0 : T(0), shr1 = FINE ? F.sig * hr1 : T(0);
  double acc = 0.0;

  // ---- plane-invariant per-thread offsets (0 where the cell does not exist) ----
  constexpr int PX = (kRbNX + kRbThreads - 1) / kRbThreads;
  constexpr int PB = (kRbNB + kRbThreads - 1) / kRbThreads;
  unsigned xo[PX], co[PX], bo[PB];
  bool xv[PX], bv[PB];
#pragma unroll
  for (int u = 0; u < PX; ++u) {
    const int e = tid + u * kRbThreads;
    const int i = i0 - 2 + e % kRbXW, j = j0 - 2 + e / kRbXW;
    xv[u] = e < kRbNX && i >= 0 && i < n && j >= 0 && j < n;
    xo[u] = xv[u] ? (unsigned)(i + n * j) * (unsigned)sizeof(T) : 0u;
    co[u] = xv[u] ? (unsigned)((i >> 1) + nc * (j >> 1)) * (unsigned)sizeof(T) : 0u;
  }
#pragma unroll
  for (int u = 0; u < PB; ++u) {
    const int e = tid + u * kRbThreads;
    const int i = i0 - 1 + e % kRbBW, j = j0 - 1 + e / kRbBW;
    bv[u] = e < kRbNB && i >= 0 && i < n && j >= 0 && j < n;
    bo[u] = bv[u] ? (unsigned)(i + n * j) : 0u;   // element offset (b: * sizeof(T))
  }
  // c1 item: one cell of colour c1 on the tile + 1-cell ring; its column alternates
  // with the plane parity
  constexpr int kHalf = kRbBW / 2;
  const bool c1_item = tid < kHalf * (kRbTY + 2);
  const int c1_r = tid / kHalf, c1_j = j0 - 1 + c1_r;
  int c1_lds[2], c1_i[2];
  unsigned c1_off[2];
  bool c1_in[2];
  T c1_inv1[2], c1_inv2[2];   // 1 / (interior faces) with one or no z wall
  {
    const int A = ((c1 - c1_j - (i0 - 1)) % 2 + 2) % 2;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int q = 2 * (tid % kHalf) + ((A + par) & 1);
      const int i = i0 - 1 + q;
      c1_i[par] = i;
      c1_lds[par] = c1_r * kRbBW + q;
      c1_in[par] = c1_item && i >= 0 && i < n && c1_j >= 0 && c1_j < n;
      c1_off[par] = c1_in[par] ? (unsigned)(i + n * c1_j) : 0u;
      const int cin = (i > 0) + (i < n - 1) + (c1_j > 0) + (c1_j < n - 1);
      c1_inv1[par] = T(1) / T(cin + 1);
      c1_inv2[par] = T(1) / T(cin + 2);
    }
  }
  // c2 / output item: the thread's own cell of the tile
  const int o_i = i0 + tid % kRbTX, o_j = j0 + tid / kRbTX;
  const bool o_ok = o_i < n && o_j < n;
  const unsigned o_off = o_ok ? (unsigned)(o_i + n * o_j) : 0u;
  const int o_lds = (tid / kRbTX + 1) * kRbBW + tid % kRbTX + 1;
  T o_inv1, o_inv2;
  {
    const int cin = (o_i > 0) + (o_i < n - 1) + (o_j > 0) + (o_j < n - 1);
    o_inv1 = T(1) / T(cin + 1);
    o_inv2 = T(1) / T(cin + 2);
  }

  // ---- loads for lead plane L (x_in of plane L+1, b / code of plane L), issued one
  //      plane ahead through registers
  T rx[PX], rb[PB];
  uint8_t rc[PB];
  auto fetch = [&](int L) {
    if (MODE != 1) {
      const int kk = L + 1;
      const bool pl = kk >= 0 && kk < n;
      const int kc = min(max(kk, 0), n - 1);
      const T* xp = xin + base + (size_t)kc * nn;
      const T* ep = ec + basec + (size_t)(kc >> 1) * ncc;
#pragma unroll
      for (int u = 0; u < PX; ++u) {
        // loads only where the cell exists: idle lanes skip them (cheaper than
        // loading a clamped address and masking)
        T v = T(0);
        if (pl && xv[u]) {
          v = ld_off(xp, xo[u]);
          if (MODE == 2) v += ld_off(ep, co[u]);
        }
        rx[u] = v;
      }
    }
    const bool pl = L >= 0 && L < n;
    const int Lc = min(max(L, 0), n - 1);
    const T* bp = rhs + base + (size_t)Lc * nn;
    const uint8_t* cp = FINE ? F.code + base + (size_t)Lc * nn : nullptr;
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      T v = T(0);
      uint8_t cd = 0;
      if (pl && bv[u]) {
        v = ld_off(bp, bo[u] * (unsigned)sizeof(T));
        if (FINE) cd = cp[bo[u]];
      }
      rb[u] = v;
      rc[u] = cd;
    }
  };
  auto commit = [&](int L) {
    if (MODE != 1) {
      T* dst = S.x[(L + 7) % 3];
#pragma unroll
      for (int u = 0; u < PX; ++u) {
        const int e = tid + u * kRbThreads;
        if (e < kRbNX) dst[e] = rx[u];
      }
    }
    const int sl = (L + 6) % 3;
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int e = tid + u * kRbThreads;
      if (e < kRbNB) {
        S.b[sl][e] = rb[u];
        if (FINE) S.code[sl][e] = rc[u];
      }
    }
  };

  // Gauss-Seidel update of one cell from its six neighbour values (walls masked);
  // nb = false when every neighbour value is zero (first colour of a sweep from zero)
  auto update = [&](bool nb, unsigned cd, size_t cell, int i, int j, int k, bool wl, bool wr,
                    bool ws, bool wn, bool wd, bool wu, T xw, T xe, T xs, T xn, T xd, T xu, T bb,
                    T inv1, T inv2) -> T {
    if (FINE && (cd & 63u) == 0u) {
      T sum = T(0);
      if (nb) {
        sum = (wl ? xw : T(0)) + (wr ? xe : T(0));
        sum += (ws ? xs : T(0)) + (wn ? xn : T(0));
        sum += (wd ? xd : T(0)) + (wu ? xu : T(0));
      }
      const T hr = (cd & 64u) ? hr1 : hr0;
      if (plain) {
        const T inv = (wd && wu) ? inv2 : inv1;
        return (sum - hr * bb) * inv;
      }
      const T cnt = T((int)wl + (int)wr + (int)ws + (int)wn + (int)wd + (int)wu);
      return (sum - hr * bb) / (cnt + ((cd & 64u) ? shr1 : shr0));
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

  // one lead-plane step: c1 values of plane L, then c2 / output of plane L - 1
  auto step = [&](int L) {
    lds_barrier();
    if (L >= 0 && L < n) {
      const int par = L & 1;
      if (c1_in[par]) {
        const int sl = (L + 6) % 3, sm = (L + 5) % 3, sp = (L + 7) % 3;
        const int lb = c1_lds[par];
        const int lx = lb + (lb / kRbBW) * 2 + kRbXW + 1;   // same cell in the x tile
        const int i = c1_i[par];
        const unsigned cd = FINE ? S.code[sl][lb] : 0u;
        T xw = T(0), xe = T(0), xs = T(0), xn = T(0), xd = T(0), xu = T(0);
        if (MODE != 1) {
          xw = S.x[sl][lx - 1];
          xe = S.x[sl][lx + 1];
          xs = S.x[sl][lx - kRbXW];
          xn = S.x[sl][lx + kRbXW];
          xd = S.x[sm][lx];
          xu = S.x[sp][lx];
        }
        S.c1[sl][lb] = update(MODE != 1, cd, base + (size_t)L * nn + c1_off[par], i, c1_j, L, i > 0,
                              i < n - 1, c1_j > 0, c1_j < n - 1, L > 0, L < n - 1, xw, xe, xs,
                              xn, xd, xu, S.b[sl][lb], c1_inv1[par], c1_inv2[par]);
      }
    }
    lds_barrier();
    const int k = L - 1;
    if (k >= k0 && k < k1 && o_ok) {
      const int sl = (k + 6) % 3, sm = (k + 5) % 3, sp = (k + 7) % 3;
      const int q = o_lds;
      const T bb = S.b[sl][q];
      T out;
      if (((o_i + o_j + k) & 1) == c1) {
        out = S.c1[sl][q];
      } else {
        // c1 entries outside the domain were never written: the wall masks skip them
        const unsigned cd = FINE ? S.code[sl][q] : 0u;
        out = update(true, cd, base + (size_t)k * nn + o_off, o_i, o_j, k, o_i > 0, o_i < n - 1,
                     o_j > 0, o_j < n - 1, k > 0, k < n - 1, S.c1[sl][q - 1], S.c1[sl][q + 1],
                     S.c1[sl][q - kRbBW], S.c1[sl][q + kRbBW], S.c1[sm][q], S.c1[sp][q], bb,
                     o_inv1, o_inv2);
      }
      xout[base + (size_t)k * nn + o_off] = out;
      if (dot) acc += (double)bb * (double)out;
    }
  };

  // prologue: x_in of planes k0-2 and k0-1 into LDS
  if (MODE != 1) {
    fetch(k0 - 3);
    commit(k0 - 3);
    fetch(k0 - 2);
    commit(k0 - 2);
  }
  fetch(k0 - 1);
  for (int L = k0 - 1; L <= k1; ++L) {
    commit(L);
    if (L < k1) fetch(L + 1);
    step(L);
  }
  if (dot) block_partial(acc, ctl, b);
}

}  // namespace mpp
