// Streaming stencil kernels on the finest level: y = A x (with x.y), r = b - A x
// (with ||r||^2), and the coarse right-hand side mean_children(b - A x).
//
// A block owns a 64 x 4 column of cells (one thread per column, x fastest) and
// marches up a chunk of planes, holding x of planes k-1, k, k+1 of its own column in
// registers; in-plane neighbours come through the caches.  Everything a plane needs
// is loaded one plane ahead.  Offsets within a plane are 32-bit and computed once.
#pragma once

#include "rbgs.h"

namespace mpp {

constexpr int kStTX = 64;
constexpr int kStTY = 4;
constexpr int kStKZ = 16;
constexpr int kStThreads = kStTX * kStTY;

struct StTiles {
  int ntx, nty, nkz, ntiles;
};

inline StTiles st_tiles(int n, int kz) {
  StTiles t;
  t.ntx = (n + kStTX - 1) / kStTX;
  t.nty = (n + kStTY - 1) / kStTY;
  t.nkz = (n + kz - 1) / kz;
  t.ntiles = t.ntx * t.nty * t.nkz;
  return t;
}

inline int st_grid(const StTiles& t) { return 8 * ((t.ntiles + 7) / 8); }

// In-plane neighbours and the code byte of one cell (zeros outside the domain).
template <typename T>
struct Nb {
  T w, e, s, nn;
  unsigned cd;
};

template <typename T, bool FINE>
__device__ inline void load_nb(const T* xp, const uint8_t* cp, int off, int i, int j, int n,
                               Nb<T>& v) {
  v.w = i > 0 ? xp[off - 1] : T(0);
  v.e = i < n - 1 ? xp[off + 1] : T(0);
  v.s = j > 0 ? xp[off - n] : T(0);
  v.nn = j < n - 1 ? xp[off + n] : T(0);
  v.cd = FINE ? cp[off] : 0u;
}

// ((A - sig I) x)_c from the centre value, its six neighbours and the face coefficients
template <typename T>
__device__ inline T stencil7(const T w[6], T xc, T xw, T xe, T xs, T xn, T xd, T xu, int i, int j,
                             int k, int n, T inv_h2, T sig) {
  T s = T(0);
  if (i > 0) s += w[0] * (xw - xc);
  if (i < n - 1) s += w[1] * (xe - xc);
  if (j > 0) s += w[2] * (xs - xc);
  if (j < n - 1) s += w[3] * (xn - xc);
  if (k > 0) s += w[4] * (xd - xc);
  if (k < n - 1) s += w[5] * (xu - xc);
  return s * inv_h2 - sig * xc;
}

// Loads of one batch of kStZ planes of a thread's column, all issued before any use:
// x at planes k0-1 .. k0+kStZ, the four in-plane neighbours and the code byte of the
// kStZ planes.  Values outside the domain are 0.
constexpr int kStZ = 4;

template <typename T, bool FINE>
struct ColBatch {
  T xc[kStZ + 2];
  T w[kStZ], e[kStZ], s[kStZ], nb[kStZ];
  uint8_t cd[kStZ];
};

template <typename T, bool FINE>
__device__ inline void load_batch(const T* xb, const uint8_t* cb, int off, int i, int j, int k0,
                                  int n, size_t nn, bool xzero, ColBatch<T, FINE>& B) {
#pragma unroll
  for (int h = 0; h < kStZ + 2; ++h) {
    const int k = k0 - 1 + h;
    B.xc[h] = (!xzero && k >= 0 && k < n) ? xb[(size_t)k * nn + off] : T(0);
  }
#pragma unroll
  for (int h = 0; h < kStZ; ++h) {
    const int k = k0 + h;
    const bool pl = k < n;
    const T* xp = xb + (size_t)(pl ? k : 0) * nn + off;
    B.w[h] = (!xzero && pl && i > 0) ? xp[-1] : T(0);
    B.e[h] = (!xzero && pl && i < n - 1) ? xp[1] : T(0);
    B.s[h] = (!xzero && pl && j > 0) ? xp[-n] : T(0);
    B.nb[h] = (!xzero && pl && j < n - 1) ? xp[n] : T(0);
    B.cd[h] = (FINE && pl) ? cb[(size_t)k * nn + off] : 0;
  }
}

// KIND 0: y = A x (+ x.y partials when dot);  KIND 1: y = b - A x (+ ||y||^2 partials),
// with x taken as 0 when xzero.  y = nullptr: the partials only.  Threads own columns of a 64 x 4 tile and handle its
// z-chunk in batches of kStZ planes.
template <typename T, int KIND>
__global__ void __launch_bounds__(kStThreads)
    k_stencil_z(Faces<T> F, int n, StTiles tl, int kz, const T* __restrict__ x,
                const T* __restrict__ bvec, T* __restrict__ y, Ctl ctl, int dot, int xzero,
                Sel sel) {
  const int b = sel_problem(sel, blockIdx.y);
  if (b < 0) return;
  const int tile = xcd_tile(blockIdx.x, tl.ntiles);
  if (tile < 0) {
    if (dot && threadIdx.x == 0) ctl.partials[(size_t)b * ctl.pstride + blockIdx.x] = 0.0;
    return;
  }
  const int ti = tile % tl.ntx, tj = (tile / tl.ntx) % tl.nty, tk = tile / (tl.ntx * tl.nty);
  const int i = ti * kStTX + threadIdx.x % kStTX, j = tj * kStTY + threadIdx.x / kStTX;
  const int k0 = tk * kz, k1 = min(k0 + kz, n);
  const size_t nn = (size_t)n * n;
  const size_t base = (size_t)b * nn * n;
  const T inv_h2 = (T)((double)n * (double)n);
  double acc = 0.0;
  if (i < n && j < n) {
    const int off = i + n * j;
    const T ir0 = F.inv_rho[2 * b], ir1 = F.inv_rho[2 * b + 1];
    const bool xz = (KIND == 1 && xzero);
    for (int kb = k0; kb < k1; kb += kStZ) {
      ColBatch<T, true> B;
      load_batch<T, true>(x + base, F.code + base, off, i, j, kb, n, nn, xz, B);
      T bv[kStZ];
      if (KIND == 1) {
#pragma unroll
        for (int h = 0; h < kStZ; ++h)
          bv[h] = (kb + h < k1) ? bvec[base + (size_t)(kb + h) * nn + off] : T(0);
      }
#pragma unroll
      for (int h = 0; h < kStZ; ++h) {
        const int k = kb + h;
        if (k >= k1) break;
        const size_t cell = base + (size_t)k * nn + off;
        T w[6];
        coded_faces_at(F.bx + cell, F.by + cell, F.bz + cell, B.cd[h], i, j, k, n, nn,
                       (B.cd[h] & 64u) ? ir1 : ir0, w);
        const T ax = stencil7(w, B.xc[h + 1], B.w[h], B.e[h], B.s[h], B.nb[h], B.xc[h],
                              B.xc[h + 2], i, j, k, n, inv_h2, F.sig);
        T out;
        if (KIND == 0) {
          out = ax;
          if (dot) acc += (double)B.xc[h + 1] * (double)out;
        } else {
          out = bv[h] - ax;
          if (dot) acc += (double)out * (double)out;
        }
        if (y) y[cell] = out;
      }
    }
  }
  if (dot) block_partial(acc, ctl, b);
}

// Coarse rhs: b_c(I,J,K) = mean over the 8 children of (b - A x).  Threads own fine
// columns; a batch of kStZ fine planes gives kStZ/2 coarse planes, and the 2x2
// in-plane sum goes through a shuffle (x pairs are neighbouring lanes) and LDS (y
// pairs are rows).
template <typename T, bool FINE>
__global__ void __launch_bounds__(kStThreads)
    k_resid_restrict_z(Faces<T> F, int n, StTiles tl, int kz, const T* __restrict__ bvec,
                       const T* __restrict__ x, T* __restrict__ bc, Sel sel) {
  const int b = sel_problem(sel, blockIdx.y);
  if (b < 0) return;
  const int tile = xcd_tile(blockIdx.x, tl.ntiles);
  if (tile < 0) return;
  __shared__ T part[kStZ / 2][kStTY][kStTX / 2];
  const int lx = threadIdx.x % kStTX, ly = threadIdx.x / kStTX;
  const int ti = tile % tl.ntx, tj = (tile / tl.ntx) % tl.nty, tk = tile / (tl.ntx * tl.nty);
  const int i = ti * kStTX + lx, j = tj * kStTY + ly;
  const int k0 = tk * kz, k1 = min(k0 + kz, n);   // kz and n even: k0, k1 even
  const size_t nn = (size_t)n * n;
  const size_t base = (size_t)b * nn * n;
  const int nc = n >> 1;
  const size_t ncc = (size_t)nc * nc;
  const size_t basec = (size_t)b * ncc * nc;
  const T inv_h2 = (T)((double)n * (double)n);
  const bool in = i < n && j < n;
  const int off = in ? i + n * j : 0;
  const T ir0 = FINE ? F.inv_rho[2 * b] : T(0), ir1 = FINE ? F.inv_rho[2 * b + 1] : T(0);
  for (int kb = k0; kb < k1; kb += kStZ) {
    T s2[kStZ / 2] = {};
    if (in) {
      ColBatch<T, FINE> B;
      load_batch<T, FINE>(x + base, FINE ? F.code + base : nullptr, off, i, j, kb, n, nn, false, B);
      T bv[kStZ];
#pragma unroll
      for (int h = 0; h < kStZ; ++h)
        bv[h] = (kb + h < k1) ? bvec[base + (size_t)(kb + h) * nn + off] : T(0);
#pragma unroll
      for (int h = 0; h < kStZ; ++h) {
        const int k = kb + h;
        if (k >= k1) break;
        const size_t cell = base + (size_t)k * nn + off;
        T w[6];
        sweep_faces<T, FINE>(F, cell, B.cd[h], i, j, k, n, nn, ir0, ir1, w);
        s2[h >> 1] += bv[h] - stencil7(w, B.xc[h + 1], B.w[h], B.e[h], B.s[h], B.nb[h], B.xc[h],
                                       B.xc[h + 2], i, j, k, n, inv_h2, F.sig);
      }
    }
#pragma unroll
    for (int c = 0; c < kStZ / 2; ++c) {
      const T t = s2[c] + __shfl_xor(s2[c], 1, 64);
      if ((lx & 1) == 0) part[c][ly][lx >> 1] = t;
    }
    __syncthreads();
    if ((ly & 1) == 0 && (lx & 1) == 0 && in) {
#pragma unroll
      for (int c = 0; c < kStZ / 2; ++c) {
        const int K = (kb >> 1) + c;
        if (2 * K < k1) {
          const T t = part[c][ly][lx >> 1] + part[c][ly + 1][lx >> 1];
          bc[basec + (size_t)K * ncc + (i >> 1) + (size_t)nc * (j >> 1)] = t * T(0.125);
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace mpp
