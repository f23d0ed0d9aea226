// Block-structured layout: the grid as a set of blocks of cells (Sec. 2; the setup
// command of Sec. 4 uses 16^3 blocks), each with g guard layers that the guard-cell
// fill (Sec. 4) takes from the neighbouring blocks and, outside the domain, from the
// field mirrored about the wall (the zero-gradient condition of the no-flux walls).
//
// A problem of n^3 cells is cut into nbx^3 blocks (nbx = n / nb) of nb^3 cells; block
// (bi, bj, bk) has index bi + nbx (bj + nbx bk) and is stored as P^3 values (P = nb + 2g,
// x fastest, the interior at offsets g .. g + nb - 1); problems follow each other.  Every
// kernel runs one workgroup per (block, problem).
#pragma once

#include "kernels.h"

namespace mpp {

constexpr int kBlkThreads = 256;

struct BlkShape {
  int n, nb, g, nbx, P;
  size_t P3;     // values per block
  size_t nblk;   // blocks per problem
};

inline BlkShape blk_shape(int n, int nb, int g) {
  BlkShape s;
  s.n = n;
  s.nb = nb;
  s.g = g;
  s.nbx = n / nb;
  s.P = nb + 2 * g;
  s.P3 = (size_t)s.P * s.P * s.P;
  s.nblk = (size_t)s.nbx * s.nbx * s.nbx;
  return s;
}

// block coordinates of the workgroup's block
__device__ inline void blk_coords(const BlkShape& S, size_t blk, int& bi, int& bj, int& bk) {
  bi = (int)(blk % S.nbx);
  bj = (int)((blk / S.nbx) % S.nbx);
  bk = (int)(blk / ((size_t)S.nbx * S.nbx));
}

// The kernels take the block edge and guard width as template constants when they are
// the common ones (NB, G > 0: index arithmetic by constants), else from S (NB = G = 0).

// DIR 0: grid -> block interiors (scatter); DIR 1: block interiors -> grid (gather)
template <int DIR, int NB, int G>
__global__ void __launch_bounds__(kBlkThreads)
    k_blk_copy(BlkShape S, const double* __restrict__ src, double* __restrict__ dst) {
  const size_t blk = blockIdx.x;
  const int pb = blockIdx.y;
  int bi, bj, bk;
  blk_coords(S, blk, bi, bj, bk);
  const int nb = NB > 0 ? NB : S.nb, g = NB > 0 ? G : S.g, P = nb + 2 * g, n = S.n;
  const size_t gbase = (size_t)pb * n * n * n;
  const size_t bbase = ((size_t)pb * S.nblk + blk) * S.P3;
  const int cells = nb * nb * nb;
  for (int q = threadIdx.x; q < cells; q += kBlkThreads) {
    const int li = q % nb, lj = (q / nb) % nb, lk = q / (nb * nb);
    const size_t gc = gbase + (size_t)(bi * nb + li) +
                      (size_t)n * ((size_t)(bj * nb + lj) + (size_t)n * (size_t)(bk * nb + lk));
    const size_t bc = bbase + (size_t)(li + g) + (size_t)P * ((size_t)(lj + g) + (size_t)P * (lk + g));
    if (DIR == 0)
      dst[bc] = src[gc];
    else
      dst[gc] = src[bc];
  }
}

__device__ inline int blk_mirror(int a, int n) { return a < 0 ? -1 - a : (a >= n ? 2 * n - 1 - a : a); }

// Local coordinates (each in [-g, nb + g)) of guard cell q of a block: the g planes below
// the interior, the g planes above, then the ring of every interior plane (the g rows
// before, the g rows after, then g cells at each end of every interior row).
__device__ inline void blk_guard_cell(int q, int nb, int g, int P, int& li, int& lj, int& lk) {
  const int P2 = P * P, slab = g * P2;
  if (q < 2 * slab) {
    const int top = q >= slab;
    const int r = top ? q - slab : q;
    lk = top ? nb + r / P2 : r / P2 - g;
    lj = (r % P2) / P - g;
    li = r % P - g;
    return;
  }
  const int ring = 2 * g * P + 2 * g * nb;
  const int r = q - 2 * slab;
  lk = r / ring;
  int t = r % ring;
  if (t < 2 * g * P) {
    const int top = t >= g * P;
    if (top) t -= g * P;
    lj = top ? nb + t / P : t / P - g;
    li = t % P - g;
    return;
  }
  t -= 2 * g * P;
  lj = t / (2 * g);
  const int e = t % (2 * g);
  li = e < g ? e - g : nb + (e - g);
}

// Every guard cell from the interior of the block owning its (mirrored) position.
// Guards are only written and interiors only read, so blocks need no ordering.
template <int NB, int G>
__global__ void __launch_bounds__(kBlkThreads) k_blk_fill(BlkShape S, double* __restrict__ blocks) {
  const size_t blk = blockIdx.x;
  const int pb = blockIdx.y;
  int bi, bj, bk;
  blk_coords(S, blk, bi, bj, bk);
  const int nb = NB > 0 ? NB : S.nb, g = NB > 0 ? G : S.g, P = nb + 2 * g, n = S.n, nbx = S.nbx;
  const size_t pbase = (size_t)pb * S.nblk * S.P3;
  double* const own = blocks + pbase + blk * S.P3;
  const int guards = P * P * P - nb * nb * nb;
  for (int q = threadIdx.x; q < guards; q += kBlkThreads) {
    int li, lj, lk;
    blk_guard_cell(q, nb, g, P, li, lj, lk);
    const int I = blk_mirror(bi * nb + li, n), J = blk_mirror(bj * nb + lj, n),
              K = blk_mirror(bk * nb + lk, n);
    const size_t src_blk = (size_t)(I / nb) + (size_t)nbx * ((size_t)(J / nb) + (size_t)nbx * (K / nb));
    const double v = blocks[pbase + src_blk * S.P3 + (size_t)(I % nb + g) +
                            (size_t)P * ((size_t)(J % nb + g) + (size_t)P * (size_t)(K % nb + g))];
    own[(size_t)(li + g) + (size_t)P * ((size_t)(lj + g) + (size_t)P * (size_t)(lk + g))] = v;
  }
}

// y = A x block by block: the padded x block is staged in LDS (dynamic, P^3 doubles),
// each interior cell takes its six neighbours from there and its face coefficients from
// the grid-layout arrays (walls carry 0); the guards of y are set to 0.
template <int NB, int G>
__global__ void __launch_bounds__(kBlkThreads)
    k_blk_apply(BlkShape S, const double* __restrict__ bx, const double* __restrict__ by,
                const double* __restrict__ bz, const double* __restrict__ x,
                double* __restrict__ y) {
#pragma clang fp contract(off)
  extern __shared__ double xs[];
  const size_t blk = blockIdx.x;
  const int pb = blockIdx.y;
  int bi, bj, bk;
  blk_coords(S, blk, bi, bj, bk);
  const int nb = NB > 0 ? NB : S.nb, g = NB > 0 ? G : S.g, P = nb + 2 * g, n = S.n;
  const size_t bbase = ((size_t)pb * S.nblk + blk) * S.P3;
  const size_t gbase = (size_t)pb * n * n * n;
  const size_t nn = (size_t)n * n;
  const int P3 = P * P * P;
  for (int q = threadIdx.x; q < P3; q += kBlkThreads) xs[q] = x[bbase + q];
  __syncthreads();
  for (int q = threadIdx.x; q < P3; q += kBlkThreads) {
    const int li = q % P - g, lj = (q / P) % P - g, lk = q / (P * P) - g;
    double out = 0.0;
    if (li >= 0 && li < nb && lj >= 0 && lj < nb && lk >= 0 && lk < nb) {
      const int i = bi * nb + li, j = bj * nb + lj, k = bk * nb + lk;
      const size_t c = gbase + (size_t)i + (size_t)n * ((size_t)j + (size_t)n * k);
      const double w[6] = {bx[c], i < n - 1 ? bx[c + 1] : 0.0, by[c], j < n - 1 ? by[c + n] : 0.0,
                           bz[c], k < n - 1 ? bz[c + nn] : 0.0};
      const double xc = xs[q];
      const double xn[6] = {xs[q - 1], xs[q + 1], xs[q - P], xs[q + P], xs[q - P * P], xs[q + P * P]};
      double s = 0.0;
#pragma unroll
      for (int f = 0; f < 6; ++f) s += w[f] * (xn[f] - xc);
      out = s * ((double)n * (double)n);
    }
    y[bbase + q] = out;
  }
}

// Launches KERNEL<..., NB, G> with the constants of the common shapes, else the generic
// instantiation.
#define MPP_BLK_DISPATCH(S, LAUNCH)                  \
  do {                                               \
    if ((S).nb == 16 && (S).g == 1) LAUNCH(16, 1);   \
    else if ((S).nb == 16 && (S).g == 2) LAUNCH(16, 2); \
    else if ((S).nb == 8 && (S).g == 1) LAUNCH(8, 1); \
    else LAUNCH(0, 0);                               \
  } while (0)

}  // namespace mpp
