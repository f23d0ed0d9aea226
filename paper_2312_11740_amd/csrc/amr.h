// Two-level composite grid (Sec. 2 and Fig. 2: blocks of cells at two resolutions, the
// finer one around the interface).  Level 0 has n0^3 cells in (n0/nb)^3 blocks of nb^3
// cells, every one stored; the refined ones are covered by level 1, whose cells have half
// the spacing.  Level 1 is stored sparsely: the 8 children of every refined level-0 block,
// each a block of nb^3 level-1 cells, in the order of their parents (child a + 2b + 4c for
// the offsets a, b, c in x, y, z).  Blocks of both levels are P^3 values with g guard
// layers (P = nb + 2g, x fastest), as in the uniform block layout.
//
// Tables (built on the host, read by every kernel): refined0[nblk0] marks the refined
// level-0 blocks; map1[(2 n0 / nb)^3] holds, for each level-1 block position, the index
// of its stored block or -1; list1[nblk1] is the position of each stored level-1 block.
//
// The leaf cells are those of the unrefined level-0 blocks and of the level-1 blocks.
// The operator is the conservative finite-volume Laplacian on the leaves: each face flux
// is area * beta * (x_other - x_self) / distance of the two centres, divided by the cell
// volume.  Across a coarse-fine face the fine cell sees the coarse cell itself (centres
// 1.5 fine spacings apart) and the coarse cell the four fine cells across its face, each
// through a quarter of its face; so every flux enters one cell and leaves the other.
// beta is the ghost-fluid coefficient of the two cells (lower coordinate first).
#pragma once

#include "blocks.h"

namespace mpp {

struct AmrShape {
  int n0, nb, g, P;
  int nbx0, nbx1;     // blocks per edge on level 0 and level 1 (nbx1 = 2 nbx0)
  int nblk0, nblk1;   // stored blocks per level
  size_t P3;
  // the operator's face factors, each 1 / (distance * spacing) of its kind of face
  double same0, same1, fine_side, coarse_side;
};

// position (bi, bj, bk) of stored block b of level `lev`
__device__ inline void amr_block_coords(const AmrShape& A, int lev, int b, const int* list1,
                                        int& bi, int& bj, int& bk) {
  const int nbx = lev ? A.nbx1 : A.nbx0;
  const int pos = lev ? list1[b] : b;
  bi = pos % nbx;
  bj = (pos / nbx) % nbx;
  bk = pos / (nbx * nbx);
}

__device__ inline size_t amr_local(int P, int g, int li, int lj, int lk) {
  return (size_t)(li + g) + (size_t)P * ((size_t)(lj + g) + (size_t)P * (size_t)(lk + g));
}

// value of level-1 cell (i, j, k) of a refined region (its block is stored)
template <int NB, int G>
__device__ inline double amr_fine(const AmrShape& A, const int* __restrict__ map1,
                                  const double* __restrict__ b1, int i, int j, int k) {
  const int nb = NB > 0 ? NB : A.nb, g = NB > 0 ? G : A.g, P = nb + 2 * g;
  const int blk = map1[i / nb + A.nbx1 * (j / nb + A.nbx1 * (k / nb))];
  return b1[(size_t)blk * A.P3 + amr_local(P, g, i % nb, j % nb, k % nb)];
}

// Guard cells of every stored block of both levels, in place (interiors only read).  A
// guard position is mirrored about the walls on its own level; inside, a level-0 guard
// takes the level-0 value where its block is not refined and the mean of the 8 level-1
// cells it covers where it is (pairwise: x pairs, then y, then z); a level-1 guard takes
// the level-1 value where that block is stored and the value of the level-0 cell
// containing it where it is not.  One workgroup per stored block (level 0 first).
template <int NB, int G>
__global__ void __launch_bounds__(kBlkThreads)
    k_amr_fill(AmrShape A, const uint8_t* __restrict__ refined0, const int* __restrict__ map1,
               const int* __restrict__ list1, double* __restrict__ b0, double* __restrict__ b1) {
  const int lev = (int)blockIdx.x >= A.nblk0;
  const int blk = lev ? (int)blockIdx.x - A.nblk0 : (int)blockIdx.x;
  int bi, bj, bk;
  amr_block_coords(A, lev, blk, list1, bi, bj, bk);
  const int nb = NB > 0 ? NB : A.nb, g = NB > 0 ? G : A.g, P = nb + 2 * g;
  const int n = lev ? 2 * A.n0 : A.n0;
  double* const own = (lev ? b1 : b0) + (size_t)blk * A.P3;
  const int guards = P * P * P - nb * nb * nb;
  for (int q = threadIdx.x; q < guards; q += kBlkThreads) {
    int li, lj, lk;
    blk_guard_cell(q, nb, g, P, li, lj, lk);
    const int I = blk_mirror(bi * nb + li, n), J = blk_mirror(bj * nb + lj, n),
              K = blk_mirror(bk * nb + lk, n);
    double v;
    if (lev == 0) {
      const int ob = I / nb + A.nbx0 * (J / nb + A.nbx0 * (K / nb));
      if (!refined0[ob]) {
        v = b0[(size_t)ob * A.P3 + amr_local(P, g, I % nb, J % nb, K % nb)];
      } else {
        double s[4];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            s[b + 2 * c] = amr_fine<NB, G>(A, map1, b1, 2 * I, 2 * J + b, 2 * K + c) +
                           amr_fine<NB, G>(A, map1, b1, 2 * I + 1, 2 * J + b, 2 * K + c);
        v = 0.125 * ((s[0] + s[1]) + (s[2] + s[3]));
      }
    } else {
      const int fb = map1[I / nb + A.nbx1 * (J / nb + A.nbx1 * (K / nb))];
      if (fb >= 0) {
        v = b1[(size_t)fb * A.P3 + amr_local(P, g, I % nb, J % nb, K % nb)];
      } else {
        const int Ic = I / 2, Jc = J / 2, Kc = K / 2;
        const int ob = Ic / nb + A.nbx0 * (Jc / nb + A.nbx0 * (Kc / nb));
        v = b0[(size_t)ob * A.P3 + amr_local(P, g, Ic % nb, Jc % nb, Kc % nb)];
      }
    }
    own[amr_local(P, g, li, lj, lk)] = v;
  }
}

// y = A x on the leaves, x and phi in blocks with filled guards (g >= 1).  A level-1 cell
// and an unrefined level-0 cell take every neighbour of their own level, and a fine
// cell its coarse neighbours, from the guards of their own block; a level-0 cell next to
// a refined block reads the four level-1 cells across the face from their blocks.  The
// terms are summed in the order x-, x+, y-, y+, z-, z+ (the four fine cells of a face in
// the order of the next two axes, cyclically).  Guards of y and every value of a refined
// level-0 block are set to 0.  One workgroup per stored block (level 0 first).
template <int NB, int G>
__global__ void __launch_bounds__(kBlkThreads)
    k_amr_apply(AmrShape A, const uint8_t* __restrict__ refined0, const int* __restrict__ map1,
                const int* __restrict__ list1, const double* __restrict__ phi0,
                const double* __restrict__ phi1, const double* __restrict__ x0,
                const double* __restrict__ x1, double rn, double rp, double* __restrict__ y0,
                double* __restrict__ y1) {
#pragma clang fp contract(off)
  const int lev = (int)blockIdx.x >= A.nblk0;
  const int blk = lev ? (int)blockIdx.x - A.nblk0 : (int)blockIdx.x;
  int bi, bj, bk;
  amr_block_coords(A, lev, blk, list1, bi, bj, bk);
  const int nb = NB > 0 ? NB : A.nb, g = NB > 0 ? G : A.g, P = nb + 2 * g;
  const int n = lev ? 2 * A.n0 : A.n0;
  const size_t base = (size_t)blk * A.P3;
  const double* const xb = (lev ? x1 : x0) + base;
  const double* const pb = (lev ? phi1 : phi0) + base;
  double* const yb = (lev ? y1 : y0) + base;
  const int P3 = P * P * P;
  if (lev == 0 && refined0[blk]) {
    for (int q = threadIdx.x; q < P3; q += kBlkThreads) yb[q] = 0.0;
    return;
  }
  const int stride[3] = {1, P, P * P};
  const double same = lev ? A.same1 : A.same0;
  for (int q = threadIdx.x; q < P3; q += kBlkThreads) {
    const int l[3] = {q % P - g, (q / P) % P - g, q / (P * P) - g};
    double out = 0.0;
    if (l[0] >= 0 && l[0] < nb && l[1] >= 0 && l[1] < nb && l[2] >= 0 && l[2] < nb) {
      const int c[3] = {bi * nb + l[0], bj * nb + l[1], bk * nb + l[2]};
      const double xc = xb[q], pc = pb[q];
      double s = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int dir = -1; dir <= 1; dir += 2) {
          const int pd = c[d] + dir;
          if (pd < 0 || pd >= n) continue;
          const int ld = l[d] + dir;
          const bool in_block = ld >= 0 && ld < nb;
          int e1 = d + 1, e2 = d + 2;
          if (e1 >= 3) e1 -= 3;
          if (e2 >= 3) e2 -= 3;
          if (lev == 1) {
            // neighbour on level 1 where its block is stored, else the coarse cell (both
            // in this block's guards)
            bool same_level = in_block;
            if (!in_block) {
              int p[3] = {c[0], c[1], c[2]};
              p[d] = pd;
              same_level = map1[p[0] / nb + A.nbx1 * (p[1] / nb + A.nbx1 * (p[2] / nb))] >= 0;
            }
            const int qn = q + dir * stride[d];
            const double xq = xb[qn], pq = pb[qn];
            const double beta = dir > 0 ? ghost_fluid_beta(pc, pq, rn, rp)
                                        : ghost_fluid_beta(pq, pc, rn, rp);
            s += beta * (xq - xc) * (same_level ? same : A.fine_side);
          } else {
            bool fine = false;
            if (!in_block) {
              int p[3] = {c[0], c[1], c[2]};
              p[d] = pd;
              fine = refined0[p[0] / nb + A.nbx0 * (p[1] / nb + A.nbx0 * (p[2] / nb))] != 0;
            }
            if (!fine) {
              const int qn = q + dir * stride[d];
              const double xq = xb[qn], pq = pb[qn];
              const double beta = dir > 0 ? ghost_fluid_beta(pc, pq, rn, rp)
                                          : ghost_fluid_beta(pq, pc, rn, rp);
              s += beta * (xq - xc) * same;
            } else {
#pragma unroll
              for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                  int f[3];
                  f[d] = dir > 0 ? 2 * pd : 2 * pd + 1;
                  f[e1] = 2 * c[e1] + a;
                  f[e2] = 2 * c[e2] + b;
                  const int fblk = map1[f[0] / nb + A.nbx1 * (f[1] / nb + A.nbx1 * (f[2] / nb))];
                  const size_t fo = (size_t)fblk * A.P3 + amr_local(P, g, f[0] % nb, f[1] % nb, f[2] % nb);
                  const double xq = x1[fo], pq = phi1[fo];
                  const double beta = dir > 0 ? ghost_fluid_beta(pc, pq, rn, rp)
                                              : ghost_fluid_beta(pq, pc, rn, rp);
                  s += beta * (xq - xc) * A.coarse_side;
                }
            }
          }
        }
      out = s;
    }
    yb[q] = out;
  }
}

}  // namespace mpp
