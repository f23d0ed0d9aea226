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

// Guard cells of every stored block of both levels, in place (interiors only read).  A
// guard position is mirrored about the walls on its own level; inside, a level-0 guard
// takes the level-0 value where its block is not refined and the mean of the 8 level-1
// cells it covers where it is (pairwise: x pairs, then y, then z); a level-1 guard takes
// the level-1 value where that block is stored and the value of the level-0 cell
// containing it where it is not.  One workgroup per stored block (level 0 first).  The
// workgroup first looks up the 27 blocks around its own (itself included) once: a mirrored
// guard position lies in one of them.  The children of a refined block are stored one
// after the other (child a + 2b + 4c), so the first child's index locates all eight.
template <int NB, int G>
__global__ void __launch_bounds__(kBlkThreads)
    k_amr_fill(AmrShape A, const uint8_t* __restrict__ refined0, const int* __restrict__ map1,
               const int* __restrict__ list1, double* __restrict__ b0, double* __restrict__ b1) {
  __shared__ int s_blk[27], s_kind[27];
  const int lev = (int)blockIdx.x >= A.nblk0;
  const int blk = lev ? (int)blockIdx.x - A.nblk0 : (int)blockIdx.x;
  int bi, bj, bk;
  amr_block_coords(A, lev, blk, list1, bi, bj, bk);
  const int nb = NB > 0 ? NB : A.nb, g = NB > 0 ? G : A.g, P = nb + 2 * g;
  const int n = lev ? 2 * A.n0 : A.n0;
  const int nbx = lev ? A.nbx1 : A.nbx0;
  if (threadIdx.x < 27) {
    // kind 0: a block of this level (s_blk its index); kind 1: level 0 over a refined
    // block (s_blk its first child) or level 1 over an unstored block (s_blk the level-0
    // block containing it); kind -1: outside the domain (never used)
    const int e = threadIdx.x;
    const int p[3] = {bi + e % 3 - 1, bj + (e / 3) % 3 - 1, bk + e / 9 - 1};
    int kind = -1, id = 0;
    if (p[0] >= 0 && p[0] < nbx && p[1] >= 0 && p[1] < nbx && p[2] >= 0 && p[2] < nbx) {
      const int pos = p[0] + nbx * (p[1] + nbx * p[2]);
      if (lev == 0) {
        kind = refined0[pos] != 0;
        id = kind ? map1[2 * p[0] + A.nbx1 * (2 * p[1] + A.nbx1 * 2 * p[2])] : pos;
      } else {
        const int fb = map1[pos];
        kind = fb < 0;
        id = kind ? p[0] / 2 + A.nbx0 * (p[1] / 2 + A.nbx0 * (p[2] / 2)) : fb;
      }
    }
    s_kind[e] = kind;
    s_blk[e] = id;
  }
  __syncthreads();
  double* const own = (lev ? b1 : b0) + (size_t)blk * A.P3;
  const int guards = P * P * P - nb * nb * nb;
  for (int q = threadIdx.x; q < guards; q += kBlkThreads) {
    int li, lj, lk;
    blk_guard_cell(q, nb, g, P, li, lj, lk);
    const int I = blk_mirror(bi * nb + li, n), J = blk_mirror(bj * nb + lj, n),
              K = blk_mirror(bk * nb + lk, n);
    const int e = (I / nb - bi + 1) + 3 * (J / nb - bj + 1) + 9 * (K / nb - bk + 1);
    const int kind = s_kind[e], id = s_blk[e];
    double v;
    if (kind == 0) {
      v = (lev ? b1 : b0)[(size_t)id * A.P3 + amr_local(P, g, I % nb, J % nb, K % nb)];
    } else if (lev == 0) {
      // the 8 level-1 cells under level-0 cell (I, J, K), in child blocks id + a + 2b + 4c
      double s[4];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int fj = 2 * J + b, fk = 2 * K + c;
          double v2[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const int fi = 2 * I + a;
            const int ch = ((fi / nb) & 1) + 2 * ((fj / nb) & 1) + 4 * ((fk / nb) & 1);
            v2[a] = b1[(size_t)(id + ch) * A.P3 + amr_local(P, g, fi % nb, fj % nb, fk % nb)];
          }
          s[b + 2 * c] = v2[0] + v2[1];
        }
      v = 0.125 * ((s[0] + s[1]) + (s[2] + s[3]));
    } else {
      const int Ic = I / 2, Jc = J / 2, Kc = K / 2;
      v = b0[(size_t)id * A.P3 + amr_local(P, g, Ic % nb, Jc % nb, Kc % nb)];
    }
    own[amr_local(P, g, li, lj, lk)] = v;
  }
}

// Ghost-fluid coefficient of the face between centres a (lower) and b: 1/rho of the phase
// when both are on one side (irn = 1/rn, irp = 1/rp, the same correctly rounded values a
// division gives), else the series value 1 / (theta rho_a + (1 - theta) rho_b) with theta
// the fraction of the segment on a's side.
__device__ inline double amr_beta(double pa, double pb, double rn, double rp, double irn,
                                  double irp) {
#pragma clang fp contract(off)
  const bool a = pa > 0.0, b = pb > 0.0;
  if (a == b) return a ? irp : irn;
  const double theta = fabs(pa) / (fabs(pa) + fabs(pb));
  return 1.0 / (theta * (a ? rp : rn) + (1.0 - theta) * (b ? rp : rn));
}

// (A x)_c of one leaf cell c (global coordinates c[], local l[] in its block of level
// `lev`), its value xc and level set pc, and the values xn[f], pn[f] of the six guard or
// interior positions next to it in its padded block (f = 2 d + (dir > 0)).  other[f] is 1
// where the block across face f is on the other level (coarser for a level-1 block,
// refined for a level-0 block), else 0 (read only for cells on that face).  Terms in the
// order x-, x+, y-, y+, z-, z+; the four fine cells of a coarse-fine face in the order of
// the next two axes, cyclically.  DIAG: the diagonal A_cc instead (x read as 1 at c and 0
// at every neighbour).
template <bool DIAG = false>
__device__ inline double amr_cell(const AmrShape& A, int lev, int nb, int g, int P, int n,
                                  const int* __restrict__ map1, const double* __restrict__ phi1,
                                  const double* __restrict__ x1, const int other[6],
                                  const int c[3], const int l[3],
                                  double xc, double pc, const double xn[6], const double pn[6],
                                  double rn, double rp, double same) {
#pragma clang fp contract(off)
  const double irn = 1.0 / rn, irp = 1.0 / rp;
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int dir = side ? 1 : -1;
      const int pd = c[d] + dir;
      if (pd < 0 || pd >= n) continue;
      const int ld = l[d] + dir;
      const bool in_block = ld >= 0 && ld < nb;
      const double xq = xn[2 * d + side], pq = pn[2 * d + side];
      const bool same_level = in_block || other[2 * d + side] == 0;
      if (lev == 1) {
        // a neighbour on level 1 where its block is stored, else the coarse cell (both
        // held by this block's guards)
        const double beta = side ? amr_beta(pc, pq, rn, rp, irn, irp) : amr_beta(pq, pc, rn, rp, irn, irp);
        s += beta * (xq - xc) * (same_level ? same : A.fine_side);
      } else if (same_level) {
        const double beta = side ? amr_beta(pc, pq, rn, rp, irn, irp) : amr_beta(pq, pc, rn, rp, irn, irp);
        s += beta * (xq - xc) * same;
      } else {
        int e1 = d + 1, e2 = d + 2;
        if (e1 >= 3) e1 -= 3;
        if (e2 >= 3) e2 -= 3;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            int f[3];
            f[d] = side ? 2 * pd : 2 * pd + 1;
            f[e1] = 2 * c[e1] + a;
            f[e2] = 2 * c[e2] + b;
            const int fblk = map1[f[0] / nb + A.nbx1 * (f[1] / nb + A.nbx1 * (f[2] / nb))];
            const size_t fo = (size_t)fblk * A.P3 + amr_local(P, g, f[0] % nb, f[1] % nb, f[2] % nb);
            const double xf = DIAG ? 0.0 : x1[fo], pf = phi1[fo];
            const double beta = side ? amr_beta(pc, pf, rn, rp, irn, irp) : amr_beta(pf, pc, rn, rp, irn, irp);
            s += beta * (xf - xc) * A.coarse_side;
          }
      }
    }
  return s;
}

// y = A x on the leaves, x and phi in blocks with filled guards (g >= 1).  A level-1 cell
// and an unrefined level-0 cell take every neighbour of their own level, and a fine
// cell its coarse neighbours, from the guards of their own block; a level-0 cell next to
// a refined block reads the four level-1 cells across the face from their blocks.  Guards
// of y and every value of a refined level-0 block are set to 0.  One workgroup per stored
// block (level 0 first; two per block for 16^3 blocks with one guard layer, one
// otherwise).  When a plane of the block has as many cells as the workgroup has threads,
// each thread marches up one column, keeping the values below and at the current cell in
// registers; otherwise the threads stride over the block.
template <int NB, int G>
__global__ void __launch_bounds__(kBlkThreads)
    k_amr_apply(AmrShape A, const uint8_t* __restrict__ refined0, const int* __restrict__ map1,
                const int* __restrict__ list1, const double* __restrict__ phi0,
                const double* __restrict__ phi1, const double* __restrict__ x0,
                const double* __restrict__ x1, double rn, double rp, double* __restrict__ y0,
                double* __restrict__ y1) {
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
    // each of the gridDim.y workgroups of the block clears its share of the planes
    const int pl0 = P * (int)blockIdx.y / (int)gridDim.y, pl1 = P * ((int)blockIdx.y + 1) / (int)gridDim.y;
    for (int q = pl0 * P * P + threadIdx.x; q < pl1 * P * P; q += kBlkThreads) yb[q] = 0.0;
    return;
  }
  const double same = lev ? A.same1 : A.same0;
  // level of the block across each face (a face on a wall is never read)
  int other[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    int p[3] = {bi, bj, bk};
    p[f >> 1] += (f & 1) ? 1 : -1;
    const int nbx = lev ? A.nbx1 : A.nbx0;
    other[f] = 0;
    if (p[f >> 1] >= 0 && p[f >> 1] < nbx)
      other[f] = lev ? (map1[p[0] + nbx * (p[1] + nbx * p[2])] < 0)
                     : (refined0[p[0] + nbx * (p[1] + nbx * p[2])] != 0);
  }
  if constexpr (NB == 16 && G == 1) {
    // Two workgroups per block (blockIdx.y: lower or upper 8 planes).  The 10 padded
    // planes x and phi of a half need are staged in LDS (51840 bytes, three workgroups
    // per compute unit) with every load in flight at once; each thread then marches up
    // one column of the half.  A half writes y on 9 of the 18 padded planes.
    constexpr int PPl = 18 * 18, HZ = 8, NPL = HZ + 2;
    __shared__ double sx[NPL * PPl], sp[NPL * PPl];
    const int hz = blockIdx.y;
    const int k0 = hz * HZ;   // first interior plane of the half; padded plane k0 is below it
    const double* const xs = xb + (size_t)k0 * PPl;
    const double* const ps = pb + (size_t)k0 * PPl;
    for (int t = threadIdx.x; t < NPL * PPl; t += kBlkThreads) {
      sx[t] = xs[t];
      sp[t] = ps[t];
    }
    for (int t = threadIdx.x; t < 9 * PPl; t += kBlkThreads) {
      const int pk = hz * 9 + t / PPl, pj = (t % PPl) / 18, pi = t % 18;
      if (pk == 0 || pk == 17 || pj == 0 || pj == 17 || pi == 0 || pi == 17)
        yb[(size_t)pk * PPl + pj * 18 + pi] = 0.0;
    }
    __syncthreads();
    const int li = threadIdx.x % 16, lj = threadIdx.x / 16;
    for (int kk = 0; kk < HZ; ++kk) {
      const int lk = k0 + kk;
      const int t = (kk + 1) * PPl + (lj + 1) * 18 + (li + 1);
      const double xn[6] = {sx[t - 1], sx[t + 1], sx[t - 18], sx[t + 18], sx[t - PPl], sx[t + PPl]};
      const double pn[6] = {sp[t - 1], sp[t + 1], sp[t - 18], sp[t + 18], sp[t - PPl], sp[t + PPl]};
      const int c[3] = {bi * 16 + li, bj * 16 + lj, bk * 16 + lk};
      const int l[3] = {li, lj, lk};
      yb[amr_local(18, 1, li, lj, lk)] = amr_cell(A, lev, 16, 1, 18, n, map1, phi1, x1,
                                                  other, c, l, sx[t], sp[t], xn, pn, rn, rp, same);
    }
  } else if constexpr (NB > 0 && NB * NB == kBlkThreads) {
    const int guards = P3 - NB * NB * NB;
    for (int q = threadIdx.x; q < guards; q += kBlkThreads) {
      int li, lj, lk;
      blk_guard_cell(q, NB, G, P, li, lj, lk);
      yb[amr_local(P, G, li, lj, lk)] = 0.0;
    }
    const int li = threadIdx.x % NB, lj = threadIdx.x / NB;
    const int PP = P * P;
    int q = (int)amr_local(P, G, li, lj, 0);
    double xlo = xb[q - PP], plo = pb[q - PP], xc = xb[q], pc = pb[q];
    for (int lk = 0; lk < NB; ++lk, q += PP) {
      const double xn[6] = {xb[q - 1], xb[q + 1], xb[q - P], xb[q + P], xlo, xb[q + PP]};
      const double pn[6] = {pb[q - 1], pb[q + 1], pb[q - P], pb[q + P], plo, pb[q + PP]};
      const int c[3] = {bi * NB + li, bj * NB + lj, bk * NB + lk};
      const int l[3] = {li, lj, lk};
      yb[q] = amr_cell(A, lev, NB, G, P, n, map1, phi1, x1, other, c, l, xc, pc, xn, pn, rn,
                       rp, same);
      xlo = xc;
      plo = pc;
      xc = xn[5];
      pc = pn[5];
    }
  } else {
    const int stride[3] = {1, P, P * P};
    for (int q = threadIdx.x; q < P3; q += kBlkThreads) {
      const int l[3] = {q % P - g, (q / P) % P - g, q / (P * P) - g};
      double out = 0.0;
      if (l[0] >= 0 && l[0] < nb && l[1] >= 0 && l[1] < nb && l[2] >= 0 && l[2] < nb) {
        const int c[3] = {bi * nb + l[0], bj * nb + l[1], bk * nb + l[2]};
        double xn[6], pn[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const int qn = q + ((f & 1) ? 1 : -1) * stride[f >> 1];
          xn[f] = xb[qn];
          pn[f] = pb[qn];
        }
        out = amr_cell(A, lev, nb, g, P, n, map1, phi1, x1, other, c, l, xb[q], pb[q], xn, pn,
                       rn, rp, same);
      }
      yb[q] = out;
    }
  }
}

// ------------------------------------------------------------------------------------
// Conjugate gradients on the composite grid, preconditioned with the inverse diagonal, in
// the volume-weighted inner product <u, v> = sum over leaves of V_c u_c v_c (A is
// symmetric in it and -A positive semi-definite).  Vectors live in the block layout of
// both levels; only the interiors of leaf blocks are read or written.  Every reduction is
// a per-block partial followed by one workgroup summing the partials in a fixed order, so
// results do not depend on scheduling.  Scalars stay on the device.
// ------------------------------------------------------------------------------------
enum AmrSlot { AS_MEAN, AS_BB, AS_RZ, AS_RR, AS_ALPHA, AS_BETA, AS_FLAG, AS_XMEAN, AS_COUNT };

// -diag(A) on the interiors of leaf blocks (phi with filled guards)
template <int NB, int G>
__global__ void __launch_bounds__(kBlkThreads)
    k_amr_negdiag(AmrShape A, const uint8_t* __restrict__ refined0, const int* __restrict__ map1,
                  const int* __restrict__ list1, const double* __restrict__ phi0,
                  const double* __restrict__ phi1, double rn, double rp, double* __restrict__ d0,
                  double* __restrict__ d1) {
  const int lev = (int)blockIdx.x >= A.nblk0;
  const int blk = lev ? (int)blockIdx.x - A.nblk0 : (int)blockIdx.x;
  if (lev == 0 && refined0[blk]) return;
  int bi, bj, bk;
  amr_block_coords(A, lev, blk, list1, bi, bj, bk);
  const int nb = NB > 0 ? NB : A.nb, g = NB > 0 ? G : A.g, P = nb + 2 * g;
  const int n = lev ? 2 * A.n0 : A.n0;
  const int nbx = lev ? A.nbx1 : A.nbx0;
  int other[6];
  for (int f = 0; f < 6; ++f) {
    int p[3] = {bi, bj, bk};
    p[f >> 1] += (f & 1) ? 1 : -1;
    other[f] = 0;
    if (p[f >> 1] >= 0 && p[f >> 1] < nbx)
      other[f] = lev ? (map1[p[0] + nbx * (p[1] + nbx * p[2])] < 0)
                     : (refined0[p[0] + nbx * (p[1] + nbx * p[2])] != 0);
  }
  const size_t base = (size_t)blk * A.P3;
  const double* const pb = (lev ? phi1 : phi0) + base;
  double* const db = (lev ? d1 : d0) + base;
  const int stride[3] = {1, P, P * P};
  const double zero[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < nb * nb * nb; t += kBlkThreads) {
    const int l[3] = {t % nb, (t / nb) % nb, t / (nb * nb)};
    const int c[3] = {bi * nb + l[0], bj * nb + l[1], bk * nb + l[2]};
    const int q = (int)amr_local(P, g, l[0], l[1], l[2]);
    double pn[6];
    for (int f = 0; f < 6; ++f) pn[f] = pb[q + ((f & 1) ? 1 : -1) * stride[f >> 1]];
    db[q] = -amr_cell<true>(A, lev, nb, g, P, n, map1, phi1, nullptr, other, c, l, 1.0, pb[q],
                            zero, pn, rn, rp, lev ? A.same1 : A.same0);
  }
}

// sum over the workgroup of v (every thread passes its value; thread 0 gets the total)
__device__ inline double amr_block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBlkThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Vector steps over the interiors of leaf blocks, each with up to two weighted partial
// sums per block (part[blockIdx.x] and part[nblocks + blockIdx.x]):
//   MEAN:  partial <u, 1>                              (u = a)
//   INIT:  r = b - S[MEAN] (a = b), partial <r, r>
//   RES:   r -= q, z = r / negd, p = z, partials <r, z>, <r, r>
//   DOT:   partial <p, q>
//   STEP:  x -= S[ALPHA] p, r += S[ALPHA] q, z = r / negd, partials <r, z>, <r, r>
//   DIR:   p = z + S[BETA] p
//   SHIFT: x -= S[XMEAN]
// and the steps of the two-level preconditioner z ~= (-A)^{-1} r:
//   MOVE:  x -= S[ALPHA] p, r += S[ALPHA] q
//   R:     r -= q, partial <r, r> (second slot)
//   JAC0:  z = omega r / negd
//   JAC:   z += omega (r + t) / negd            (t = A z: damped Jacobi on -A z = r)
//   CADD:  z -= zc(parent level-0 cell)         (zc ~= A0^{-1} of the averaged residual)
//   ZDOT:  partials <r, z>, <r, r>
//   ZDOTP: as ZDOT, and p = z
// Refined level-0 blocks contribute 0 and are left as they are.
enum AmrVec { AV_MEAN, AV_INIT, AV_RES, AV_DOT, AV_STEP, AV_DIR, AV_SHIFT, AV_MOVE, AV_R,
              AV_JAC0, AV_JAC, AV_CADD, AV_ZDOT, AV_ZDOTP };

struct AmrVecs {
  double *x[2], *r[2], *z[2], *p[2], *q[2], *t[2];
  const double *b[2], *negd[2];
  const double* zc;   // coarse correction on the level-0 grid (n0^3, x fastest)
  double omega;       // Jacobi damping of the multigrid smoother
};

template <int MODE, int NB, int G>
__global__ void __launch_bounds__(kBlkThreads)
    k_amr_vec(AmrShape A, const uint8_t* __restrict__ refined0, const int* __restrict__ list1,
              AmrVecs V, const double* __restrict__ S, double* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ double sh[kBlkThreads];
  const int lev = (int)blockIdx.x >= A.nblk0;
  const int blk = lev ? (int)blockIdx.x - A.nblk0 : (int)blockIdx.x;
  const int nblocks = A.nblk0 + A.nblk1;
  if (lev == 0 && refined0[blk]) {
    if (threadIdx.x == 0) {
      part[blockIdx.x] = 0.0;
      part[nblocks + blockIdx.x] = 0.0;
    }
    return;
  }
  const int nb = NB > 0 ? NB : A.nb, g = NB > 0 ? G : A.g, P = nb + 2 * g;
  const size_t base = (size_t)blk * A.P3;
  double* const x = V.x[lev] + base;
  double* const r = V.r[lev] + base;
  double* const z = V.z[lev] + base;
  double* const p = V.p[lev] + base;
  double* const q = V.q[lev] + base;
  double* const tt = V.t[lev] ? V.t[lev] + base : nullptr;
  const double* const bb = V.b[lev] ? V.b[lev] + base : nullptr;
  const double* const nd = V.negd[lev] + base;
  const double alpha = S[AS_ALPHA], beta = S[AS_BETA], om = V.omega;
  int bi = 0, bj = 0, bk = 0;
  if (MODE == AV_CADD) amr_block_coords(A, lev, blk, list1, bi, bj, bk);
  double s1 = 0.0, s2 = 0.0;
  for (int t = threadIdx.x; t < nb * nb * nb; t += kBlkThreads) {
    const int li = t % nb, lj = (t / nb) % nb, lk = t / (nb * nb);
    const int c = (int)amr_local(P, g, li, lj, lk);
    if (MODE == AV_MOVE) {
      x[c] = x[c] - alpha * p[c];
      r[c] = r[c] + alpha * q[c];
    } else if (MODE == AV_R) {
      const double rv = r[c] - q[c];
      r[c] = rv;
      s2 += rv * rv;
    } else if (MODE == AV_JAC0) {
      z[c] = om * r[c] / nd[c];
    } else if (MODE == AV_JAC) {
      z[c] = z[c] + om * (r[c] + tt[c]) / nd[c];
    } else if (MODE == AV_CADD) {
      // the parent level-0 cell of a level-1 cell is at half its coordinates
      const int I = lev ? (bi * nb + li) >> 1 : bi * nb + li;
      const int J = lev ? (bj * nb + lj) >> 1 : bj * nb + lj;
      const int K = lev ? (bk * nb + lk) >> 1 : bk * nb + lk;
      z[c] = z[c] - V.zc[(size_t)I + (size_t)A.n0 * ((size_t)J + (size_t)A.n0 * K)];
    } else if (MODE == AV_ZDOT || MODE == AV_ZDOTP) {
      const double rv = r[c], zv = z[c];
      if (MODE == AV_ZDOTP) p[c] = zv;
      s1 += rv * zv;
      s2 += rv * rv;
    } else if (MODE == AV_MEAN) {
      s1 += bb[c];
    } else if (MODE == AV_INIT) {
      const double v = bb[c] - S[AS_MEAN];
      r[c] = v;
      s1 += v * v;
    } else if (MODE == AV_RES || MODE == AV_STEP) {
      double rv;
      if (MODE == AV_RES) {
        rv = r[c] - q[c];
      } else {
        x[c] = x[c] - alpha * p[c];
        rv = r[c] + alpha * q[c];
      }
      const double zv = rv / nd[c];
      r[c] = rv;
      z[c] = zv;
      if (MODE == AV_RES) p[c] = zv;
      s1 += rv * zv;
      s2 += rv * rv;
    } else if (MODE == AV_DOT) {
      s1 += p[c] * q[c];
    } else if (MODE == AV_DIR) {
      p[c] = z[c] + beta * p[c];
    } else if (MODE == AV_SHIFT) {
      x[c] = x[c] - S[AS_XMEAN];
    }
  }
  if (MODE == AV_DIR || MODE == AV_SHIFT || MODE == AV_MOVE || MODE == AV_JAC0 ||
      MODE == AV_JAC || MODE == AV_CADD)
    return;
  const double vol = lev ? 1.0 / (8.0 * (double)A.n0 * A.n0 * A.n0) : 1.0 / ((double)A.n0 * A.n0 * A.n0);
  const double t1 = amr_block_sum(s1, sh);
  const double t2 = (MODE == AV_RES || MODE == AV_STEP || MODE == AV_R || MODE == AV_ZDOT ||
                     MODE == AV_ZDOTP)
                        ? amr_block_sum(s2, sh)
                        : 0.0;
  if (threadIdx.x == 0) {
    part[blockIdx.x] = vol * t1;
    part[nblocks + blockIdx.x] = vol * t2;
  }
}

// One workgroup: sums the partials (thread t takes t, t + 256, ..., then a tree) and
// updates the scalars for the step that produced them.
enum AmrFin { AF_MEAN, AF_BB, AF_RZ0, AF_ALPHA, AF_BETA, AF_XMEAN, AF_RR };

__global__ void __launch_bounds__(kBlkThreads)
    k_amr_finish(int MODE, const double* __restrict__ part, int nblocks, double* __restrict__ S) {
  __shared__ double sh[kBlkThreads];
  double a = 0.0, b = 0.0;
  for (int t = threadIdx.x; t < nblocks; t += kBlkThreads) {
    a += part[t];
    b += part[nblocks + t];
  }
  const double ta = amr_block_sum(a, sh);
  const double tb = amr_block_sum(b, sh);
  if (threadIdx.x != 0) return;
  switch (MODE) {
    case AF_MEAN: S[AS_MEAN] = ta; break;
    case AF_BB: S[AS_BB] = ta; break;
    case AF_RZ0: S[AS_RZ] = ta; S[AS_RR] = tb; break;
    case AF_ALPHA:
      // <p, A p> < 0 unless p = 0 (then the search has nothing left to do)
      if (ta < 0.0) {
        S[AS_ALPHA] = -S[AS_RZ] / ta;
      } else {
        S[AS_ALPHA] = 0.0;
        S[AS_FLAG] = 1.0;
      }
      break;
    case AF_BETA:
      S[AS_BETA] = S[AS_RZ] != 0.0 ? ta / S[AS_RZ] : 0.0;
      S[AS_RZ] = ta;
      S[AS_RR] = tb;
      break;
    case AF_XMEAN: S[AS_XMEAN] = ta; break;
    case AF_RR: S[AS_RR] = tb; break;
  }
}

// Volume average over every level-0 cell of a + b (b may be null), two composite fields,
// onto the level-0 grid (n0^3, x fastest): the level-0 value where the block is not
// refined, else the mean of the 8 level-1 cells (pairwise: x pairs, then y, then z).
template <int NB, int G>
__global__ void __launch_bounds__(kBlkThreads)
    k_amr_restrict(AmrShape A, const uint8_t* __restrict__ refined0, const int* __restrict__ map1,
                   const double* __restrict__ a0, const double* __restrict__ a1,
                   const double* __restrict__ b0, const double* __restrict__ b1,
                   double* __restrict__ out) {
  const int nb = NB > 0 ? NB : A.nb, g = NB > 0 ? G : A.g, P = nb + 2 * g;
  const int n0 = A.n0;
  const size_t cells = (size_t)n0 * n0 * n0;
  for (size_t c = (size_t)blockIdx.x * kBlkThreads + threadIdx.x; c < cells;
       c += (size_t)gridDim.x * kBlkThreads) {
    const int I = (int)(c % n0), J = (int)((c / n0) % n0), K = (int)(c / ((size_t)n0 * n0));
    const int ob = I / nb + A.nbx0 * (J / nb + A.nbx0 * (K / nb));
    double v;
    if (!refined0[ob]) {
      const size_t o = (size_t)ob * A.P3 + amr_local(P, g, I % nb, J % nb, K % nb);
      v = b0 ? a0[o] + b0[o] : a0[o];
    } else {
      // children of a refined block are stored one after the other from the first
      const int id = map1[2 * (I / nb) + A.nbx1 * (2 * (J / nb) + A.nbx1 * 2 * (K / nb))];
      double s[4];
      for (int cc = 0; cc < 2; ++cc)
        for (int b = 0; b < 2; ++b) {
          const int fj = 2 * J + b, fk = 2 * K + cc;
          double v2[2];
          for (int a = 0; a < 2; ++a) {
            const int fi = 2 * I + a;
            const int ch = ((fi / nb) & 1) + 2 * ((fj / nb) & 1) + 4 * ((fk / nb) & 1);
            const size_t o = (size_t)(id + ch) * A.P3 + amr_local(P, g, fi % nb, fj % nb, fk % nb);
            v2[a] = b1 ? a1[o] + b1[o] : a1[o];
          }
          s[b + 2 * cc] = v2[0] + v2[1];
        }
      v = 0.125 * ((s[0] + s[1]) + (s[2] + s[3]));
    }
    out[c] = v;
  }
}

// The level-0 operator of the two-level cycle, made to see the fine level: every face of
// the level-0 grid that touches a refined block takes the mean of the four fine-level
// coefficients across it (as the uniform hierarchy averages faces from level to level):
// between two refined blocks the coefficients of the four pairs of level-1 cells, across
// a coarse-fine face those of the four level-1 cells and the level-0 cell.  The faces are
// written in the grid layout of the operator (low face of each cell, FP64 and FP32), and
// every cell's code byte marks each of its faces so changed as crossed, so that every
// sweep reads the face arrays there.  One thread per level-0 cell; each writes only its
// own faces and code byte.
template <int NB, int G>
__global__ void __launch_bounds__(256)
    k_amr_coarse_faces(AmrShape A, const uint8_t* __restrict__ refined0,
                       const int* __restrict__ map1, const double* __restrict__ phi0,
                       const double* __restrict__ phi1, double rn, double rp,
                       uint8_t* __restrict__ code, double* __restrict__ bx, double* __restrict__ by,
                       double* __restrict__ bz, float* __restrict__ fx, float* __restrict__ fy,
                       float* __restrict__ fz) {
#pragma clang fp contract(off)
  const int nb = NB > 0 ? NB : A.nb, g = NB > 0 ? G : A.g, P = nb + 2 * g;
  const int n0 = A.n0;
  const size_t cells = (size_t)n0 * n0 * n0;
  const double irn = 1.0 / rn, irp = 1.0 / rp;
  auto refined = [&](int I, int J, int K) {
    return refined0[I / nb + A.nbx0 * (J / nb + A.nbx0 * (K / nb))] != 0;
  };
  // level set at level-1 cell f of a refined block, else at the level-0 cell containing it
  auto phi_at = [&](const int f[3]) {
    const int I = f[0] >> 1, J = f[1] >> 1, K = f[2] >> 1;
    if (!refined(I, J, K)) return phi0[(size_t)I + (size_t)n0 * ((size_t)J + (size_t)n0 * K)];
    const int blk = map1[f[0] / nb + A.nbx1 * (f[1] / nb + A.nbx1 * (f[2] / nb))];
    return phi1[(size_t)blk * A.P3 + amr_local(P, g, f[0] % nb, f[1] % nb, f[2] % nb)];
  };
  double* const bd[3] = {bx, by, bz};
  float* const fd[3] = {fx, fy, fz};
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < cells; c += (size_t)gridDim.x * 256) {
    const int C[3] = {(int)(c % n0), (int)((c / n0) % n0), (int)(c / ((size_t)n0 * n0))};
    const bool rc = refined(C[0], C[1], C[2]);
    unsigned mark = 0;
    for (int d = 0; d < 3; ++d) {
      int e1 = d + 1, e2 = d + 2;
      if (e1 >= 3) e1 -= 3;
      if (e2 >= 3) e2 -= 3;
      // low face: between c - e_d and c
      if (C[d] > 0) {
        int L[3] = {C[0], C[1], C[2]};
        L[d] -= 1;
        if (rc || refined(L[0], L[1], L[2])) {
          double s[4];
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
              int lo[3], hi[3];
              lo[d] = 2 * C[d] - 1;
              hi[d] = 2 * C[d];
              lo[e1] = hi[e1] = 2 * C[e1] + a;
              lo[e2] = hi[e2] = 2 * C[e2] + b;
              s[a + 2 * b] = amr_beta(phi_at(lo), phi_at(hi), rn, rp, irn, irp);
            }
          const double v = 0.25 * ((s[0] + s[1]) + (s[2] + s[3]));
          bd[d][c] = v;
          fd[d][c] = (float)v;
          mark |= 1u << (2 * d);
        }
      }
      // high face: its value is written by the cell above; only the mark is ours
      if (C[d] < n0 - 1) {
        int H[3] = {C[0], C[1], C[2]};
        H[d] += 1;
        if (rc || refined(H[0], H[1], H[2])) mark |= 2u << (2 * d);
      }
    }
    if (mark) code[c] = (uint8_t)(code[c] | mark);
  }
}

}  // namespace mpp
