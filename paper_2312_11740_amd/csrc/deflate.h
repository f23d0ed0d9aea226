// Deflation of the bubble regions (subdomain deflation for bubbly flows: Nicolaides 1987;
// Tang & Vuik 2007, the "DEF1" variant of Tang, Nabben, Vuik & Erlangga 2009).
//
// At a density ratio of 1000 each connected region of the light phase (a bubble) adds a
// small eigenvalue to the multigrid-preconditioned operator: inside a bubble the face
// coefficients are a thousand times those of the liquid, so a field that is constant on
// the bubble costs almost nothing and the V-cycle damps it slowly.  With Z the matrix
// whose columns are the indicator fields of the k regions (k <= kDefMax), E = Z^T A Z
// (k x k, negative definite) and P = I - A Z E^{-1} Z^T, CG runs on the deflated system
// P A x^ = P b with the V-cycle as preconditioner, and the solution is
//     x = x^ + Z E^{-1} Z^T (b - A x^).
// P A p = q - (A Z) a with q = A p, s = Z^T q = (A Z)^T p (A is symmetric) and a = E^{-1} s,
// so the deflation costs, per iteration, sums over the cells where some A z_j is nonzero
// (the "band": cells next to a region's boundary, on both sides) and a correction of r
// there; p.(P q) = p.q - a.s needs no pass of its own.  The preconditioned residual is
// projected, z = P^T V(r) (z -= Z E^{-1} (A Z)^T z: band sums and a pass over the region
// cells), which makes the preconditioned operator symmetric and keeps the directions
// A-orthogonal to the regions: the V-cycle amplifies exactly the slow region modes, and
// without the projection p.q - a.s becomes the difference of two nearly equal large
// terms, which FP32 inner solves do not survive.  r.z needs no change (P r = r).
//
// Regions: connected components (through faces) of the cells on the light side of the
// interface, found by label propagation (each cell takes the smallest cell index among
// itself and its neighbours, then follows labels and hooks the old root), which ends with
// every component labelled by its smallest cell index; the kDefMax components with the
// smallest such indices are kept, numbered 1..k in that order.  Every step is
// deterministic (integer minima, compactions in cell order, sums in fixed order).
#pragma once

#include "kernels.h"
#include "rbgs.h"

namespace mpp {

constexpr int kDefThreads = 256;
constexpr int kDefChunk = 4096;      // cells per block of the compactions over the grid

// ---- labels of the light-phase regions --------------------------------------------
// light[b]: side bit (0: phi <= 0, 1: phi > 0) of the lighter phase, -1: no deflation.
// The light cells are first compacted into a list (cell order); the labels are kept in a
// grid-sized array but only ever read at light cells (a neighbour's phase comes from its
// code byte), so nothing else of the array needs a value.
__device__ inline bool is_light(const uint8_t* __restrict__ code, size_t base, int c, int ls) {
  return ls >= 0 && (int)((code[base + c] >> 6) & 1) == ls;
}

__global__ void k_ccl_init(const int* __restrict__ list, const int* __restrict__ lcount, int lcap,
                           int cells, int* __restrict__ lab) {
  const int b = blockIdx.y;
  const int cnt = lcount[b];
  const int* Lst = list + (size_t)b * lcap;
  int* L = lab + (size_t)b * cells;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
    const int c = Lst[q];
    L[c] = c;
  }
}

// One round of propagation over the light cells: smallest label among the cell and its
// light face neighbours, then up to four steps along the labels, and the old label's cell
// takes the new one too (labels only decrease and always name a cell of the same
// component).
// prev: the previous round's changed flags (nullptr for the first round of a batch); a
// round after one that changed nothing has nothing to do.
__global__ void k_ccl_round(int n, const uint8_t* __restrict__ code, const int* __restrict__ light,
                            const int* __restrict__ list, const int* __restrict__ lcount, int lcap,
                            int* __restrict__ lab, const int* __restrict__ prev,
                            int* __restrict__ changed) {
  const int b = blockIdx.y;
  if (prev && prev[b] == 0) return;
  const int cells = n * n * n;
  const size_t base = (size_t)b * cells;
  const int ls = light[b];
  const int cnt = lcount[b];
  const int* Lst = list + (size_t)b * lcap;
  int* L = lab + base;
  const int nn = n * n;
  int any = 0;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
    const int c = Lst[q];
    const int old = L[c];
    int i, j, k;
    ijk(c, n, i, j, k);
    int m = old;
    if (i > 0 && is_light(code, base, c - 1, ls)) m = min(m, L[c - 1]);
    if (i < n - 1 && is_light(code, base, c + 1, ls)) m = min(m, L[c + 1]);
    if (j > 0 && is_light(code, base, c - n, ls)) m = min(m, L[c - n]);
    if (j < n - 1 && is_light(code, base, c + n, ls)) m = min(m, L[c + n]);
    if (k > 0 && is_light(code, base, c - nn, ls)) m = min(m, L[c - nn]);
    if (k < n - 1 && is_light(code, base, c + nn, ls)) m = min(m, L[c + nn]);
    for (int t = 0; t < 4; ++t) {
      const int m2 = L[m];
      if (m2 < m) m = m2;
      else break;
    }
    if (m < old) {
      atomicMin(&L[c], m);
      // many cells of a component share `old`: the atomic only where it still lowers the
      // label (the same result, without thousands of atomics on one word)
      if (L[old] > m) atomicMin(&L[old], m);
      any = 1;
    }
  }
  if (__builtin_amdgcn_ballot_w64(any != 0) != 0 && (threadIdx.x & 63) == 0) changed[b] = 1;
}

__global__ void k_int_fill(int* __restrict__ v, int count, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) v[i] = value;
}

// Counts that follow from a compaction, on the device: the light cells of a problem
// (none if it has no lighter phase or more than lcap of them), its regions (the first
// kDefMax components; none without light cells) and its band cells (at most cap).
__global__ void k_light_done(int* __restrict__ lcount, const int* __restrict__ total,
                             const int* __restrict__ light, int lcap, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) lcount[b] = (light[b] >= 0 && total[b] <= lcap) ? total[b] : 0;
}
__global__ void k_regions_done(int* __restrict__ k, const int* __restrict__ total,
                               const int* __restrict__ lcount, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) k[b] = lcount[b] > 0 ? min(total[b], kDefMax) : 0;
}
__global__ void k_band_done(int* __restrict__ bcount, const int* __restrict__ total, int cap,
                            int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) bcount[b] = min(total[b], cap);
}

// ---- deterministic compaction over the cells of a problem ---------------------------
// The block handles cells [blk * kDefChunk, (blk + 1) * kDefChunk); ranks within a block
// follow cell order (wave ballots, then waves in order).
__device__ inline int block_rank(bool hit, int& total, int* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long m = __builtin_amdgcn_ballot_w64(hit);
  const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
  if (lane == 0) sh[w] = __builtin_popcountll(m);
  __syncthreads();
  int off = 0;
  total = 0;
  for (int q = 0; q < kDefThreads / 64; ++q) {
    if (q < w) off += sh[q];
    total += sh[q];
  }
  __syncthreads();
  return off + below;
}

// Exclusive prefix over the per-block counts of each problem (one block per problem);
// total[b] receives the sum.
__global__ void __launch_bounds__(1024)
    k_scan_counts(int* __restrict__ counts, int nblk, int* __restrict__ total) {
  const int b = blockIdx.x;
  int* C = counts + (size_t)b * nblk;
  __shared__ int sh[1024];
  const int per = (nblk + 1023) / 1024;
  const int t0 = threadIdx.x * per;
  int s = 0;
  for (int q = t0; q < min(t0 + per, nblk); ++q) s += C[q];
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int q = 0; q < 1024; ++q) {
      const int v = sh[q];
      sh[q] = acc;
      acc += v;
    }
    total[b] = acc;
  }
  __syncthreads();
  int acc = sh[threadIdx.x];
  for (int q = t0; q < min(t0 + per, nblk); ++q) {
    const int v = C[q];
    C[q] = acc;
    acc += v;
  }
}

// light cells of each problem: per-block counts over chunks of cells
__global__ void __launch_bounds__(kDefThreads)
    k_light_count(const uint8_t* __restrict__ code, int cells, const int* __restrict__ light,
                  int* __restrict__ counts, int nblk) {
  const int b = blockIdx.y;
  const size_t base = (size_t)b * cells;
  const int ls = light[b];
  __shared__ int sh[kDefThreads / 64];
  int cnt = 0;
  const int c0 = blockIdx.x * kDefChunk;
  if (ls >= 0)
    for (int c = c0 + threadIdx.x; c < min(c0 + kDefChunk, cells); c += kDefThreads)
      cnt += is_light(code, base, c, ls);
  int v = cnt;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int q = 0; q < kDefThreads / 64; ++q) s += sh[q];
    counts[(size_t)b * nblk + blockIdx.x] = s;
  }
}

// the light cells in cell order (a problem with more than lcap of them: not written)
__global__ void __launch_bounds__(kDefThreads)
    k_light_write(const uint8_t* __restrict__ code, int cells, const int* __restrict__ light,
                  const int* __restrict__ offs, const int* __restrict__ total, int nblk,
                  int* __restrict__ list, int lcap) {
  const int b = blockIdx.y;
  const int ls = light[b];
  if (ls < 0 || total[b] > lcap) return;
  const size_t base = (size_t)b * cells;
  __shared__ int sh[kDefThreads / 64];
  int rank0 = offs[(size_t)b * nblk + blockIdx.x];
  const int c0 = blockIdx.x * kDefChunk;
  for (int s0 = c0; s0 < min(c0 + kDefChunk, cells); s0 += kDefThreads) {
    const int c = s0 + threadIdx.x;
    const bool hit = c < cells && is_light(code, base, c, ls);
    int tot = 0;
    const int r = block_rank(hit, tot, sh);
    if (hit) list[(size_t)b * lcap + rank0 + r] = c;
    rank0 += tot;
  }
}

// roots (cells whose label is their own index): per-block counts over chunks of the list
__global__ void __launch_bounds__(kDefThreads)
    k_root_count(const int* __restrict__ lab, int cells, const int* __restrict__ list,
                 const int* __restrict__ lcount, int lcap, int* __restrict__ counts, int nblk) {
  const int b = blockIdx.y;
  const int* L = lab + (size_t)b * cells;
  const int* Lst = list + (size_t)b * lcap;
  const int cnt_l = lcount[b];
  __shared__ int sh[kDefThreads / 64];
  int cnt = 0;
  const int q0 = blockIdx.x * kDefChunk;
  for (int q = q0 + threadIdx.x; q < min(q0 + kDefChunk, cnt_l); q += kDefThreads) {
    const int c = Lst[q];
    cnt += L[c] == c;
  }
  int v = cnt;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int q = 0; q < kDefThreads / 64; ++q) s += sh[q];
    counts[(size_t)b * nblk + blockIdx.x] = s;
  }
}

// the first kDefMax roots of each problem (in cell order) are marked -(rank + 2)
__global__ void __launch_bounds__(kDefThreads)
    k_root_mark(int* __restrict__ lab, int cells, const int* __restrict__ list,
                const int* __restrict__ lcount, int lcap, const int* __restrict__ offs, int nblk) {
  const int b = blockIdx.y;
  int* L = lab + (size_t)b * cells;
  const int* Lst = list + (size_t)b * lcap;
  const int cnt_l = lcount[b];
  __shared__ int sh[kDefThreads / 64];
  int base_rank = offs[(size_t)b * nblk + blockIdx.x];
  const int q0 = blockIdx.x * kDefChunk;
  for (int s0 = q0; s0 < min(q0 + kDefChunk, cnt_l); s0 += kDefThreads) {
    const int q = s0 + threadIdx.x;
    const int c = q < cnt_l ? Lst[q] : 0;
    const bool hit = q < cnt_l && L[c] == c;
    int total = 0;
    const int r = block_rank(hit, total, sh);
    if (hit && base_rank + r < kDefMax) L[c] = -(base_rank + r + 2);
    base_rank += total;
    if (base_rank >= kDefMax) break;   // uniform: the block's later roots are not kept
  }
}

__global__ void k_u8_fill(uint8_t* __restrict__ v, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    v[i] = 0;
}

// region id of every light cell (the other cells keep the 0 of the fill)
__global__ void k_region_ids(const int* __restrict__ lab, int cells, const int* __restrict__ list,
                             const int* __restrict__ lcount, int lcap, uint8_t* __restrict__ out) {
  const int b = blockIdx.y;
  const size_t base = (size_t)b * cells;
  const int* L = lab + base;
  const int* Lst = list + (size_t)b * lcap;
  const int cnt = lcount[b];
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
    const int c = Lst[q];
    const int l = L[c];
    int id = 0;
    if (l <= -2) id = -l - 1;
    else {
      const int r = L[l];
      if (r <= -2) id = -r - 1;
    }
    out[base + c] = (uint8_t)id;
  }
}

// ---- the band: cells where some A z_j is nonzero ------------------------------------
// Pairs of a cell c (region id lc, face coefficients w over h^2): (lc, -sum of w over the
// faces to cells not in lc) when lc != 0, and for every other region j next to it
// (j, sum of w over the faces to cells of j).  Returns the number of pairs (>= 1: a band
// cell), or kDefPairs + 1 if they do not fit.
__device__ inline int band_pairs(const Faces<double>& F, const uint8_t* __restrict__ lab, int b,
                                 size_t base, int c, int n, double inv_h2, uint8_t* pl,
                                 double* pv) {
  int i, j, k;
  ijk(c, n, i, j, k);
  const size_t nn = (size_t)n * n;
  const unsigned cd = F.code[base + c];
  const double ir = F.inv_rho[2 * b + ((cd >> 6) & 1)];
  double w[6];
  coded_faces_at(F.bx + base + c, F.by + base + c, F.bz + base + c, cd, i, j, k, n, nn, ir, w);
  const int lc = lab[base + c];
  int nbl[6];
  nbl[0] = i > 0 ? lab[base + c - 1] : lc;
  nbl[1] = i < n - 1 ? lab[base + c + 1] : lc;
  nbl[2] = j > 0 ? lab[base + c - n] : lc;
  nbl[3] = j < n - 1 ? lab[base + c + n] : lc;
  nbl[4] = k > 0 ? lab[base + c - nn] : lc;
  nbl[5] = k < n - 1 ? lab[base + c + nn] : lc;
  int np = 0;
  double own = 0.0;
  bool any = false;
  for (int f = 0; f < 6; ++f)
    if (nbl[f] != lc) {
      any = true;
      if (lc != 0) own -= w[f] * inv_h2;
    }
  if (!any) return 0;
  if (lc != 0) {
    pl[np] = (uint8_t)lc;
    pv[np] = own;
    ++np;
  }
  for (int f = 0; f < 6; ++f) {
    const int l = nbl[f];
    if (l == 0 || l == lc) continue;
    int q = (lc != 0) ? 1 : 0;
    while (q < np && pl[q] != l) ++q;
    if (q == np) {
      if (np == kDefPairs) return kDefPairs + 1;
      pl[np] = (uint8_t)l;
      pv[np] = 0.0;
      ++np;
    }
    pv[q] += w[f] * inv_h2;
  }
  return np;
}

// The band marked from the light-cell list: a cell of region l with a face neighbour of
// another label marks itself and that neighbour (a cell is in the band exactly when
// band_pairs finds a neighbour of another label, and one of the two is in a region).
// mask: a byte per cell, zero on entry.
__global__ void k_band_mark(const uint8_t* __restrict__ lab, int n, const int* __restrict__ list,
                            const int* __restrict__ lcount, int lcap, const int* __restrict__ dk,
                            uint8_t* __restrict__ mask) {
  const int b = blockIdx.y;
  if (dk[b] <= 0) return;
  const int cells = n * n * n;
  const size_t base = (size_t)b * cells;
  const int nn = n * n;
  const int* Lst = list + (size_t)b * lcap;
  const int cnt = lcount[b];
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
    const int c = Lst[q];
    const int l = lab[base + c];
    if (l == 0) continue;
    int i, j, k;
    ijk(c, n, i, j, k);
    const int nb[6] = {c - 1, c + 1, c - n, c + n, c - nn, c + nn};
    const bool in[6] = {i > 0, i < n - 1, j > 0, j < n - 1, k > 0, k < n - 1};
    bool edge = false;
    for (int f = 0; f < 6; ++f)
      if (in[f] && lab[base + nb[f]] != l) {
        mask[base + nb[f]] = 1;
        edge = true;
      }
    if (edge) mask[base + c] = 1;
  }
}

__global__ void __launch_bounds__(kDefThreads)
    k_band_count(const uint8_t* __restrict__ mask, int n, const int* __restrict__ dk,
                 int* __restrict__ counts, int nblk) {
  const int b = blockIdx.y;
  const int cells = n * n * n;
  const size_t base = (size_t)b * cells;
  __shared__ int sh[kDefThreads / 64];
  int cnt = 0;
  if (dk[b] > 0) {
    const int c0 = blockIdx.x * kDefChunk;
    for (int c = c0 + threadIdx.x; c < min(c0 + kDefChunk, cells); c += kDefThreads)
      cnt += mask[base + c] != 0;
  }
  int v = cnt;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int q = 0; q < kDefThreads / 64; ++q) s += sh[q];
    counts[(size_t)b * nblk + blockIdx.x] = s;
  }
}

// Writes the band cells in cell order.  A problem whose band does not fit its capacity,
// or has a cell with more than kDefPairs regions around it, gets overflow[b] = 1.
__global__ void __launch_bounds__(kDefThreads)
    k_band_write(Faces<double> F, const uint8_t* __restrict__ lab, const uint8_t* __restrict__ mask,
                 int n, const int* __restrict__ dk, const int* __restrict__ offs, int nblk, Defl D,
                 int* __restrict__ overflow) {
  const int b = blockIdx.y;
  if (dk[b] <= 0) return;
  const int cells = n * n * n;
  const size_t base = (size_t)b * cells;
  const double inv_h2 = (double)n * (double)n;
  __shared__ int sh[kDefThreads / 64];
  int rank0 = offs[(size_t)b * nblk + blockIdx.x];
  const int c0 = blockIdx.x * kDefChunk;
  for (int s0 = c0; s0 < min(c0 + kDefChunk, cells); s0 += kDefThreads) {
    const int c = s0 + threadIdx.x;
    uint8_t pl[kDefPairs] = {0, 0, 0, 0};
    double pv[kDefPairs] = {0.0, 0.0, 0.0, 0.0};
    const int np =
        c < cells && mask[base + c] ? band_pairs(F, lab, b, base, c, n, inv_h2, pl, pv) : 0;
    int total = 0;
    const int r = block_rank(np > 0, total, sh);
    if (np > 0) {
      const int q = rank0 + r;
      if (np > kDefPairs || q >= D.cap) {
        overflow[b] = 1;
      } else {
        const size_t e = (size_t)b * D.cap + q;
        D.bcell[e] = c;
        // the first pair is the cell's own region when it has one; byte 0 = 0 otherwise
        const int lc = lab[base + c];
        uint32_t packed = 0;
        double vals[kDefPairs] = {0.0, 0.0, 0.0, 0.0};
        int slot = 1;
        for (int t = 0; t < np; ++t) {
          if (lc != 0 && pl[t] == lc) {
            packed |= (uint32_t)pl[t];
            vals[0] = pv[t];
          } else {
            packed |= (uint32_t)pl[t] << (8 * slot);
            vals[slot] = pv[t];
            ++slot;
          }
        }
        D.blab[e] = packed;
        for (int t = 0; t < kDefPairs; ++t) D.bval[e * kDefPairs + t] = vals[t];
      }
    }
    rank0 += total;
  }
}

// E[i][j] = z_i^T A z_j: the pairs of the band cells of region i.  Block (i, b); per-thread
// sums in LDS, added in a fixed order.
__global__ void __launch_bounds__(kDefThreads)
    k_defl_e(Defl D, double* __restrict__ E) {
  const int b = blockIdx.y, i = blockIdx.x + 1;
  const int k = D.k[b];
  __shared__ double acc[kDefMax][kDefThreads];
  for (int j = 0; j < kDefMax; ++j) acc[j][threadIdx.x] = 0.0;
  if (i <= k) {
    const int cnt = D.bcount[b];
    const size_t e0 = (size_t)b * D.cap;
    for (int q = threadIdx.x; q < cnt; q += kDefThreads) {
      const uint32_t pk = D.blab[e0 + q];
      if ((int)(pk & 255u) != i) continue;
      for (int t = 0; t < kDefPairs; ++t) {
        const int j = (pk >> (8 * t)) & 255u;
        if (j) acc[j - 1][threadIdx.x] += D.bval[(e0 + q) * kDefPairs + t];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < kDefMax) {
    double s = 0.0;
    for (int t = 0; t < kDefThreads; ++t) s += acc[threadIdx.x][t];
    E[((size_t)b * kDefMax + (i - 1)) * kDefMax + threadIdx.x] = i <= k ? s : 0.0;
  }
}

// E^{-1} by Gauss-Jordan on -E (symmetric positive definite); one block per problem.  A
// pivot that is not clearly positive switches the problem's deflation off.
__global__ void __launch_bounds__(kDefMax * kDefMax)
    k_defl_inverse(const double* __restrict__ E, Defl D, int* __restrict__ overflow) {
  const int b = blockIdx.x;
  const int k = D.k[b];
  __shared__ double M[kDefMax][2 * kDefMax];
  __shared__ int bad;
  const int r = threadIdx.x / kDefMax, c = threadIdx.x % kDefMax;
  if (threadIdx.x == 0) bad = 0;
  M[r][c] = r < k && c < k ? -E[((size_t)b * kDefMax + r) * kDefMax + c] : 0.0;
  M[r][kDefMax + c] = r == c ? 1.0 : 0.0;
  __syncthreads();
  double scale = 0.0;
  for (int q = 0; q < k; ++q) scale = fmax(scale, fabs(-E[((size_t)b * kDefMax + q) * kDefMax + q]));
  for (int p = 0; p < k; ++p) {
    const double piv = M[p][p];
    __syncthreads();
    if (!(piv > 1e-13 * scale)) {
      if (threadIdx.x == 0) bad = 1;
      break;
    }
    const double f = M[r][p] / piv;
    double a0 = M[r][c], a1 = M[r][kDefMax + c];
    const double p0 = M[p][c] / piv, p1 = M[p][kDefMax + c] / piv;
    __syncthreads();
    if (r == p) {
      a0 = p0;
      a1 = p1;
    } else {
      a0 -= f * M[p][c];
      a1 -= f * M[p][kDefMax + c];
    }
    __syncthreads();
    M[r][c] = a0;
    M[r][kDefMax + c] = a1;
    __syncthreads();
  }
  __syncthreads();
  // E^{-1} = -(-E)^{-1}
  D.einv[((size_t)b * kDefMax + r) * kDefMax + c] = r < k && c < k ? -M[r][kDefMax + c] : 0.0;
  if (threadIdx.x == 0 && bad) overflow[b] = 1;
}

__global__ void k_defl_off(Defl D, const int* __restrict__ overflow, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B && overflow[b]) {
    D.k[b] = 0;
    D.bcount[b] = 0;
  }
}

// ---- per-solve and per-iteration pieces ---------------------------------------------
// Sums of v over each region (over the light cells): per-block partials part[b][blk][j]
// (thread sums in LDS, added in a fixed order)
template <typename T>
__global__ void __launch_bounds__(kDefThreads)
    k_region_sums(const T* __restrict__ v, const uint8_t* __restrict__ lab, int cells, Defl D,
                  const int* __restrict__ active) {
  const int b = blockIdx.y;
  const int k = D.k[b];
  if (k <= 0 || (active && !active[b])) return;
  __shared__ double acc[kDefMax][kDefThreads];
  for (int j = 0; j < k; ++j) acc[j][threadIdx.x] = 0.0;
  const size_t base = (size_t)b * cells;
  const int* Lst = D.light + (size_t)b * D.lcap;
  const int cnt = D.lcount[b];
  for (int q = blockIdx.x * kDefThreads + threadIdx.x; q < cnt; q += gridDim.x * kDefThreads) {
    const int c = Lst[q];
    const int l = lab[base + c];
    if (l) acc[l - 1][threadIdx.x] += (double)v[base + c];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = w; j < k; j += kDefThreads / 64) {
    double s = ((acc[j][lane] + acc[j][lane + 64]) + (acc[j][lane + 128] + acc[j][lane + 192]));
    s = wave_sum(s);
    if (lane == 0) D.part[((size_t)b * D.pcap + blockIdx.x) * kDefMax + j] = s;
  }
}

// (A Z)^T v over the band: per-block partials part[b][blk][j]
template <typename T>
__global__ void __launch_bounds__(kDefThreads)
    k_band_sums(const T* __restrict__ v, int cells, Defl D, Sel sel) {
  const int b = sel_problem(sel, blockIdx.y);
  if (b < 0) return;
  const int k = D.k[b];
  if (k <= 0) return;
  __shared__ double acc[kDefMax][kDefThreads];
  for (int j = 0; j < k; ++j) acc[j][threadIdx.x] = 0.0;
  const int cnt = D.bcount[b];
  const int per = (cnt + kDefBandBlocks - 1) / kDefBandBlocks;
  const int q0 = blockIdx.x * per, q1 = min(q0 + per, cnt);
  const size_t e0 = (size_t)b * D.cap;
  const size_t base = (size_t)b * cells;
  for (int q = q0 + threadIdx.x; q < q1; q += kDefThreads) {
    const uint32_t pk = D.blab[e0 + q];
    const double x = (double)v[base + D.bcell[e0 + q]];
    for (int t = 0; t < kDefPairs; ++t) {
      const int j = (pk >> (8 * t)) & 255u;
      if (j) acc[j - 1][threadIdx.x] += D.bval[(e0 + q) * kDefPairs + t] * x;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = w; j < k; j += kDefThreads / 64) {
    double s = ((acc[j][lane] + acc[j][lane + 64]) + (acc[j][lane + 128] + acc[j][lane + 192]));
    s = wave_sum(s);
    if (lane == 0) D.part[((size_t)b * D.pcap + blockIdx.x) * kDefMax + j] = s;
  }
}

// Totals of the regions over nblk per-block partials, by the block's first wave: lane l
// adds the partials l, l + 64, ... and the wave sums them in a fixed order (deterministic;
// the partials of a region load in parallel instead of one chain).  out[j] for j < k is
// valid after the caller's barrier.
__device__ inline void region_totals(const Defl& D, int b, int nblk, int k, double* out) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  const double* P = D.part + (size_t)b * D.pcap * kDefMax;
  for (int j = 0; j < k; ++j) {
    double t = 0.0;
    for (int q = lane; q < nblk; q += 64) t += P[(size_t)q * kDefMax + j];
    t = wave_sum(t);
    if (lane == 0) out[j] = t;
  }
}

// zb = Z^T b from k_region_sums partials
__global__ void __launch_bounds__(64) k_defl_zb(Defl D, int nblk, const int* __restrict__ active) {
  const int b = blockIdx.x;
  const int k = D.k[b];
  if (k <= 0 || (active && !active[b])) return;
  __shared__ double t[kDefMax];
  region_totals(D, b, nblk, k, t);
  __syncthreads();
  if (threadIdx.x < k) D.zb[(size_t)b * kDefMax + threadIdx.x] = t[threadIdx.x];
}

// coef = E^{-1} (zb - s), s from k_band_sums partials (mode 0: s = 0; mode 1: zb - s;
// mode 2: -s, i.e. zb = 0)
__global__ void __launch_bounds__(64) k_defl_coef(Defl D, int mode, const int* __restrict__ active) {
  const int b = blockIdx.x;
  const int k = D.k[b];
  if (k <= 0 || (active && !active[b])) return;
  __shared__ double s[kDefMax];
  if (mode) region_totals(D, b, kDefBandBlocks, k, s);
  else
    for (int j = threadIdx.x; j < k; j += blockDim.x) s[j] = 0.0;
  __syncthreads();
  if (threadIdx.x < k)
    s[threadIdx.x] = (mode == 2 ? 0.0 : D.zb[(size_t)b * kDefMax + threadIdx.x]) - s[threadIdx.x];
  __syncthreads();
  if (threadIdx.x < k) {
    const double* Ei = D.einv + ((size_t)b * kDefMax + threadIdx.x) * kDefMax;
    double a = 0.0;
    for (int j = 0; j < k; ++j) a += Ei[j] * s[j];
    D.coef[(size_t)b * kDefMax + threadIdx.x] = a;
  }
}

// r += g (A Z coef) on the band, g = scal[slot] of the problem or -1 (slot < 0); the
// change of ||r||^2 goes to the partials after the producer's (offset off).  store = 0:
// only the change of ||r||^2, r left as it is.
template <typename T>
__global__ void __launch_bounds__(kDefThreads)
    k_band_fix(T* __restrict__ r, int cells, Defl D, Ctl ctl, int slot, int off,
               Sel sel, int store = 1) {
  const int b = sel_problem(sel, blockIdx.y);
  if (b < 0) return;
  const int k = D.k[b];
  double delta = 0.0;
  if (k > 0) {
    const double g = slot >= 0 ? ctl.scal[(size_t)b * kSlots + slot] : -1.0;
    const double* a = D.coef + (size_t)b * kDefMax;
    const int cnt = D.bcount[b];
    const int per = (cnt + kDefBandBlocks - 1) / kDefBandBlocks;
    const int q0 = blockIdx.x * per, q1 = min(q0 + per, cnt);
    const size_t e0 = (size_t)b * D.cap;
    const size_t base = (size_t)b * cells;
    for (int q = q0 + threadIdx.x; q < q1; q += kDefThreads) {
      const uint32_t pk = D.blab[e0 + q];
      double u = 0.0;
      for (int t = 0; t < kDefPairs; ++t) {
        const int j = (pk >> (8 * t)) & 255u;
        if (j) u += a[j - 1] * D.bval[(e0 + q) * kDefPairs + t];
      }
      const size_t c = base + D.bcell[e0 + q];
      const T old = r[c];
      const T nv = (T)((double)old + g * u);
      if (store) r[c] = nv;
      delta += (double)nv * (double)nv - (double)old * (double)old;
    }
  }
  __shared__ double sh[16];
  const double s = block_sum(delta, sh);
  if (threadIdx.x == 0) ctl.partials[(size_t)b * ctl.pstride + off + blockIdx.x] = s;
}

// x += coef of its region on every cell of a region (over the light cells).  proj: the
// block first computes coef = -E^{-1} s itself from the band partials of x (the
// projection x <- P^T x), else coef is read as it is.
template <typename T>
__global__ void __launch_bounds__(kDefThreads)
    k_region_add(T* __restrict__ x, const uint8_t* __restrict__ lab, int cells, Defl D, int proj,
                 Sel sel) {
  const int b = sel_problem(sel, blockIdx.y);
  if (b < 0) return;
  const int k = D.k[b];
  if (k <= 0) return;
  __shared__ double a[kDefMax];
  __shared__ double s[kDefMax];
  if (proj) {
    region_totals(D, b, kDefBandBlocks, k, s);
    __syncthreads();
    if (threadIdx.x < k) {
      const double* Ei = D.einv + ((size_t)b * kDefMax + threadIdx.x) * kDefMax;
      double t = 0.0;
      for (int j = 0; j < k; ++j) t += Ei[j] * s[j];
      a[threadIdx.x] = -t;
    }
  } else if (threadIdx.x < k) {
    a[threadIdx.x] = D.coef[(size_t)b * kDefMax + threadIdx.x];
  }
  __syncthreads();
  const size_t base = (size_t)b * cells;
  const int* Lst = D.light + (size_t)b * D.lcap;
  const int cnt = D.lcount[b];
  for (int q = blockIdx.x * kDefThreads + threadIdx.x; q < cnt; q += gridDim.x * kDefThreads) {
    const int c = Lst[q];
    const int l = lab[base + c];
    if (l) x[base + c] = (T)((double)x[base + c] + a[l - 1]);
  }
}

// The CG epilogue of p.q with deflation: p.(P q) = p.q - a.s with s = (A Z)^T p (the band
// partials) and a = E^{-1} s kept in coef; then alpha and the breakdown check as E_PQ.
__global__ void __launch_bounds__(1024) k_finish_pq_defl(Ctl ctl, int nparts, EpiArgs e, Defl D) {
  const int b = row_problem(ctl.list, blockIdx.x);
  if (b < 0 || (e.only_active && !ctl.active[b])) return;
  __shared__ double sh[16];
  __shared__ double s[kDefMax];
  const double* P = ctl.partials + (size_t)b * ctl.pstride;
  double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
  const int st = blockDim.x;
  int q = threadIdx.x;
  for (; q + 3 * st < nparts; q += 4 * st) {
    t0 += P[q];
    t1 += P[q + st];
    t2 += P[q + 2 * st];
    t3 += P[q + 3 * st];
  }
  for (; q < nparts; q += st) t0 += P[q];
  double tot = block_sum((t0 + t1) + (t2 + t3), sh);
  const int k = D.k[b];
  if (k > 0) {
    region_totals(D, b, kDefBandBlocks, k, s);
    __syncthreads();
    if (threadIdx.x == 0) {
      double as = 0.0;
      for (int i = 0; i < k; ++i) {
        const double* Ei = D.einv + ((size_t)b * kDefMax + i) * kDefMax;
        double a = 0.0;
        for (int j = 0; j < k; ++j) a += Ei[j] * s[j];
        D.coef[(size_t)b * kDefMax + i] = a;
        as += a * s[i];
      }
      tot -= as;
    }
  }
  if (threadIdx.x == 0) finish(ctl, b, tot, e);
}

}  // namespace mpp
