// Device kernels of the gfx950 pressure-projection library: operator build,
// stencil sweeps, grid transfers, coarsest solve and the CG vector updates with
// deterministic reductions.
//
// Layout: a problem's field is n^3 values, x fastest; batched fields are
// [B][n^3].  Cell kernels run on a (blocks-per-problem, B) grid of kBlock threads,
// each thread striding over the cells of its problem, so every block belongs to
// exactly one problem and reductions stay per problem.
#pragma once

#include "mpp_internal.h"

namespace mpp {

// Workgroup barrier that waits for LDS traffic only: global loads issued before it
// stay in flight (the compiler still waits for them before their values are used).
__device__ inline void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ------------------------------------------------------------------------------
// reductions: wave shuffles, one partial per block, last block finishes in a fixed
// order (no floating-point atomics: bitwise reproducible)
// ------------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over the block; the result is valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int q = 0; q < nw; ++q) s += sh[q];
  }
  __syncthreads();
  return s;
}

// Per-problem sums without atomics: every block of a producer kernel stores its
// partial sum; a separate one-block-per-problem kernel (k_finish) adds the partials
// in a fixed order and runs the epilogue, so results are bitwise reproducible.
__device__ inline void block_partial(double v, const Ctl& ctl, int b) {
  __shared__ double sh[16];
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) ctl.partials[(size_t)b * ctl.pstride + blockIdx.x] = s;
}

// What the last block does with a finished sum.
enum Epi {
  E_STORE_MEAN = 0,  // scal[slot] = total / cells
  E_MEAN,            // scal[S_MEAN] = total / cells
  E_BB,              // scal[S_BB] = total, scal[S_TOL2] = rtol^2 total
  E_START,           // scal[S_RR] = total; active = total > tol2 && status OK
  E_START_REL,       // as E_START with tol2 = rtol^2 total (a solve relative to this rhs)
  E_RZ,              // beta = total / rz (0 on the first iteration), rz = total
  E_PQ,              // alpha = rz / total; breakdown check
  E_RR_ITER,         // rr = total; ++iters; active = rr > tol2 && iters < max
};

struct EpiArgs {
  int kind;
  int only_active;   // skip problems whose active flag is 0 (their partials are stale)
  int slot;
  double rtol2;
  double inv_cells;
  int first;
  const int* gate;   // E_START_REL: problems whose gate is 0 stay inactive
  // E_START_REL of an inner solve in residual refinement: the outer solve's slots
  // and its target; the inner target is relaxed to what the outer step still needs
  const double* outer_scal;
  double outer_rtol;
  // E_START_REL of a deflated solve: the target is relative to scal[S_SUM] (the norm^2
  // of the residual before deflation) instead of the deflated residual's
  int rel_base;
};

__device__ inline void finish(const Ctl& ctl, int b, double tot, const EpiArgs& e) {
  double* s = ctl.scal + (size_t)b * kSlots;
  switch (e.kind) {
    case E_STORE_MEAN: s[e.slot] = tot * e.inv_cells; break;
    case E_MEAN: s[S_MEAN] = tot * e.inv_cells; break;
    case E_BB:
      s[S_BB] = tot;
      s[S_TOL2] = e.rtol2 * tot;
      break;
    case E_START_REL: {
      const double base = e.rel_base ? s[S_SUM] : tot;
      s[S_BB] = base;
      double rel2 = e.rtol2;
      if (e.outer_scal) {
        // the refinement step only has to bring ||r|| below outer_rtol ||b||: ask the
        // inner solve for that reduction with a factor 2 margin, never for less than
        // halving the residual, never for more than rtol2
        const double* os = e.outer_scal + (size_t)b * kSlots;
        const double need2 = 0.25 * e.outer_rtol * e.outer_rtol * os[S_BB] / os[S_RR];
        rel2 = fmin(0.25, fmax(rel2, need2));
      }
      s[S_TOL2] = rel2 * base;
    }
      [[fallthrough]];
    case E_START:
      s[S_RR] = tot;
      ctl.active[b] = (tot > s[S_TOL2] && ctl.status[b] == MPP_OK) ? 1 : 0;
      if (e.gate && !e.gate[b]) ctl.active[b] = 0;
      if (!(tot == tot)) { ctl.active[b] = 0; ctl.status[b] = MPP_EBREAKDOWN; }
      break;
    case E_RZ: {
      const double rz_old = s[S_RZ];
      s[S_BETA] = e.first ? 0.0 : tot / rz_old;
      s[S_RZ] = tot;
      // A is negative semidefinite and the V-cycle approximates its inverse, so
      // r.z < 0 for r != 0; anything else is a breakdown of the preconditioner
      if (!(tot < 0.0)) { ctl.active[b] = 0; ctl.status[b] = MPP_EBREAKDOWN; }
      break;
    }
    case E_PQ:
      s[S_PQ] = tot;
      s[S_ALPHA] = s[S_RZ] / tot;
      if (!(tot < 0.0)) { ctl.active[b] = 0; ctl.status[b] = MPP_EBREAKDOWN; }
      break;
    case E_RR_ITER: {
      s[S_RR] = tot;
      const int it = ctl.iters[b] + 1;
      ctl.iters[b] = it;
      if (!(tot == tot)) { ctl.active[b] = 0; ctl.status[b] = MPP_EBREAKDOWN; }
      else if (tot <= s[S_TOL2]) ctl.active[b] = 0;
      else if (it >= ctl.max_iter) { ctl.active[b] = 0; ctl.status[b] = MPP_ENOTCONVERGED; }
      break;
    }
  }
}

__global__ void __launch_bounds__(1024) k_finish(Ctl ctl, int nparts, EpiArgs e) {
  const int b = row_problem(ctl.list, blockIdx.x);
  if (b < 0 || (e.only_active && !ctl.active[b])) return;
  __shared__ double sh[16];
  const double* P = ctl.partials + (size_t)b * ctl.pstride;
  // four independent loads in flight per thread, fixed order of the sums
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
  const double tot = block_sum((t0 + t1) + (t2 + t3), sh);
  if (threadIdx.x == 0) finish(ctl, b, tot, e);
}

// ------------------------------------------------------------------------------
// cell indexing and faces
// ------------------------------------------------------------------------------
__device__ inline void ijk(int c, int n, int& i, int& j, int& k) {
  i = c % n;
  const int t = c / n;
  j = t % n;
  k = t / n;
}

// Coefficients of the six faces -x,+x,-y,+y,-z,+z of cell c (0 through walls).
template <typename T, bool FINE>
__device__ inline void cell_faces(const Faces<T>& F, int b, size_t base, int c, int i, int j,
                                  int k, int n, T w[6]) {
  const size_t nn = (size_t)n * n;
  if (FINE) {
    const unsigned cd = F.code[base + c];
    const T ir = F.inv_rho[2 * b + ((cd >> 6) & 1u)];
    w[0] = i > 0 ? ((cd & 1u) ? F.bx[base + c] : ir) : T(0);
    w[1] = i < n - 1 ? ((cd & 2u) ? F.bx[base + c + 1] : ir) : T(0);
    w[2] = j > 0 ? ((cd & 4u) ? F.by[base + c] : ir) : T(0);
    w[3] = j < n - 1 ? ((cd & 8u) ? F.by[base + c + n] : ir) : T(0);
    w[4] = k > 0 ? ((cd & 16u) ? F.bz[base + c] : ir) : T(0);
    w[5] = k < n - 1 ? ((cd & 32u) ? F.bz[base + c + nn] : ir) : T(0);
  } else {
    w[0] = i > 0 ? F.bx[base + c] : T(0);
    w[1] = i < n - 1 ? F.bx[base + c + 1] : T(0);
    w[2] = j > 0 ? F.by[base + c] : T(0);
    w[3] = j < n - 1 ? F.by[base + c + n] : T(0);
    w[4] = k > 0 ? F.bz[base + c] : T(0);
    w[5] = k < n - 1 ? F.bz[base + c + nn] : T(0);
  }
}

// ((A - sig I) x)_c = sum_f w_f (x_nb - x_c) / h^2 - sig x_c
template <typename T>
__device__ inline T stencil_at(const T w[6], const T* x, size_t base, int c, int i, int j, int k,
                               int n, T inv_h2, T sig) {
  const size_t nn = (size_t)n * n;
  const T xc = x[base + c];
  T s = T(0);
  if (i > 0) s += w[0] * (x[base + c - 1] - xc);
  if (i < n - 1) s += w[1] * (x[base + c + 1] - xc);
  if (j > 0) s += w[2] * (x[base + c - n] - xc);
  if (j < n - 1) s += w[3] * (x[base + c + n] - xc);
  if (k > 0) s += w[4] * (x[base + c - nn] - xc);
  if (k < n - 1) s += w[5] * (x[base + c + nn] - xc);
  return s * inv_h2 - sig * xc;
}

#define CELL_LOOP(cells)                                                     \
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < (int)(cells);      \
       c += gridDim.x * blockDim.x)

// ------------------------------------------------------------------------------
// operator build (FP64, no contraction so that the coefficients are the exactly
// rounded values of their defining expressions)
// ------------------------------------------------------------------------------
__device__ inline bool plus_side(double phi) { return phi > 0.0; }

__device__ inline double ghost_fluid_beta(double pa, double pb, double rn, double rp) {
#pragma clang fp contract(off)
  const double ra = plus_side(pa) ? rp : rn;
  const double rb = plus_side(pb) ? rp : rn;
  if (plus_side(pa) == plus_side(pb)) return 1.0 / ra;
  const double theta = fabs(pa) / (fabs(pa) + fabs(pb));
  return 1.0 / (theta * ra + (1.0 - theta) * rb);
}

__global__ void k_params(const double* rho, double* ir64, float* ir32, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double a = 1.0 / rho[3 * b + 0], c = 1.0 / rho[3 * b + 1];
  ir64[2 * b + 0] = a;
  ir64[2 * b + 1] = c;
  ir32[2 * b + 0] = (float)a;
  ir32[2 * b + 1] = (float)c;
}

// Blocks are handed to the 8 XCDs round-robin; give each XCD a contiguous run of
// tiles so that neighbouring tiles (which share halo rows) sit in the same L2.
// The grid has 8 * ceil(ntiles / 8) blocks; the surplus ones get -1.
__device__ inline int xcd_tile(int bid, int ntiles) {
  const int per = (ntiles + 7) / 8;
  const int t = (bid & 7) * per + (bid >> 3);
  return t < ntiles ? t : -1;
}

// Face coefficients (low face of each cell), FP32 copies and the finest-level code,
// marching columns: a block owns a 64 x 4 column of cells and a chunk of kz planes, holding phi of planes k - 1, k, k + 1 of its own column
// in registers; in-plane neighbours come through the caches.
__global__ void __launch_bounds__(256)
    k_faces(const double* __restrict__ phi, const double* __restrict__ rho, int n, int ntx, int nty,
            int kz, int ntiles, uint8_t* __restrict__ code, double* __restrict__ bx,
            double* __restrict__ by, double* __restrict__ bz, float* __restrict__ fx,
            float* __restrict__ fy, float* __restrict__ fz, int* __restrict__ bad) {
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int b = blockIdx.y;
  const int ti = tile % ntx, tj = (tile / ntx) % nty, tk = tile / (ntx * nty);
  const int i = ti * 64 + (int)(threadIdx.x % 64), j = tj * 4 + (int)(threadIdx.x / 64);
  if (i >= n || j >= n) return;
  const int k0 = tk * kz, k1 = min(k0 + kz, n);
  const size_t nn = (size_t)n * n;
  const size_t col = (size_t)b * nn * n + (size_t)i + (size_t)n * j;
  const double rn = rho[3 * b + 0], rp = rho[3 * b + 1];
  double pm = k0 > 0 ? phi[col + (size_t)(k0 - 1) * nn] : 0.0;
  double pc = phi[col + (size_t)k0 * nn];
  for (int k = k0; k < k1; ++k) {
    const size_t q = col + (size_t)k * nn;
    const double pp = k < n - 1 ? phi[q + nn] : 0.0;
    const double pw = i > 0 ? phi[q - 1] : 0.0, pe = i < n - 1 ? phi[q + 1] : 0.0;
    const double ps = j > 0 ? phi[q - n] : 0.0, pn = j < n - 1 ? phi[q + n] : 0.0;
    if (!isfinite(pc)) atomicOr(bad, 1);
    const bool s = plus_side(pc);
    const double vx = i > 0 ? ghost_fluid_beta(pw, pc, rn, rp) : 0.0;
    const double vy = j > 0 ? ghost_fluid_beta(ps, pc, rn, rp) : 0.0;
    const double vz = k > 0 ? ghost_fluid_beta(pm, pc, rn, rp) : 0.0;
    bx[q] = vx;
    by[q] = vy;
    bz[q] = vz;
    fx[q] = (float)vx;
    fy[q] = (float)vy;
    fz[q] = (float)vz;
    unsigned cd = s ? 64u : 0u;
    if (i > 0 && plus_side(pw) != s) cd |= 1u;
    if (i < n - 1 && plus_side(pe) != s) cd |= 2u;
    if (j > 0 && plus_side(ps) != s) cd |= 4u;
    if (j < n - 1 && plus_side(pn) != s) cd |= 8u;
    if (k > 0 && plus_side(pm) != s) cd |= 16u;
    if (k < n - 1 && plus_side(pp) != s) cd |= 32u;
    code[q] = (uint8_t)cd;
    pm = pc;
    pc = pp;
  }
}

// phi with linear extrapolation beyond the walls, axis by axis (x, then y, then z).
__device__ inline double phi_ld(const double* phi, size_t base, int n, int i, int j, int k) {
  return phi[base + (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k)];
}
__device__ inline double phi_ez(const double* phi, size_t base, int n, int i, int j, int k) {
  if (k < 0) return 2.0 * phi_ld(phi, base, n, i, j, 0) - phi_ld(phi, base, n, i, j, 1);
  if (k > n - 1) return 2.0 * phi_ld(phi, base, n, i, j, n - 1) - phi_ld(phi, base, n, i, j, n - 2);
  return phi_ld(phi, base, n, i, j, k);
}
__device__ inline double phi_ey(const double* phi, size_t base, int n, int i, int j, int k) {
  if (j < 0) return 2.0 * phi_ez(phi, base, n, i, 0, k) - phi_ez(phi, base, n, i, 1, k);
  if (j > n - 1) return 2.0 * phi_ez(phi, base, n, i, n - 1, k) - phi_ez(phi, base, n, i, n - 2, k);
  return phi_ez(phi, base, n, i, j, k);
}
__device__ inline double phi_ex(const double* phi, size_t base, int n, int i, int j, int k) {
  if (i < 0) return 2.0 * phi_ey(phi, base, n, 0, j, k) - phi_ey(phi, base, n, 1, j, k);
  if (i > n - 1) return 2.0 * phi_ey(phi, base, n, n - 1, j, k) - phi_ey(phi, base, n, n - 2, j, k);
  return phi_ey(phi, base, n, i, j, k);
}

// Mean curvature -div(grad phi/|grad phi|) from central differences at interface
// cells (cells with a crossed face), 0 elsewhere.
__global__ void k_curvature(const double* __restrict__ phi, const uint8_t* __restrict__ code,
                            int n, int cells, double* __restrict__ kappa) {
#pragma clang fp contract(off)
  const int b = blockIdx.y;
  const size_t base = (size_t)b * cells;
  const double h = 1.0 / n;
  CELL_LOOP(cells) {
    if ((code[base + c] & 63u) == 0) {
      kappa[base + c] = 0.0;
      continue;
    }
    int i, j, k;
    ijk(c, n, i, j, k);
#define P(a, bb, cc) phi_ex(phi, base, n, i + (a), j + (bb), k + (cc))
    const double p0 = P(0, 0, 0);
    const double px = (P(1, 0, 0) - P(-1, 0, 0)) / (2.0 * h);
    const double py = (P(0, 1, 0) - P(0, -1, 0)) / (2.0 * h);
    const double pz = (P(0, 0, 1) - P(0, 0, -1)) / (2.0 * h);
    const double pxx = (P(1, 0, 0) - 2.0 * p0 + P(-1, 0, 0)) / (h * h);
    const double pyy = (P(0, 1, 0) - 2.0 * p0 + P(0, -1, 0)) / (h * h);
    const double pzz = (P(0, 0, 1) - 2.0 * p0 + P(0, 0, -1)) / (h * h);
    const double pxy = (P(1, 1, 0) - P(1, -1, 0) - P(-1, 1, 0) + P(-1, -1, 0)) / (4.0 * h * h);
    const double pxz = (P(1, 0, 1) - P(1, 0, -1) - P(-1, 0, 1) + P(-1, 0, -1)) / (4.0 * h * h);
    const double pyz = (P(0, 1, 1) - P(0, 1, -1) - P(0, -1, 1) + P(0, -1, -1)) / (4.0 * h * h);
#undef P
    const double g2 = px * px + py * py + pz * pz;
    const double g = sqrt(g2);
    double kap = 0.0;
    if (!(g < 1e-12)) {
      const double num = (pyy + pzz) * px * px + (pxx + pzz) * py * py + (pxx + pyy) * pz * pz -
                         2.0 * px * py * pxy - 2.0 * px * pz * pxz - 2.0 * py * pz * pyz;
      kap = -num / (g2 * g);
    }
    kappa[base + c] = kap;
  }
}

// One crossed face between a (low) and b (high): the term s_a beta^ J / h^2 that
// the face adds to cell a (and subtracts from cell b).
__device__ inline double jump_face_term(double pa, double pb, double ka, double kb, double rn,
                                        double rp, double sigma, double inv_h2) {
#pragma clang fp contract(off)
  const double theta = fabs(pa) / (fabs(pa) + fabs(pb));
  const double J = sigma * ((1.0 - theta) * ka + theta * kb);
  const double bh = ghost_fluid_beta(pa, pb, rn, rp);
  const double s_a = plus_side(pa) ? -1.0 : 1.0;
  return s_a * bh * J * inv_h2;
}

// jterm_c = sum over the crossed faces of c of the face term (+ for the low cell,
// - for the high cell), in the order -x, +x, -y, +y, -z, +z.
__global__ void k_jump(const double* __restrict__ phi, const uint8_t* __restrict__ code,
                       const double* __restrict__ kappa, const double* __restrict__ rho, int n,
                       int cells, double* __restrict__ jterm) {
#pragma clang fp contract(off)
  const int b = blockIdx.y;
  const size_t base = (size_t)b * cells;
  const double rn = rho[3 * b + 0], rp = rho[3 * b + 1], sg = rho[3 * b + 2];
  const double inv_h2 = (double)n * (double)n;
  const size_t nn = (size_t)n * n;
  CELL_LOOP(cells) {
    const unsigned cd = code[base + c];
    double acc = 0.0;
    if (cd & 63u) {
      const size_t cc = base + c;
      const double pc = phi[cc], kc = kappa[cc];
      const size_t off[3] = {1, (size_t)n, nn};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (cd & (1u << (2 * d))) {
          const size_t a = cc - off[d];
          acc -= jump_face_term(phi[a], pc, kappa[a], kc, rn, rp, sg, inv_h2);
        }
        if (cd & (2u << (2 * d))) {
          const size_t bq = cc + off[d];
          acc += jump_face_term(pc, phi[bq], kc, kappa[bq], rn, rp, sg, inv_h2);
        }
      }
    }
    jterm[base + c] = acc;
  }
}

// Coarse face = mean of the 2x2 fine faces on the same plane (FP64 and FP32 copy).
__global__ void k_coarsen_faces(const double* __restrict__ fx, const double* __restrict__ fy,
                                const double* __restrict__ fz, int nf, double* __restrict__ cx,
                                double* __restrict__ cy, double* __restrict__ cz,
                                float* __restrict__ gx, float* __restrict__ gy,
                                float* __restrict__ gz) {
#pragma clang fp contract(off)
  const int b = blockIdx.y;
  const int nc = nf / 2;
  const int cells_c = nc * nc * nc;
  const size_t bf = (size_t)b * nf * nf * nf, bc = (size_t)b * cells_c;
  CELL_LOOP(cells_c) {
    int I, J, K;
    ijk(c, nc, I, J, K);
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int e = 0; e < 2; ++e) {
        sx += fx[bf + (size_t)(2 * I) + (size_t)nf * ((size_t)(2 * J + a) + (size_t)nf * (2 * K + e))];
        sy += fy[bf + (size_t)(2 * I + a) + (size_t)nf * ((size_t)(2 * J) + (size_t)nf * (2 * K + e))];
        sz += fz[bf + (size_t)(2 * I + a) + (size_t)nf * ((size_t)(2 * J + e) + (size_t)nf * (2 * K))];
      }
    const double vx = 0.25 * sx, vy = 0.25 * sy, vz = 0.25 * sz;
    cx[bc + c] = vx;
    cy[bc + c] = vy;
    cz[bc + c] = vz;
    gx[bc + c] = (float)vx;
    gy[bc + c] = (float)vy;
    gz[bc + c] = (float)vz;
  }
}

// Coarsest level: dense M = -A + 11^T/m (sig == 0: the singular pressure operator,
// regularised on the constants) or M = -A + sig I (a shifted operator, already definite),
// and its inverse.  One block per problem; up to 64 cells by Gauss-Jordan elimination in
// LDS, above that by a Cholesky factor M = L L^T in the [B][m][m] scratch `work` and
// M^{-1} column by column.
__global__ void __launch_bounds__(1024) k_coarse_factor(const double* __restrict__ cx, const double* __restrict__ cy,
                                const double* __restrict__ cz, int n, double sig,
                                double* __restrict__ work, double* __restrict__ inv) {
  const int b = blockIdx.x;
  const int m = n * n * n;
  const size_t bm = (size_t)b * m * m, bc = (size_t)b * m;
  // small coarsest levels (the usual 4^3) are factored in LDS
  constexpr int kLdsM = 64;
  __shared__ double Ms[kLdsM * kLdsM], Xs[kLdsM * kLdsM];
  __shared__ double Ms2[kLdsM * kLdsM], Xs2[kLdsM * kLdsM];   // the other buffer of [M | I]
  const double* Xfin = Xs;   // LDS: the buffer holding M^{-1} at the end
  const bool lds = m <= kLdsM;
  double* M = lds ? Ms : work + bm;
  double* X = lds ? Xs : inv + bm;
  const double inv_h2 = (double)n * (double)n, jm = sig == 0.0 ? 1.0 / m : 0.0;
  for (size_t q = threadIdx.x; q < (size_t)m * m; q += blockDim.x) M[q] = jm;
  __syncthreads();
  for (int c = threadIdx.x; c < m; c += blockDim.x) {
    int i, j, k;
    ijk(c, n, i, j, k);
    const bool in[6] = {i > 0, i < n - 1, j > 0, j < n - 1, k > 0, k < n - 1};
    const int nb[6] = {c - 1, c + 1, c - n, c + n, c - n * n, c + n * n};
    const int fc[6] = {c, c + 1, c, c + n, c, c + n * n};
    const double* arr[6] = {cx, cx, cy, cy, cz, cz};
    double d = 0.0;
    for (int f = 0; f < 6; ++f)
      if (in[f]) {
        const double w = arr[f][bc + fc[f]];
        M[(size_t)c * m + nb[f]] -= w * inv_h2;
        d += w;
      }
    M[(size_t)c * m + c] += d * inv_h2 + sig;
  }
  __syncthreads();
  if (lds) {
    // Gauss-Jordan on [M | I] in LDS, every thread on every pivot (M is symmetric
    // positive definite: no pivoting needed).  Each pivot step reads one buffer of
    // [M | I] and writes the other, so one barrier per step separates them.
    for (int q = threadIdx.x; q < m * m; q += blockDim.x) X[q] = (q / m == q % m) ? 1.0 : 0.0;
    // thread t owns column t % (2m) of [M | I] and rows t / (2m), + rows_step, ...
    const int tw = 2 * m, col = threadIdx.x % tw, row0 = threadIdx.x / tw;
    const int rows_step = blockDim.x / tw;
    const bool has_col = (int)threadIdx.x < rows_step * tw;
    double *Ma = Ms, *Xa = Xs, *Mb = Ms2, *Xb = Xs2;
    __syncthreads();
    for (int k = 0; k < m; ++k) {
      const double pinv = 1.0 / Ma[(size_t)k * m + k];
      if (has_col) {
        const double* ca = col < m ? Ma + col : Xa + (col - m);   // this column, stride m
        double* cb = col < m ? Mb + col : Xb + (col - m);
        const double pk = ca[(size_t)k * m] * pinv;               // pivot row, scaled
        for (int i = row0; i < m; i += rows_step)
          cb[(size_t)i * m] = i == k ? pk : ca[(size_t)i * m] - Ma[(size_t)i * m + k] * pk;
      }
      __syncthreads();
      double* t = Ma;
      Ma = Mb;
      Mb = t;
      t = Xa;
      Xa = Xb;
      Xb = t;
    }
    Xfin = Xa;
  } else {
  // left-looking Cholesky, lower triangle of M
  __shared__ double piv;
  for (int j = 0; j < m; ++j) {
    if (threadIdx.x == 0) {
      double d = M[(size_t)j * m + j];
      for (int q = 0; q < j; ++q) d -= M[(size_t)j * m + q] * M[(size_t)j * m + q];
      piv = sqrt(d);
      M[(size_t)j * m + j] = piv;
    }
    __syncthreads();
    for (int r = j + 1 + threadIdx.x; r < m; r += blockDim.x) {
      double s = M[(size_t)r * m + j];
      for (int q = 0; q < j; ++q) s -= M[(size_t)r * m + q] * M[(size_t)j * m + q];
      M[(size_t)r * m + j] = s / piv;
    }
    __syncthreads();
  }
  // columns of the inverse: L y = e_col, L^T x = y.  Column col is kept at stride m
  // (X[r m + col]) so that the lanes of a wave touch consecutive words; M^{-1} is
  // symmetric, so this is also its row-major layout.
  for (int col = threadIdx.x; col < m; col += blockDim.x) {
    double* x = X + col;
    for (int r = 0; r < m; ++r) {
      double s = (r == col) ? 1.0 : 0.0;
      for (int q = 0; q < r; ++q) s -= M[(size_t)r * m + q] * x[(size_t)q * m];
      x[(size_t)r * m] = s / M[(size_t)r * m + r];
    }
    for (int r = m - 1; r >= 0; --r) {
      double s = x[(size_t)r * m];
      for (int q = r + 1; q < m; ++q) s -= M[(size_t)q * m + r] * x[(size_t)q * m];
      x[(size_t)r * m] = s / M[(size_t)r * m + r];
    }
  }
  }
  if (lds) {
    __syncthreads();
    for (int q = threadIdx.x; q < m * m; q += blockDim.x) inv[bm + q] = Xfin[q];
  }
}

// ------------------------------------------------------------------------------
// right-hand side
// ------------------------------------------------------------------------------
__global__ void k_rhs_sum(const double* __restrict__ f, const double* __restrict__ jterm,
                          double* __restrict__ b, int cells, Ctl ctl, EpiArgs e) {
  const int pb = blockIdx.y;
  const size_t base = (size_t)pb * cells;
  double acc = 0.0;
  CELL_LOOP(cells) {
    const double v = f[base + c] + jterm[base + c];
    b[base + c] = v;
    acc += v;
  }
  block_partial(acc, ctl, pb);
}

// v -= scal[S_MEAN]; optional sum of squares into an epilogue; v32 (optional): an FP32
// copy of the result
__global__ void k_sub_mean_sq(double* __restrict__ v, int cells, Ctl ctl, EpiArgs e, int slot,
                              int want_sq, float* __restrict__ v32 = nullptr) {
  const int pb = blockIdx.y;
  const size_t base = (size_t)pb * cells;
  const double mean = ctl.scal[(size_t)pb * kSlots + slot];
  double acc = 0.0;
  CELL_LOOP(cells) {
    const double x = v[base + c] - mean;
    v[base + c] = x;
    if (v32) v32[base + c] = (float)x;
    acc += x * x;
  }
  if (want_sq) block_partial(acc, ctl, pb);
}

// x = (double) x32
__global__ void k_widen(const float* __restrict__ x32, double* __restrict__ x, int cells) {
  const size_t base = (size_t)blockIdx.y * cells;
  CELL_LOOP(cells) x[base + c] = (double)x32[base + c];
}

template <typename T>
__global__ void k_sum(const T* __restrict__ v, int cells, Ctl ctl, EpiArgs e) {
  const int pb = blockIdx.y;
  const size_t base = (size_t)pb * cells;
  double acc = 0.0;
  CELL_LOOP(cells) acc += (double)v[base + c];
  block_partial(acc, ctl, pb);
}

// ------------------------------------------------------------------------------
// stencil kernels
// ------------------------------------------------------------------------------
// ------------------------------------------------------------------------------
// CG vector updates
// ------------------------------------------------------------------------------
template <typename T>
__global__ void k_dot(const T* __restrict__ a, const T* __restrict__ bv, int cells, Ctl ctl,
                      EpiArgs e, Sel sel) {
  const int pb = sel_problem(sel, blockIdx.y);
  if (pb < 0) return;
  const size_t base = (size_t)pb * cells;
  double acc = 0.0;
  CELL_LOOP(cells) acc += (double)a[base + c] * (double)bv[base + c];
  block_partial(acc, ctl, pb);
}

// The sum of p and p.b in one pass: per problem, the block partials of the sum at
// [0, gridDim.x) of its partials row and those of p.b right after them
__global__ void k_sum_dot(const double* __restrict__ p, const double* __restrict__ b, int cells,
                          Ctl ctl) {
  const int q = blockIdx.y;
  const size_t base = (size_t)q * cells;
  double s1 = 0.0, s2 = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += gridDim.x * blockDim.x) {
    const double v = p[base + c];
    s1 += v;
    s2 += v * b[base + c];
  }
  __shared__ double sh[16];
  const double t1 = block_sum(s1, sh);
  const double t2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    double* P = ctl.partials + (size_t)q * ctl.pstride;
    P[blockIdx.x] = t1;
    P[gridDim.x + blockIdx.x] = t2;
  }
}

// p = z + beta p   (first: p = z)
template <typename T>
__global__ void k_update_p(const T* __restrict__ z, T* __restrict__ p, int cells, Ctl ctl,
                           int first) {
  const int pb = sel_problem(sel_of(ctl), blockIdx.y);
  if (pb < 0) return;
  const size_t base = (size_t)pb * cells;
  const T beta = (T)ctl.scal[(size_t)pb * kSlots + S_BETA];
  CELL_LOOP(cells) p[base + c] = first ? z[base + c] : z[base + c] + beta * p[base + c];
}

// x += alpha p, r -= alpha q, ||r||^2 into the iteration epilogue
template <typename T>
__global__ void k_update_xr(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                            const T* __restrict__ q, int cells, Ctl ctl, EpiArgs e) {
  const int pb = sel_problem(sel_of(ctl), blockIdx.y);
  if (pb < 0) return;
  const size_t base = (size_t)pb * cells;
  const T alpha = (T)ctl.scal[(size_t)pb * kSlots + S_ALPHA];
  double acc = 0.0;
  CELL_LOOP(cells) {
    x[base + c] += alpha * p[base + c];
    const T rc = r[base + c] - alpha * q[base + c];
    r[base + c] = rc;
    acc += (double)rc * (double)rc;
  }
  block_partial(acc, ctl, pb);
}

// r = rhs with ||r||^2 block partials: the residual of a zero iterate
template <typename T>
__global__ void k_copy_sq(const T* __restrict__ rhs, T* __restrict__ r, int cells, Ctl ctl) {
  const int pb = blockIdx.y;
  const size_t base = (size_t)pb * cells;
  double acc = 0.0;
  CELL_LOOP(cells) {
    const T v = rhs[base + c];
    r[base + c] = v;
    acc += (double)v * (double)v;
  }
  block_partial(acc, ctl, pb);
}

template <typename T>
__global__ void k_fill(T* __restrict__ v, int cells, T val) {
  const size_t base = (size_t)blockIdx.y * cells;
  CELL_LOOP(cells) v[base + c] = val;
}

// mixed mode: r32 = r64 / ||r64|| (scale from the outer control block), the inner
// solve's iterate d32 = 0, and ||r32||^2 block partials into the inner control block
// (zero for a problem the outer loop no longer refines): the inner solve starts from
// d32 = 0, so r32 is its residual and these are its start partials
__global__ void k_scale_down(const double* __restrict__ r, float* __restrict__ r32,
                             float* __restrict__ d32, int cells, const double* __restrict__ oscal,
                             const int* __restrict__ oactive, Ctl ictl) {
  const int pb = blockIdx.y;
  if (!oactive[pb]) {
    if (threadIdx.x == 0) ictl.partials[(size_t)pb * ictl.pstride + blockIdx.x] = 0.0;
    return;
  }
  const size_t base = (size_t)pb * cells;
  const double inv = 1.0 / sqrt(oscal[(size_t)pb * kSlots + S_RR]);
  double acc = 0.0;
  CELL_LOOP(cells) {
    const float v = (float)(r[base + c] * inv);
    r32[base + c] = v;
    d32[base + c] = 0.0f;
    acc += (double)v * (double)v;
  }
  block_partial(acc, ictl, pb);
}

// The right-hand side's mean and norm from another control block (one that assembled the
// same right-hand side): S_MEAN, S_BB and S_TOL2 = rtol2 S_BB, as the assembly's epilogues
__global__ void k_take_rhs(Ctl dst, const double* __restrict__ src_scal, int B, double rtol2) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double* sc = src_scal + (size_t)b * kSlots;
  double* d = dst.scal + (size_t)b * kSlots;
  d[S_MEAN] = sc[S_MEAN];
  d[S_BB] = sc[S_BB];
  d[S_TOL2] = rtol2 * sc[S_BB];
}

// A control block back to its start: active flags, iteration counts, statuses and the
// scalar slots zero (one launch instead of four fills)
__global__ void k_ctl_reset(Ctl ctl, int B) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < B) {
    ctl.active[t] = 0;
    ctl.iters[t] = 0;
    ctl.status[t] = 0;
  }
  if (t < B * kSlots) ctl.scal[t] = 0.0;
}

// mixed mode: x64 += ||r64|| d32
__global__ void k_correct(double* __restrict__ x, const float* __restrict__ d, int cells,
                          const double* __restrict__ oscal, const int* __restrict__ oactive) {
  const int pb = blockIdx.y;
  if (!oactive[pb]) return;
  const size_t base = (size_t)pb * cells;
  const double s = sqrt(oscal[(size_t)pb * kSlots + S_RR]);
  CELL_LOOP(cells) x[base + c] += s * (double)d[base + c];
}

// Residual refinement: a problem whose inner solve ended in a breakdown or ran out of
// the inner iteration budget stops refining (its outer status takes the inner one, so
// the next outer residual does not re-arm it); the other problems go on.
__global__ void k_stop_failed(int B, const int* __restrict__ istatus, int* __restrict__ ostatus,
                              int* __restrict__ oactive) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B && istatus[b] != MPP_OK && ostatus[b] == MPP_OK) {
    ostatus[b] = istatus[b];
    oactive[b] = 0;
  }
}

// list = [count, the problems whose active flag is set, in ascending order]: the row map
// of the CG iterations (one block of 1024 threads; a wave ballot and the counts of the
// waves before it place each problem)
__global__ void __launch_bounds__(1024)
    k_live_list(const int* __restrict__ active, int B, int* __restrict__ list) {
  __shared__ int wcount[16];
  __shared__ int base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) base = 0;
  for (int c0 = 0; c0 < B; c0 += 1024) {
    const int b = c0 + (int)threadIdx.x;
    const int on = (b < B && active[b]) ? 1 : 0;
    const unsigned long long m = __ballot(on);
    if (lane == 0) wcount[w] = __popcll(m);
    __syncthreads();
    int at = base + __popcll(m & ((1ull << lane) - 1ull));
    for (int q = 0; q < w; ++q) at += wcount[q];
    if (on) list[1 + at] = b;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int q = 0; q < 16; ++q) base += wcount[q];
    __syncthreads();
  }
  if (threadIdx.x == 0) list[0] = base;
}

}  // namespace mpp

namespace mpp {

// ------------------------------------------------------------------------------
// the bottom of the V-cycle in one launch: levels with at most kSmallCells cells per
// problem are smoothed, restricted, solved and prolonged by a single workgroup per
// problem, with barriers between phases.  Same operations, in the same order, as the
// per-level kernels.  Every level's iterate and right-hand side live in LDS for the
// whole launch (the first level's rhs is read in, its iterate written out at the end),
// and so do the face coefficients when they fit (kSmallLdsBytes: all of them in FP32;
// in FP64 they are read through the caches).
// ------------------------------------------------------------------------------
constexpr int kSmallCells = 4096;   // 16^3
constexpr int kSmallBlock = 1024;
constexpr int kSmallLdsBytes = 144 * 1024;

template <typename T>
struct SmallLevel {
  int n;
  const T* bx;
  const T* by;
  const T* bz;
  T* b;
  T* x;
  T sig;   // diagonal shift of the level (operator A - sig I)
};

template <typename T>
struct SmallCycle {
  int nlev;                        // levels in the sub-cycle (the last one is solved directly)
  SmallLevel<T> lv[kMaxLevels];
  const double* inv;               // [B][m][m]
  int m;
  int nu;
};

// LDS elements the small cycle needs: x, b and the reciprocal diagonal of every level
// plus a residual scratch of the first level's size (`fixed`), and the faces of every
// level (`faces`)
template <typename T>
inline void small_lds_bytes(const SmallCycle<T>& S, size_t& fixed, size_t& faces) {
  size_t cells = 0;
  for (int l = 0; l < S.nlev; ++l) cells += (size_t)S.lv[l].n * S.lv[l].n * S.lv[l].n;
  const size_t c0 = (size_t)S.lv[0].n * S.lv[0].n * S.lv[0].n;
  fixed = (3 * cells + c0) * sizeof(T);
  faces = 3 * cells * sizeof(T);
}

// One level as the kernel sees it: x, b and 1/diagonal in LDS; the faces in LDS (FL) or
// in global memory.  Pointers are formed from the LDS base inside the kernel, so the
// compiler addresses LDS directly.
template <typename T, bool FL>
struct SmallView {
  int n, lg;   // lg = log2(n) when n is a power of two, else -1
  T* x;
  T* b;
  T* rd;
  const T* bx;
  const T* by;
  const T* bz;
  T sig;
};

__device__ inline int small_cube(int n) { return n * n * n; }

// LDS element offset of level l's block (x, b, rd [, bx, by, bz]); l == nlev: the scratch
template <typename T, bool FL>
__device__ inline int small_off(const SmallCycle<T>& S, int l) {
  int off = 0;
  for (int q = 0; q < l; ++q) off += (FL ? 6 : 3) * small_cube(S.lv[q].n);
  return off;
}

template <typename T, bool FL>
__device__ inline SmallView<T, FL> small_view(const SmallCycle<T>& S, T* lds, int pb, int l) {
  const SmallLevel<T>& G = S.lv[l];
  const int n = G.n, cells = small_cube(n);
  T* p = lds + small_off<T, FL>(S, l);
  SmallView<T, FL> v;
  v.n = n;
  v.lg = (n & (n - 1)) == 0 ? __builtin_ctz((unsigned)n) : -1;
  v.x = p;
  v.b = p + cells;
  v.rd = p + 2 * cells;
  if (FL) {
    v.bx = p + 3 * cells;
    v.by = p + 4 * cells;
    v.bz = p + 5 * cells;
  } else {
    const size_t gb = (size_t)pb * cells;
    v.bx = G.bx + gb;
    v.by = G.by + gb;
    v.bz = G.bz + gb;
  }
  v.sig = G.sig;
  return v;
}

// (i, j, k) of cell c; shifts when n is a power of two
__device__ inline void small_ijk(int c, int n, int lg, int& i, int& j, int& k) {
  if (lg >= 0) {
    i = c & (n - 1);
    j = (c >> lg) & (n - 1);
    k = c >> (2 * lg);
  } else {
    ijk(c, n, i, j, k);
  }
}

// cell of colour `colour` with index q among the cells/2 of that colour (n even: half
// of every x-row)
__device__ inline int small_colour_cell(int q, int n, int lg, int colour, int& i, int& j, int& k) {
  const int nh = n >> 1;
  int row, ih;
  if (lg >= 1) {
    ih = q & (nh - 1);
    row = q >> (lg - 1);
    j = row & (n - 1);
    k = row >> lg;
  } else {
    ih = q % nh;
    row = q / nh;
    j = row % n;
    k = row / n;
  }
  i = 2 * ih + ((colour + j + k) & 1);
  return i + n * (j + n * k);
}

template <typename T, bool FL>
__device__ inline void small_faces(const SmallView<T, FL>& L, int c, int i, int j, int k, T w[6]) {
  const int n = L.n, nn = n * n;
  w[0] = i > 0 ? L.bx[c] : T(0);
  w[1] = i < n - 1 ? L.bx[c + 1] : T(0);
  w[2] = j > 0 ? L.by[c] : T(0);
  w[3] = j < n - 1 ? L.by[c + n] : T(0);
  w[4] = k > 0 ? L.bz[c] : T(0);
  w[5] = k < n - 1 ? L.bz[c + nn] : T(0);
}

// rd = 1 / (sum of the faces + sig h^2) of every cell
template <typename T, bool FL>
__device__ void small_diag(const SmallView<T, FL>& L) {
  const int n = L.n, cells = small_cube(n);
  const T h2 = (T)(1.0 / ((double)n * (double)n));
  for (int c = threadIdx.x; c < cells; c += blockDim.x) {
    int i, j, k;
    small_ijk(c, n, L.lg, i, j, k);
    T w[6];
    small_faces(L, c, i, j, k, w);
    L.rd[c] = T(1) / (w[0] + w[1] + w[2] + w[3] + w[4] + w[5] + L.sig * h2);
  }
}

// one colour of Gauss-Seidel; from_zero: the other colour is taken as (and set to) zero
template <typename T, bool FL>
__device__ void small_smooth(const SmallView<T, FL>& L, int colour, int from_zero) {
  const int n = L.n, half = small_cube(n) / 2, nn = n * n;
  const T h2 = (T)(1.0 / ((double)n * (double)n));
  if (from_zero)
    for (int q = threadIdx.x; q < half; q += blockDim.x) {
      int i, j, k;
      L.x[small_colour_cell(q, n, L.lg, colour + 1, i, j, k)] = T(0);
    }
  for (int q = threadIdx.x; q < half; q += blockDim.x) {
    int i, j, k;
    const int c = small_colour_cell(q, n, L.lg, colour, i, j, k);
    T w[6];
    small_faces(L, c, i, j, k, w);
    T num = T(0);
    if (!from_zero) {
      if (i > 0) num += w[0] * L.x[c - 1];
      if (i < n - 1) num += w[1] * L.x[c + 1];
      if (j > 0) num += w[2] * L.x[c - n];
      if (j < n - 1) num += w[3] * L.x[c + n];
      if (k > 0) num += w[4] * L.x[c - nn];
      if (k < n - 1) num += w[5] * L.x[c + nn];
    }
    L.x[c] = (num - h2 * L.b[c]) * L.rd[c];
  }
  __syncthreads();
}

// coarse b = mean over the 8 children of (b - A x): residuals of every fine cell into
// `tmp`, then the sums over children
template <typename T, bool FL>
__device__ void small_resid_restrict(const SmallView<T, FL>& F, const SmallView<T, FL>& C,
                                     T* tmp) {
  const int nf = F.n, nc = C.n, cells_f = small_cube(nf), cells_c = small_cube(nc);
  const T inv_h2 = (T)((double)nf * (double)nf);
  for (int c = threadIdx.x; c < cells_f; c += blockDim.x) {
    int i, j, k;
    small_ijk(c, nf, F.lg, i, j, k);
    T w[6];
    small_faces(F, c, i, j, k, w);
    tmp[c] = F.b[c] - stencil_at(w, F.x, 0, c, i, j, k, nf, inv_h2, F.sig);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < cells_c; c += blockDim.x) {
    int I, J, K;
    small_ijk(c, nc, C.lg, I, J, K);
    T s = T(0);
    for (int e = 0; e < 2; ++e)
      for (int d = 0; d < 2; ++d)
        for (int a = 0; a < 2; ++a)
          s += tmp[(2 * I + a) + nf * ((2 * J + d) + nf * (2 * K + e))];
    C.b[c] = s * T(0.125);
  }
  __syncthreads();
}

template <typename T, bool FL>
__device__ void small_prolong(const SmallView<T, FL>& F, const SmallView<T, FL>& C) {
  const int nf = F.n, nc = C.n, cells_f = small_cube(nf);
  for (int c = threadIdx.x; c < cells_f; c += blockDim.x) {
    int i, j, k;
    small_ijk(c, nf, F.lg, i, j, k);
    F.x[c] += C.x[(i >> 1) + nc * ((j >> 1) + nc * (k >> 1))];
  }
  __syncthreads();
}

// Copies the global arrays the cycle reads into their LDS places: the first level's
// right-hand side and (FL) the faces of every level (at most 3 levels of at most 4096
// cells).  Every thread issues all of its loads before its first store, so the copy
// costs about one memory latency.
template <typename T, bool FL>
__device__ void small_copy_in(const SmallCycle<T>& S, T* lds, int pb) {
  constexpr int kU = kSmallCells / kSmallBlock;
  T v[3][4][kU];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        v[l][a][u] = T(0);
        if (l < S.nlev && (a < 3 ? FL : l == 0)) {
          const SmallLevel<T>& G = S.lv[l];
          const int c = small_cube(G.n), q = threadIdx.x + u * kSmallBlock;
          const T* src = a == 0 ? G.bx : (a == 1 ? G.by : (a == 2 ? G.bz : G.b));
          if (q < c) v[l][a][u] = src[(size_t)pb * c + q];
        }
      }
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (l < S.nlev && (a < 3 ? FL : l == 0)) {
          const int c = small_cube(S.lv[l].n), q = threadIdx.x + u * kSmallBlock;
          // LDS block of level l: x, b, rd, bx, by, bz
          T* dst = lds + small_off<T, FL>(S, l) + (a < 3 ? (3 + a) * c : c);
          if (q < c) dst[q] = v[l][a][u];
        }
}

template <typename T, bool FL>
__global__ void __launch_bounds__(kSmallBlock) k_small_cycle(SmallCycle<T> S, Sel sel) {
  const int pb = sel_problem(sel, blockIdx.x);
  if (pb < 0) return;
  __shared__ __align__(16) unsigned char lds_raw[kSmallLdsBytes];
  __shared__ double sb[kMaxCoarse];
  T* const lds = reinterpret_cast<T*>(lds_raw);
  T* const tmp = lds + small_off<T, FL>(S, S.nlev);
  const int nl = S.nlev;
  small_copy_in<T, FL>(S, lds, pb);
  __syncthreads();
  for (int l = 0; l + 1 < nl; ++l) small_diag(small_view<T, FL>(S, lds, pb, l));
  __syncthreads();
  for (int l = 0; l + 1 < nl; ++l) {
    const SmallView<T, FL> V = small_view<T, FL>(S, lds, pb, l);
    small_smooth(V, 0, 1);
    small_smooth(V, 1, 0);
    for (int q = 1; q < S.nu; ++q) {
      small_smooth(V, 0, 0);
      small_smooth(V, 1, 0);
    }
    small_resid_restrict(V, small_view<T, FL>(S, lds, pb, l + 1), tmp);
  }
  {
    // coarsest: x = M^{-1} (-b), FP64.  G groups of threads split the columns q of
    // row r; their partial sums meet in the scratch (read back in a fixed order).
    const SmallView<T, FL> C = small_view<T, FL>(S, lds, pb, nl - 1);
    const int m = S.m;
    for (int q = threadIdx.x; q < m; q += blockDim.x) sb[q] = -(double)C.b[q];
    __syncthreads();
    const double* Mi = S.inv + (size_t)pb * m * m;
    const int tmp_bytes = small_cube(S.lv[0].n) * (int)sizeof(T);
    const int G = max(1, min(kSmallBlock / m, tmp_bytes / (8 * m)));
    double* part = reinterpret_cast<double*>(tmp);
    if (G == 1) {
      for (int r = threadIdx.x; r < m; r += blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < m; ++q) s += Mi[(size_t)q * m + r] * sb[q];
        C.x[r] = (T)s;
      }
    } else {
      const int t = threadIdx.x;
      if (t < G * m) {
        const int r = t % m, g = t / m;
        double s = 0.0;
#pragma unroll 4
        for (int q = g; q < m; q += G) s += Mi[(size_t)q * m + r] * sb[q];
        part[g * m + r] = s;
      }
      __syncthreads();
      for (int r = threadIdx.x; r < m; r += blockDim.x) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) s += part[g * m + r];
        C.x[r] = (T)s;
      }
    }
    __syncthreads();
  }
  for (int l = nl - 2; l >= 0; --l) {
    const SmallView<T, FL> V = small_view<T, FL>(S, lds, pb, l);
    small_prolong(V, small_view<T, FL>(S, lds, pb, l + 1));
    for (int q = 0; q < S.nu; ++q) {
      small_smooth(V, 1, 0);
      small_smooth(V, 0, 0);
    }
  }
  {
    const int c0 = small_cube(S.lv[0].n);
    T* out = S.lv[0].x + (size_t)pb * c0;
    const T* x0 = lds + small_off<T, FL>(S, 0);
    for (int q = threadIdx.x; q < c0; q += blockDim.x) out[q] = x0[q];
  }
}

}  // namespace mpp
