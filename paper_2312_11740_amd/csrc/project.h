// The projection around the solve (Sec. 2: fractional step on the staggered grid):
// the right-hand side f = div(u*)/dt from the face velocities, and the correction
// u = u* - dt beta^ grad p with the jump-corrected gradient, so that the corrected
// velocity is discretely divergence-free once p solves A p = f + jterm.
//
// Face velocities use the coefficients' low-face layout: ux[i,j,k] sits on the face
// between (i-1,j,k) and (i,j,k); ux[0,j,k] is the wall (read as 0, written as 0).
#pragma once

#include "kernels.h"

namespace mpp {

// f[c] = (sum over the axes of (u_high - u_low) / h) / dt; FP64, no contraction (the
// value is the exactly rounded result of that expression order)
__global__ void k_divergence(const double* __restrict__ ux, const double* __restrict__ uy,
                             const double* __restrict__ uz, int n, int cells, double dt,
                             double* __restrict__ f) {
#pragma clang fp contract(off)
  const size_t base = (size_t)blockIdx.y * cells;
  const size_t nn = (size_t)n * n;
  const double inv_h = (double)n;
  CELL_LOOP(cells) {
    int i, j, k;
    ijk(c, n, i, j, k);
    const size_t q = base + c;
    const double xl = i > 0 ? ux[q] : 0.0, xh = i < n - 1 ? ux[q + 1] : 0.0;
    const double yl = j > 0 ? uy[q] : 0.0, yh = j < n - 1 ? uy[q + n] : 0.0;
    const double zl = k > 0 ? uz[q] : 0.0, zh = k < n - 1 ? uz[q + nn] : 0.0;
    f[q] = (((xh - xl) + (yh - yl)) + (zh - zl)) * inv_h / dt;
  }
}

// The three low faces of every cell b: u -= dt beta^ ((p_b - p_a) - d J) / h with a
// the lower neighbour, J = sigma ((1-theta) kappa_a + theta kappa_b) on a crossed face
// and d = +1 when a is on the "-" side (-1 when on the "+" side); walls set to 0.
__global__ void k_project(const double* __restrict__ phi, const double* __restrict__ kappa,
                          const double* __restrict__ p, const double* __restrict__ rho, int n,
                          int cells, double dt, double* __restrict__ ux,
                          double* __restrict__ uy, double* __restrict__ uz) {
#pragma clang fp contract(off)
  const int b = blockIdx.y;
  const size_t base = (size_t)b * cells;
  const double rn = rho[3 * b + 0], rp = rho[3 * b + 1], sg = rho[3 * b + 2];
  const size_t off[3] = {1, (size_t)n, (size_t)n * n};
  const double inv_h = (double)n;
  double* u[3] = {ux, uy, uz};
  CELL_LOOP(cells) {
    int i, j, k;
    ijk(c, n, i, j, k);
    const int pos[3] = {i, j, k};
    const size_t qb = base + c;
    for (int d = 0; d < 3; ++d) {
      if (pos[d] == 0) {
        u[d][qb] = 0.0;
        continue;
      }
      const size_t qa = qb - off[d];
      const double pa = phi[qa], pb = phi[qb];
      const double beta = ghost_fluid_beta(pa, pb, rn, rp);
      double jump = 0.0;
      if (plus_side(pa) != plus_side(pb)) {
        const double theta = fabs(pa) / (fabs(pa) + fabs(pb));
        const double J = sg * ((1.0 - theta) * kappa[qa] + theta * kappa[qb]);
        jump = plus_side(pa) ? -J : J;
      }
      u[d][qb] -= dt * beta * ((p[qb] - p[qa]) - jump) * inv_h;
    }
  }
}

}  // namespace mpp
