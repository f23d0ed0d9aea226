// Level set around the projection (Sec. 3, Multiphase / StencilsLevelSet): phi is
// moved with the flow and kept a signed distance.  The paper names these operations
// without a scheme; this library uses
//   advection:      one forward-Euler step of phi_t + u . grad phi = 0 with first-order
//                   upwind differences, the cell-centre velocity the mean of the cell's
//                   two faces along each axis (wall faces 0);
//   re-distancing:  pseudo-time steps of phi_tau + S(phi0) (|grad phi| - 1) = 0 with
//                   S(phi0) = phi0 / sqrt(phi0^2 + h^2) and the first-order Godunov
//                   upwind |grad phi|, forward Euler;
// differences across a wall are 0 (phi extended by its boundary value).  FP64, one
// thread per cell, no contraction: every value is the exactly rounded result of its
// expression in the order written.
#pragma once

#include "kernels.h"

namespace mpp {

constexpr int kLsBlock = 256;

// out = phi - dt (ax + ay + az), a_d = u_d (backward difference if u_d > 0, else
// forward difference), u_d the cell-centre velocity along axis d
__global__ void __launch_bounds__(kLsBlock)
    k_ls_advect(const double* __restrict__ phi, const double* __restrict__ ux,
                const double* __restrict__ uy, const double* __restrict__ uz, int n, int cells,
                double dt, double* __restrict__ out) {
#pragma clang fp contract(off)
  const int c = blockIdx.x * kLsBlock + threadIdx.x;
  if (c >= cells) return;
  const size_t q = (size_t)blockIdx.y * cells + c;
  int i, j, k;
  ijk(c, n, i, j, k);
  const double inv_h = (double)n;
  const size_t nn = (size_t)n * n;
  const double pc = phi[q];
  auto axis = [&](const double* __restrict__ u, int at, size_t step) {
    const double ulo = at > 0 ? u[q] : 0.0;
    const double uhi = at < n - 1 ? u[q + step] : 0.0;
    const double uc = 0.5 * (ulo + uhi);
    const double back = at > 0 ? (pc - phi[q - step]) * inv_h : 0.0;
    const double fwd = at < n - 1 ? (phi[q + step] - pc) * inv_h : 0.0;
    return uc > 0.0 ? uc * back : uc * fwd;
  };
  const double ax = axis(ux, i, 1), ay = axis(uy, j, (size_t)n), az = axis(uz, k, nn);
  out[q] = pc - dt * ((ax + ay) + az);
}

// one re-distancing step: out = phi - dtau S (G - 1), S = phi0 / sqrt(phi0^2 + h^2),
// G the Godunov |grad phi| for the sign of S
__global__ void __launch_bounds__(kLsBlock)
    k_ls_reinit(const double* __restrict__ phi0, const double* __restrict__ phi, int n, int cells,
                double dtau, double* __restrict__ out) {
#pragma clang fp contract(off)
  const int c = blockIdx.x * kLsBlock + threadIdx.x;
  if (c >= cells) return;
  const size_t q = (size_t)blockIdx.y * cells + c;
  int i, j, k;
  ijk(c, n, i, j, k);
  const double inv_h = (double)n;
  const double h = 1.0 / (double)n;
  const size_t nn = (size_t)n * n;
  const double p0 = phi0[q];
  const double s = p0 / sqrt(p0 * p0 + h * h);
  const double pc = phi[q];
  auto axis = [&](int at, size_t step) {
    const double back = at > 0 ? (pc - phi[q - step]) * inv_h : 0.0;
    const double fwd = at < n - 1 ? (phi[q + step] - pc) * inv_h : 0.0;
    double t1, t2;
    if (s > 0.0) {
      t1 = back > 0.0 ? back : 0.0;
      t2 = fwd < 0.0 ? fwd : 0.0;
    } else {
      t1 = back < 0.0 ? back : 0.0;
      t2 = fwd > 0.0 ? fwd : 0.0;
    }
    const double a = t1 * t1, b = t2 * t2;
    return a > b ? a : b;
  };
  double g2 = 0.0;
  g2 += axis(i, 1);
  g2 += axis(j, (size_t)n);
  g2 += axis(k, nn);
  out[q] = pc - dtau * s * (sqrt(g2) - 1.0);
}

__global__ void __launch_bounds__(kLsBlock)
    k_ls_copy(const double* __restrict__ src, int cells, double* __restrict__ dst) {
  const int c = blockIdx.x * kLsBlock + threadIdx.x;
  if (c >= cells) return;
  const size_t q = (size_t)blockIdx.y * cells + c;
  dst[q] = src[q];
}

}  // namespace mpp
