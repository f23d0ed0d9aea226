// Level set around the projection (Sec. 3, Multiphase / StencilsLevelSet): phi is
// moved with the flow and kept a signed distance.  The paper names these operations
// without a scheme; this library uses
//   advection:      one forward-Euler step of phi_t + u . grad phi = 0 with first-order
//                   upwind differences, the cell-centre velocity the mean of the cell's
//                   two faces along each axis (wall faces 0);
//   re-distancing:  pseudo-time steps of phi_tau + S(phi0) (|grad phi| - 1) = 0 with
//                   S(phi0) = phi0 / sqrt(phi0^2 + h^2) and the first-order Godunov
//                   upwind |grad phi|, forward Euler;
// differences across a wall are 0 (phi extended by its boundary value).  FP64, no
// contraction: every value is the exactly rounded result of its expression in the order
// written.
#pragma once

#include "rbgs.h"

namespace mpp {

constexpr int kLsBlock = 256;

// Both kernels march columns: a block owns a 64 x 4 column of cells and a chunk of
// planes, holding phi of planes k - 1, k, k + 1 of its own column in registers; in-plane
// neighbours come through the caches.
//   k_ls_advect_z: out = phi - dt (ax + ay + az), a_d = u_d (backward difference if
//                  u_d > 0, else forward difference), u_d the cell-centre velocity;
//   k_ls_reinit_z: one re-distancing step, out = phi - dtau S (G - 1), S = phi0 /
//                  sqrt(phi0^2 + h^2), G the Godunov |grad phi| for the sign of S.
constexpr int kLsTX = 64, kLsTY = 4, kLsKZ = 16;

struct LsTiles {
  int ntx, nty, nkz, ntiles;
};

inline LsTiles ls_tiles(int n) {
  LsTiles t;
  t.ntx = (n + kLsTX - 1) / kLsTX;
  t.nty = (n + kLsTY - 1) / kLsTY;
  t.nkz = (n + kLsKZ - 1) / kLsKZ;
  t.ntiles = t.ntx * t.nty * t.nkz;
  return t;
}

__global__ void __launch_bounds__(kLsTX * kLsTY)
    k_ls_advect_z(const double* __restrict__ phi, const double* __restrict__ ux,
                  const double* __restrict__ uy, const double* __restrict__ uz, int n, LsTiles tl,
                  double dt, double* __restrict__ out) {
#pragma clang fp contract(off)
  const int tile = xcd_tile(blockIdx.x, tl.ntiles);
  if (tile < 0) return;
  const int ti = tile % tl.ntx, tj = (tile / tl.ntx) % tl.nty, tk = tile / (tl.ntx * tl.nty);
  const int i = ti * kLsTX + threadIdx.x % kLsTX, j = tj * kLsTY + threadIdx.x / kLsTX;
  if (i >= n || j >= n) return;
  const int k0 = tk * kLsKZ, k1 = min(k0 + kLsKZ, n);
  const size_t nn = (size_t)n * n;
  const size_t col = (size_t)blockIdx.y * nn * n + (size_t)i + (size_t)n * j;
  const double inv_h = (double)n;
  auto flux = [&](double ulo, double uhi, double pm, double pc, double pp, bool lo, bool hi) {
    const double uc = 0.5 * (ulo + uhi);
    const double back = lo ? (pc - pm) * inv_h : 0.0;
    const double fwd = hi ? (pp - pc) * inv_h : 0.0;
    return uc > 0.0 ? uc * back : uc * fwd;
  };
  double pm = k0 > 0 ? phi[col + (size_t)(k0 - 1) * nn] : 0.0;
  double pc = phi[col + (size_t)k0 * nn];
  double uzc = k0 > 0 ? uz[col + (size_t)k0 * nn] : 0.0;
  for (int k = k0; k < k1; ++k) {
    const size_t q = col + (size_t)k * nn;
    const double pp = k < n - 1 ? phi[q + nn] : 0.0;
    const double uzn = k < n - 1 ? uz[q + nn] : 0.0;
    const double ax = flux(i > 0 ? ux[q] : 0.0, i < n - 1 ? ux[q + 1] : 0.0, i > 0 ? phi[q - 1] : 0.0,
                           pc, i < n - 1 ? phi[q + 1] : 0.0, i > 0, i < n - 1);
    const double ay = flux(j > 0 ? uy[q] : 0.0, j < n - 1 ? uy[q + n] : 0.0, j > 0 ? phi[q - n] : 0.0,
                           pc, j < n - 1 ? phi[q + n] : 0.0, j > 0, j < n - 1);
    const double az = flux(uzc, uzn, pm, pc, pp, k > 0, k < n - 1);
    out[q] = pc - dt * ((ax + ay) + az);
    pm = pc;
    pc = pp;
    uzc = uzn;
  }
}

__global__ void __launch_bounds__(kLsTX * kLsTY)
    k_ls_reinit_z(const double* __restrict__ phi0, const double* __restrict__ phi, int n,
                  LsTiles tl, double dtau, double* __restrict__ out) {
#pragma clang fp contract(off)
  const int tile = xcd_tile(blockIdx.x, tl.ntiles);
  if (tile < 0) return;
  const int ti = tile % tl.ntx, tj = (tile / tl.ntx) % tl.nty, tk = tile / (tl.ntx * tl.nty);
  const int i = ti * kLsTX + threadIdx.x % kLsTX, j = tj * kLsTY + threadIdx.x / kLsTX;
  if (i >= n || j >= n) return;
  const int k0 = tk * kLsKZ, k1 = min(k0 + kLsKZ, n);
  const size_t nn = (size_t)n * n;
  const size_t col = (size_t)blockIdx.y * nn * n + (size_t)i + (size_t)n * j;
  const double inv_h = (double)n;
  const double h = 1.0 / (double)n;
  double pm = k0 > 0 ? phi[col + (size_t)(k0 - 1) * nn] : 0.0;
  double pc = phi[col + (size_t)k0 * nn];
  for (int k = k0; k < k1; ++k) {
    const size_t q = col + (size_t)k * nn;
    const double pp = k < n - 1 ? phi[q + nn] : 0.0;
    const double p0 = phi0[q];
    const double s = p0 / sqrt(p0 * p0 + h * h);
    auto axis = [&](bool lo, bool hi, double vm, double vp) {
      const double back = lo ? (pc - vm) * inv_h : 0.0;
      const double fwd = hi ? (vp - pc) * inv_h : 0.0;
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
    g2 += axis(i > 0, i < n - 1, i > 0 ? phi[q - 1] : 0.0, i < n - 1 ? phi[q + 1] : 0.0);
    g2 += axis(j > 0, j < n - 1, j > 0 ? phi[q - n] : 0.0, j < n - 1 ? phi[q + n] : 0.0);
    g2 += axis(k > 0, k < n - 1, pm, pp);
    out[q] = pc - dtau * s * (sqrt(g2) - 1.0);
    pm = pc;
    pc = pp;
  }
}

__global__ void __launch_bounds__(kLsBlock)
    k_ls_copy(const double* __restrict__ src, int cells, double* __restrict__ dst) {
  const int c = blockIdx.x * kLsBlock + threadIdx.x;
  if (c >= cells) return;
  const size_t q = (size_t)blockIdx.y * cells + c;
  dst[q] = src[q];
}

}  // namespace mpp
