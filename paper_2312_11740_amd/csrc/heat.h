// Implicit heat diffusion: one backward-Euler step of the
// diffusion term of the transport equation (Sec. 2) with a coefficient that changes
// with the phase (the varDiffusion configuration of HeatAD, Sec. 3),
//
//     (I - dt div(K grad)) T = T_old + dt f,        insulated walls.
//
// K is read from an operator's face coefficients: built from the level set with
// rho = 1/K of each phase, they hold K of the cell's phase on uncrossed faces and the
// two conductivities in series on crossed ones.  The system is solved as
// (A - I/dt) T = -(T_old + dt f)/dt, A = div(K grad) as in the pressure operator: the
// matrix is negative definite like the pressure one, and the pressure solve's MG-PCG
// runs on it unchanged once every level carries its diagonal shift (the kernels' sig).
// The kernels below serve the other preconditioner, the inverse diagonal, which solves
// (dt A - I) T = -(T_old + dt f) with the same CG bookkeeping (r.z < 0, p.q < 0).
#pragma once

#include "stencil.h"

namespace mpp {

__global__ void k_heat_set_dt(double* scal, int B, double dt) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) scal[(size_t)b * kSlots + S_DT] = dt;
}

// b = -(t_old + dt src) scale (src may be null) with ||b||^2 block partials
__global__ void k_heat_rhs(const double* __restrict__ t_old, const double* __restrict__ src,
                           double scale, double* __restrict__ b, int cells, Ctl ctl) {
  const int pb = blockIdx.y;
  const size_t base = (size_t)pb * cells;
  const double dt = ctl.scal[(size_t)pb * kSlots + S_DT];
  double acc = 0.0;
  CELL_LOOP(cells) {
    double v = t_old[base + c];
    if (src) v = v + dt * src[base + c];
    v = -v * scale;
    b[base + c] = v;
    acc += v * v;
  }
  block_partial(acc, ctl, pb);
}

// KIND 0: y = (dt A - I) x with x.y partials (problems whose active flag is 0 are
// skipped); KIND 1: y = b - (dt A - I) x with ||y||^2 partials.  Same column march as
// the pressure stencil: a block owns a 64 x 4 column tile and a chunk of planes.
template <int KIND>
__global__ void __launch_bounds__(kStThreads)
    k_heat_z(Faces<double> F, int n, StTiles tl, int kz, const double* __restrict__ x,
             const double* __restrict__ bvec, double* __restrict__ y, Ctl ctl,
             const int* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int tile = xcd_tile(blockIdx.x, tl.ntiles);
  if (tile < 0) {
    if (threadIdx.x == 0) ctl.partials[(size_t)b * ctl.pstride + blockIdx.x] = 0.0;
    return;
  }
  const int ti = tile % tl.ntx, tj = (tile / tl.ntx) % tl.nty, tk = tile / (tl.ntx * tl.nty);
  const int i = ti * kStTX + threadIdx.x % kStTX, j = tj * kStTY + threadIdx.x / kStTX;
  const int k0 = tk * kz, k1 = min(k0 + kz, n);
  const size_t nn = (size_t)n * n;
  const size_t base = (size_t)b * nn * n;
  const double inv_h2 = (double)n * (double)n;
  const double dt = ctl.scal[(size_t)b * kSlots + S_DT];
  double acc = 0.0;
  if (i < n && j < n) {
    const int off = i + n * j;
    const double ir0 = F.inv_rho[2 * b], ir1 = F.inv_rho[2 * b + 1];
    for (int kb = k0; kb < k1; kb += kStZ) {
      ColBatch<double, true> B;
      load_batch<double, true>(x + base, F.code + base, off, i, j, kb, n, nn, false, B);
      double bv[kStZ];
      if (KIND == 1) {
#pragma unroll
        for (int h = 0; h < kStZ; ++h)
          bv[h] = (kb + h < k1) ? bvec[base + (size_t)(kb + h) * nn + off] : 0.0;
      }
#pragma unroll
      for (int h = 0; h < kStZ; ++h) {
        const int k = kb + h;
        if (k >= k1) break;
        const size_t cell = base + (size_t)k * nn + off;
        double w[6];
        coded_faces_at(F.bx + cell, F.by + cell, F.bz + cell, B.cd[h], i, j, k, n, nn,
                       (B.cd[h] & 64u) ? ir1 : ir0, w);
        const double xc = B.xc[h + 1];
        const double ax = stencil7(w, xc, B.w[h], B.e[h], B.s[h], B.nb[h], B.xc[h],
                                   B.xc[h + 2], i, j, k, n, inv_h2, 0.0);
        const double hx = dt * ax - xc;
        double out;
        if (KIND == 0) {
          out = hx;
          acc += xc * out;
        } else {
          out = bv[h] - hx;
          acc += out * out;
        }
        y[cell] = out;
      }
    }
  }
  block_partial(acc, ctl, b);
}

// z = r / diag(dt A - I) = -r / (1 + dt sum_f K_f / h^2) with r.z partials
__global__ void __launch_bounds__(kStThreads)
    k_heat_jacobi(Faces<double> F, int n, StTiles tl, int kz, const double* __restrict__ r,
                  double* __restrict__ z, Ctl ctl, const int* __restrict__ active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int tile = xcd_tile(blockIdx.x, tl.ntiles);
  if (tile < 0) {
    if (threadIdx.x == 0) ctl.partials[(size_t)b * ctl.pstride + blockIdx.x] = 0.0;
    return;
  }
  const int ti = tile % tl.ntx, tj = (tile / tl.ntx) % tl.nty, tk = tile / (tl.ntx * tl.nty);
  const int i = ti * kStTX + threadIdx.x % kStTX, j = tj * kStTY + threadIdx.x / kStTX;
  const int k0 = tk * kz, k1 = min(k0 + kz, n);
  const size_t nn = (size_t)n * n;
  const size_t base = (size_t)b * nn * n;
  const double inv_h2 = (double)n * (double)n;
  const double dt = ctl.scal[(size_t)b * kSlots + S_DT];
  double acc = 0.0;
  if (i < n && j < n) {
    const int off = i + n * j;
    const double ir0 = F.inv_rho[2 * b], ir1 = F.inv_rho[2 * b + 1];
    for (int k = k0; k < k1; ++k) {
      const size_t cell = base + (size_t)k * nn + off;
      const unsigned cd = F.code[cell];
      double w[6];
      coded_faces_at(F.bx + cell, F.by + cell, F.bz + cell, cd, i, j, k, n, nn,
                     (cd & 64u) ? ir1 : ir0, w);
      const double sw = ((w[0] + w[1]) + (w[2] + w[3])) + (w[4] + w[5]);
      const double rc = r[cell];
      const double zc = -rc / (1.0 + dt * (sw * inv_h2));
      z[cell] = zc;
      acc += rc * zc;
    }
  }
  block_partial(acc, ctl, b);
}

}  // namespace mpp
