// Glue between the solver and the learned-guess network: network inputs from an
// operator's density field and right-hand side (block means over r^3 cells), and the
// prolongation of the network's prediction back to the operator's grid.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mpp {

__device__ inline uint16_t bf16_rne(double v) {
  const float f = (float)v;
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// coarse[b][v][0..2] = means over the r^3 block of cell v of 1/rho, b and p (0 when p is
// NULL).  1/rho of a fine cell is that of its side (bit 6 of the finest-level code).
// Grid: (cells of a problem / 256, problems), 256 threads.  R > 0: r == R at compile
// time (the rows unroll); R == 0: r from the argument.  Each workgroup also writes the
// sum of the squared coarse b means of its cells to part[problem][blockIdx.x] (summed
// in a fixed order), from which k_feat_rms takes the rms.
template <int R>
__global__ void __launch_bounds__(256)
    k_feat_coarsen(const uint8_t* __restrict__ code, const double* __restrict__ inv_rho,
                   const double* __restrict__ b, const double* __restrict__ p, int nf, int r_arg,
                   int nc, double* __restrict__ coarse, double* __restrict__ part) {
  __shared__ double red[256];
  const int r = R > 0 ? R : r_arg;
  const unsigned l = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned cc = (unsigned)nc * nc * nc;
  const int q = blockIdx.y;
  if (l >= cc) {
    red[threadIdx.x] = 0.0;
  } else {
    const size_t idx = (size_t)q * cc + l;
    const int I = (int)(l % (unsigned)nc), J = (int)((l / (unsigned)nc) % (unsigned)nc),
              K = (int)(l / ((unsigned)nc * nc));
    const size_t base = (size_t)q * nf * nf * nf;
    double sr = 0.0, sb = 0.0, sp = 0.0;
    for (int dz = 0; dz < r; ++dz)
      for (int dy = 0; dy < r; ++dy)
#pragma unroll
        for (int dx = 0; dx < r; ++dx) {
          const size_t c = base + ((size_t)(K * r + dz) * nf + (J * r + dy)) * nf + (I * r + dx);
          sr += inv_rho[2 * q + ((code[c] >> 6) & 1)];
          sb += b[c];
          if (p) sp += p[c];
        }
    const double inv = 1.0 / ((double)r * r * r);
    coarse[3 * idx + 0] = sr * inv;
    coarse[3 * idx + 1] = sb * inv;
    coarse[3 * idx + 2] = sp * inv;
    red[threadIdx.x] = (sb * inv) * (sb * inv);
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)q * gridDim.x + blockIdx.x] = red[0];
}

// rms of the coarse right-hand side per problem (one block each) from the nparts
// partial sums k_feat_coarsen left per problem
__global__ void __launch_bounds__(1024)
    k_feat_rms(const double* __restrict__ part, int nparts, int cells, double* __restrict__ rms64,
               float* __restrict__ rms32) {
  __shared__ double red[1024];
  const int q = blockIdx.x, tid = threadIdx.x;
  const double* c = part + (size_t)q * nparts;
  double s = 0.0;
  for (int v = tid; v < nparts; v += 1024) s += c[v];
  red[tid] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    const double rms = sqrt(red[0] / cells);
    rms64[q] = rms;
    rms32[q] = (float)rms;
  }
}

// x[v] = (log10(mean 1/rho) / 3, b_c / rms, 0, 0) in BF16; t[v] = p_c / (rms h^2) (FP32),
// h = 1 / nc the spacing of the coarse grid (p ~ h^2 b for the discrete operator)
__global__ void k_feat_write(const double* __restrict__ coarse, const double* __restrict__ rms64,
                             int nc, int batch, uint16_t* __restrict__ x, float* __restrict__ t) {
  const int cells = nc * nc * nc;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)cells * batch) return;
  const int q = (int)(idx / cells);
  const double rms = rms64[q];
  const double* c = coarse + 3 * idx;
  const double xb = rms > 0.0 ? c[1] / rms : 0.0;
  const uint32_t lo = (uint32_t)bf16_rne(log10(c[0]) / 3.0) | ((uint32_t)bf16_rne(xb) << 16);
  *reinterpret_cast<uint2*>(x + 4 * idx) = make_uint2(lo, 0u);
  if (t) t[idx] = rms > 0.0 ? (float)(c[2] * ((double)nc * nc) / rms) : 0.f;
}

// p[fine cell] = rms h^2 * trilinear interpolation of y at the cell's centre (cell-centred
// coarse values, clamped at the walls; h = 1 / nc).  Grid: (rows of a problem = nf^2,
// problems), a block per row of nf cells along x: the row's y and z weights and coarse
// rows are the block's, each thread adds up x cells; R as for k_feat_coarsen.
template <int R>
__global__ void k_guess_prolong(const float* __restrict__ y, const double* __restrict__ rms64,
                                int nc, int r_arg, double* __restrict__ p) {
  const int r = R > 0 ? R : r_arg;
  const int nf = nc * r;
  const int row = blockIdx.x;   // j + nf k
  const int q = blockIdx.y;
  const int fj = row % nf, fk = row / nf;
  auto axis = [&](int f, int& i0, int& i1, double& w1) {
    const double u = (f + 0.5) / r - 0.5;
    const double fl = floor(u);
    w1 = u - fl;
    const int lo = (int)fl;
    i0 = lo < 0 ? 0 : (lo > nc - 1 ? nc - 1 : lo);
    i1 = lo + 1 < 0 ? 0 : (lo + 1 > nc - 1 ? nc - 1 : lo + 1);
  };
  int j0, j1, k0, k1;
  double wy, wz;
  axis(fj, j0, j1, wy);
  axis(fk, k0, k1, wz);
  const float* yq = y + (size_t)q * nc * nc * nc;
  const double scale = rms64[q] / ((double)nc * nc);
  double* pr = p + (size_t)q * nf * nf * nf + (size_t)row * nf;
  for (int fi = threadIdx.x; fi < nf; fi += blockDim.x) {
    int i0, i1;
    double wx;
    axis(fi, i0, i1, wx);
    double s = 0.0;
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          const double w = (cx ? wx : 1.0 - wx) * (cy ? wy : 1.0 - wy) * (cz ? wz : 1.0 - wz);
          const int X = cx ? i1 : i0, Y = cy ? j1 : j0, Z = cz ? k1 : k0;
          s += w * (double)yq[((size_t)Z * nc + Y) * nc + X];
        }
    pr[fi] = s * scale;
  }
}

// p = alpha (p - mean) with alpha = (p.b) / (p.Ap) from the slots (0 when p.Ap is 0 or
// either dot is not finite): the zero-mean multiple of p closest to the solution in the
// energy norm
// (p.b and p.Ap do not depend on the mean, b having zero mean and A annihilating
// constants, so the mean, scal[slot_mean], is removed in the same pass)
// (p32, optional: an FP32 copy of the result for the sweeps that follow)
__global__ void k_energy_scale(double* __restrict__ p, int cells, const double* __restrict__ scal,
                               int slot_pb, int slot_pap, int slot_mean, int slots,
                               float* __restrict__ p32) {
  const int q = blockIdx.y;
  const double* sc = scal + (size_t)q * slots;
  const double pb = sc[slot_pb], pap = sc[slot_pap], mean = sc[slot_mean];
  const double a = (pap != 0.0 && isfinite(pb) && isfinite(pap)) ? pb / pap : 0.0;
  double* pq = p + (size_t)q * cells;
  float* p32q = p32 ? p32 + (size_t)q * cells : nullptr;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += gridDim.x * blockDim.x) {
    const double v = a * (pq[c] - mean);
    pq[c] = v;
    if (p32q) p32q[c] = (float)v;
  }
}

}  // namespace mpp
