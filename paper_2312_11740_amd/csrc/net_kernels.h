// Kernels of the learned initial guess: a 3D U-Net whose 3x3x3 convolutions run as
// implicit GEMMs on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands,
// FP32 accumulation), plus its pooling, upsampling, loss and optimiser kernels.
//
// Fields are channels-last BF16 bit patterns, [sample][z][y][x][channel].  A
// convolution is the product of the im2col matrix (rows: cells, columns: k = tap * CI
// + c, tap = 9 (dz+1) + 3 (dy+1) + (dx+1)) with the weight matrix Wk[c_out][k]
// (zero-padded to Kp, a multiple of 32).  With 16 consecutive cells as the M rows of
// an MFMA tile, every lane's 8 K-values are 8 consecutive channels of one cell: one
// 16-byte load, channels being a multiple of 8.  The weight gradient is the product
// of the output gradient (transposed) with the im2col matrix, summed over cells.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mppnet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kNetThreads = 256;
constexpr int kConvMT = 4;   // 16-cell tiles per wave of the forward / data-gradient kernel
constexpr int kWgNT = 4;     // 16-column tiles per wave of the weight-gradient kernel

__host__ __device__ constexpr int kpad(int ci) { return (27 * ci + 31) / 32 * 32; }

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// FP32 -> BF16, round to nearest even (NaN stays NaN)
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline bf16x8 ld8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}

__device__ inline bf16x8 zero8() { return __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u}); }

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Input of a convolution: channels [0, CA) from `a`, at the convolution's resolution
// or (up = 1) at half of it, read at the parent cell (nearest upsampling); channels
// [CA, CI) from `b` at the convolution's resolution.
struct ConvSrc {
  const uint16_t* a;
  const uint16_t* b;
  int up;
};

__device__ inline void tap_offsets(int tap, int& dx, int& dy, int& dz) {
  dz = tap / 9 - 1;
  dy = (tap / 3) % 3 - 1;
  dx = tap % 3 - 1;
}

// im2col element group: 8 channels c.. of the input at cell (x, y, z) (inside the grid)
template <int CI, int CA>
__device__ inline const uint16_t* src_ptr(const ConvSrc& s, int b, int n, int x, int y, int z,
                                          int c) {
  if (c < CA) {
    const int na = n >> s.up;
    const size_t v = (size_t)b * na * na * na +
                     ((size_t)(z >> s.up) * na + (y >> s.up)) * na + (x >> s.up);
    return s.a + v * CA + c;
  }
  const size_t v = (size_t)b * n * n * n + ((size_t)z * n + y) * n + x;
  return s.b + v * (CI - CA) + (c - CA);
}

// ---------------------------------------------------------------------------------
// Convolution (forward, or data gradient with flipped and transposed weights).
// out[cell][co] = epilogue(sum_k im2col[cell][k] Wk[co][k]).  EPI 0: + bias, ReLU;
// EPI 1: times (mask[cell][co] > 0) when mask is given.  Rounded to BF16.
// A wave computes 4 tiles of 16 cells times all CO channels; grid (cells / 256, batch).
// Requires cells % 64 == 0.
// ---------------------------------------------------------------------------------
template <int CI, int CA, int CO, int EPI>
__global__ void __launch_bounds__(kNetThreads)
    k_conv(ConvSrc src, const uint16_t* __restrict__ w, const float* __restrict__ bias,
           const uint16_t* __restrict__ mask, uint16_t* __restrict__ out, int n) {
  constexpr int K = 27 * CI, KB = (K + 31) / 32, Kp = KB * 32, NT = CO / 16;
  static_assert(CI % 8 == 0 && CA % 8 == 0 && CO % 16 == 0, "channel counts");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int cells = n * n * n, b = blockIdx.y;
  const int m0 = (blockIdx.x * (kNetThreads / 64) + wave) * (16 * kConvMT);
  if (m0 >= cells) return;
  int vx[kConvMT], vy[kConvMT], vz[kConvMT];
#pragma unroll
  for (int t = 0; t < kConvMT; ++t) {
    const int v = m0 + 16 * t + r16;
    vx[t] = v % n;
    vy[t] = (v / n) % n;
    vz[t] = v / (n * n);
  }
  f32x4 acc[kConvMT][NT];
#pragma unroll
  for (int t = 0; t < kConvMT; ++t)
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};

  // operands of K step kb (weights of the NT column tiles, im2col rows of the kConvMT
  // cell tiles); the loads of step kb + 1 are issued before the products of step kb, so
  // that their latency overlaps the matrix-core work (same products, same order)
  auto load = [&](int kb, bf16x8 (&bw)[NT], bf16x8 (&a)[kConvMT]) {
    const int k0 = kb * 32 + 8 * g;
#pragma unroll
    for (int u = 0; u < NT; ++u) bw[u] = ld8(w + (size_t)(16 * u + r16) * Kp + k0);
    if (k0 < K) {
      const int tap = k0 / CI, c = k0 % CI;
      int dx, dy, dz;
      tap_offsets(tap, dx, dy, dz);
#pragma unroll
      for (int t = 0; t < kConvMT; ++t) {
        const int x = vx[t] + dx, y = vy[t] + dy, z = vz[t] + dz;
        const bool in = (unsigned)x < (unsigned)n && (unsigned)y < (unsigned)n &&
                        (unsigned)z < (unsigned)n;
        a[t] = in ? ld8(src_ptr<CI, CA>(src, b, n, x, y, z, c)) : zero8();
      }
    } else {
#pragma unroll
      for (int t = 0; t < kConvMT; ++t) a[t] = zero8();
    }
  };
  auto product = [&](const bf16x8 (&bw)[NT], const bf16x8 (&a)[kConvMT]) {
#pragma unroll
    for (int t = 0; t < kConvMT; ++t)
#pragma unroll
      for (int u = 0; u < NT; ++u) acc[t][u] = mfma(a[t], bw[u], acc[t][u]);
  };
  bf16x8 bw0[NT], a0[kConvMT], bw1[NT], a1[kConvMT];
  load(0, bw0, a0);
  for (int kb = 0; kb < KB; kb += 2) {
    if (kb + 1 < KB) load(kb + 1, bw1, a1);
    product(bw0, a0);
    if (kb + 1 < KB) {
      if (kb + 2 < KB) load(kb + 2, bw0, a0);
      product(bw1, a1);
    }
  }
  const size_t base = (size_t)b * cells;
#pragma unroll
  for (int t = 0; t < kConvMT; ++t)
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int co = 16 * u + r16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const size_t o = (base + m0 + 16 * t + 4 * g + q) * CO + co;
        float val = acc[t][u][q];
        if (EPI == 0) {
          val += bias[co];
          val = val > 0.f ? val : 0.f;
        } else if (mask) {
          if (!(bf2f(mask[o]) > 0.f)) val = 0.f;
        }
        out[o] = f2bf(val);
      }
    }
}

// ---------------------------------------------------------------------------------
// Weight gradient partials: part[chunk][co][k] = sum over the chunk's cells of
// gz[cell][co] * im2col[cell][k].  Grid (batch * chunks, column blocks); a wave owns
// 16 * kWgNT columns and all CO rows and walks the chunk 32 cells at a time (a lane
// takes 8 consecutive cells).  Requires cells % 32 == 0 and chunk_len % 32 == 0.
// ---------------------------------------------------------------------------------
template <int CO, int CI, int CA>
__global__ void __launch_bounds__(kNetThreads)
    k_wgrad(ConvSrc src, const uint16_t* __restrict__ gz, float* __restrict__ part, int n,
            int chunks, int chunk_len) {
  constexpr int K = 27 * CI, Kp = kpad(CI), MT = CO / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int b = blockIdx.x / chunks, ch = blockIdx.x % chunks;
  const int col0 = (blockIdx.y * (kNetThreads / 64) + wave) * 16 * kWgNT;
  if (col0 >= Kp) return;
  const int cells = n * n * n;
  const int v_begin = ch * chunk_len, v_end = min(cells, v_begin + chunk_len);
  // each lane's column of every tile: its tap and channel
  int cdx[kWgNT], cdy[kWgNT], cdz[kWgNT], cc[kWgNT];
  bool cv[kWgNT];
#pragma unroll
  for (int u = 0; u < kWgNT; ++u) {
    const int k = col0 + 16 * u + r16;
    cv[u] = k < K;
    const int tap = cv[u] ? k / CI : 13;
    cc[u] = cv[u] ? k % CI : 0;
    tap_offsets(tap, cdx[u], cdy[u], cdz[u]);
  }
  f32x4 acc[MT][kWgNT];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int u = 0; u < kWgNT; ++u) acc[t][u] = f32x4{0.f, 0.f, 0.f, 0.f};
  const size_t base = (size_t)b * cells;
  const bool row8 = (n & 7) == 0;
  for (int v0 = v_begin; v0 < v_end; v0 += 32) {
    const int vr = v0 + 8 * g;
    const int x0 = vr % n, y = (vr / n) % n, z = vr / (n * n);
    bf16x8 a[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      u16x8 h;
      const uint16_t* p = gz + (base + vr) * CO + 16 * t + r16;
#pragma unroll
      for (int i = 0; i < 8; ++i) h[i] = p[(size_t)i * CO];
      a[t] = __builtin_bit_cast(bf16x8, h);
    }
#pragma unroll
    for (int u = 0; u < kWgNT; ++u) {
      u16x8 h = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (row8) {   // the 8 cells share one x-row
        const int yy = y + cdy[u], zz = z + cdz[u];
        if (cv[u] && (unsigned)yy < (unsigned)n && (unsigned)zz < (unsigned)n) {
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int xx = x0 + i + cdx[u];
            if ((unsigned)xx < (unsigned)n) {
              const uint16_t* p = src_ptr<CI, CA>(src, b, n, xx, yy, zz, cc[u] & ~7);
              h[i] = p[cc[u] & 7];
            }
          }
        }
      } else if (cv[u]) {   // small grids: the run of 8 cells wraps rows
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int v = vr + i;
          const int xx = v % n + cdx[u], yy = (v / n) % n + cdy[u], zz = v / (n * n) + cdz[u];
          if ((unsigned)xx < (unsigned)n && (unsigned)yy < (unsigned)n &&
              (unsigned)zz < (unsigned)n) {
            const uint16_t* p = src_ptr<CI, CA>(src, b, n, xx, yy, zz, cc[u] & ~7);
            h[i] = p[cc[u] & 7];
          }
        }
      }
      const bf16x8 bb = __builtin_bit_cast(bf16x8, h);
#pragma unroll
      for (int t = 0; t < MT; ++t) acc[t][u] = mfma(a[t], bb, acc[t][u]);
    }
  }
  float* o = part + (size_t)blockIdx.x * CO * Kp;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int u = 0; u < kWgNT; ++u) {
      const int k = col0 + 16 * u + r16;
      if (k < Kp)
#pragma unroll
        for (int q = 0; q < 4; ++q) o[(size_t)(16 * t + 4 * g + q) * Kp + k] = acc[t][u][q];
    }
}

// grad[tap][co][c] (c < ci, the layer's real input channels) = sum over the partials
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nparts, int co_n, int kp,
                               int cip, int ci, float* __restrict__ grad) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int kk = 27 * cip;
  if (idx >= co_n * kk) return;
  const int co = idx / kk, k = idx % kk;
  const int tap = k / cip, c = k % cip;
  if (c >= ci) return;
  float s = 0.f;
  for (int q = 0; q < nparts; ++q) s += part[((size_t)q * co_n + co) * kp + k];
  grad[((size_t)tap * co_n + co) * ci + c] = s;
}

// ---------------------------------------------------------------------------------
// per-channel sums (bias gradients): part[block][c] over a range of cells
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(kNetThreads)
    k_chan_sum(const uint16_t* __restrict__ g, int C, size_t ncells, int per_block,
               float* __restrict__ part) {
  __shared__ float red[kNetThreads];
  const int tid = threadIdx.x;
  const int lanes = kNetThreads / C * C;   // threads in use: a multiple of C
  float s = 0.f;
  if (tid < lanes) {
    const int c = tid % C, r = tid / C, rows = lanes / C;
    const size_t v0 = (size_t)blockIdx.x * per_block;
    const size_t v1 = v0 + per_block < ncells ? v0 + per_block : ncells;
    for (size_t v = v0 + r; v < v1; v += rows) s += bf2f(g[v * C + c]);
  }
  red[tid] = s;
  __syncthreads();
  if (tid < C) {
    float t = 0.f;
    for (int q = tid; q < lanes; q += C) t += red[q];
    part[(size_t)blockIdx.x * C + tid] = t;
  }
}

__global__ void k_chan_reduce(const float* __restrict__ part, int nparts, int C,
                              float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  float s = 0.f;
  for (int q = 0; q < nparts; ++q) s += part[(size_t)q * C + c];
  out[c] = s;
}

// ---------------------------------------------------------------------------------
// weight preparation: BF16 copies of the FP32 parameters in the two GEMM layouts
// ---------------------------------------------------------------------------------
// wk[co][k], k = tap * cip + c: W[tap][co][c] for c < ci, zero for padded channels
// and for k >= 27 cip
__global__ void k_prep_fwd(const float* __restrict__ w, int co_n, int ci, int cip, int kp,
                           uint16_t* __restrict__ wk) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= co_n * kp) return;
  const int co = idx / kp, k = idx % kp;
  float v = 0.f;
  if (k < 27 * cip) {
    const int tap = k / cip, c = k % cip;
    if (c < ci) v = w[((size_t)tap * co_n + co) * ci + c];
  }
  wk[idx] = f2bf(v);
}

// data-gradient weights wb[c][k'], k' = tap' * co_n + co: W[26 - tap'][co][c]
__global__ void k_prep_bwd(const float* __restrict__ w, int co_n, int ci, int kp,
                           uint16_t* __restrict__ wb) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ci * kp) return;
  const int c = idx / kp, k = idx % kp;
  float v = 0.f;
  if (k < 27 * co_n) {
    const int tap = 26 - k / co_n, co = k % co_n;
    v = w[((size_t)tap * co_n + co) * ci + c];
  }
  wb[idx] = f2bf(v);
}

// ---------------------------------------------------------------------------------
// glue
// ---------------------------------------------------------------------------------
// 4 input channels -> 8 (the last 4 zero), one thread per cell
__global__ void k_pad_input(const uint16_t* __restrict__ x4, uint16_t* __restrict__ x8,
                            size_t ncells) {
  const size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= ncells) return;
  const uint2 a = *reinterpret_cast<const uint2*>(x4 + 4 * v);
  *reinterpret_cast<u32x4*>(x8 + 8 * v) = u32x4{a.x, a.y, 0u, 0u};
}

// mean of the 8 children, one thread per coarse cell and 8 channels
__global__ void k_pool(const uint16_t* __restrict__ in, int C, int nc, int batch,
                       uint16_t* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int groups = C / 8;
  const size_t cc = (size_t)nc * nc * nc;
  if (idx >= cc * batch * groups) return;
  const int grp = (int)(idx % groups);
  const size_t vc = idx / groups;
  const int b = (int)(vc / cc);
  const int l = (int)(vc % cc);
  const int i = l % nc, j = (l / nc) % nc, k = l / (nc * nc);
  const int nf = 2 * nc;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const size_t v = (size_t)b * nf * nf * nf +
                         ((size_t)(2 * k + dz) * nf + (2 * j + dy)) * nf + (2 * i + dx);
        const u16x8 h = *reinterpret_cast<const u16x8*>(in + v * C + 8 * grp);
#pragma unroll
        for (int q = 0; q < 8; ++q) s[q] += bf2f(h[q]);
      }
  u16x8 o;
#pragma unroll
  for (int q = 0; q < 8; ++q) o[q] = f2bf(s[q] * 0.125f);
  *reinterpret_cast<u16x8*>(out + vc * C + 8 * grp) = o;
}

// gradient through nearest upsampling (sum over the 8 children of channels
// [0, C) of g, whose cells carry CS channels), times (act > 0)
__global__ void k_up_back(const uint16_t* __restrict__ g, int CS, int C, int nc, int batch,
                          const uint16_t* __restrict__ act, uint16_t* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t cc = (size_t)nc * nc * nc;
  if (idx >= cc * batch * C) return;
  const int c = (int)(idx % C);
  const size_t vc = idx / C;
  const int b = (int)(vc / cc), l = (int)(vc % cc);
  const int i = l % nc, j = (l / nc) % nc, k = l / (nc * nc);
  const int nf = 2 * nc;
  float s = 0.f;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const size_t v = (size_t)b * nf * nf * nf +
                         ((size_t)(2 * k + dz) * nf + (2 * j + dy)) * nf + (2 * i + dx);
        s += bf2f(g[v * CS + c]);
      }
  out[idx] = bf2f(act[idx]) > 0.f ? f2bf(s) : (uint16_t)0;
}

// skip-connection gradient plus the gradient through mean pooling:
// out[v][c] = (gs[v][off + c] + gp[parent(v)][c] / 8) * (act[v][c] > 0)
__global__ void k_skip_pool_back(const uint16_t* __restrict__ gs, int CS, int off,
                                 const uint16_t* __restrict__ gp, int C, int nf, int batch,
                                 const uint16_t* __restrict__ act, uint16_t* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t cf = (size_t)nf * nf * nf;
  if (idx >= cf * batch * C) return;
  const int c = (int)(idx % C);
  const size_t v = idx / C;
  const int b = (int)(v / cf), l = (int)(v % cf);
  const int i = l % nf, j = (l / nf) % nf, k = l / (nf * nf);
  const int nc = nf / 2;
  const size_t vc = (size_t)b * nc * nc * nc + ((size_t)(k >> 1) * nc + (j >> 1)) * nc + (i >> 1);
  const float s = bf2f(gs[v * CS + off + c]) + bf2f(gp[vc * C + c]) * 0.125f;
  out[idx] = bf2f(act[idx]) > 0.f ? f2bf(s) : (uint16_t)0;
}

// head: y[v] = hb + sum_c bf16(hw[c]) d1[v][c]
__global__ void k_head_fwd(const uint16_t* __restrict__ d1, const float* __restrict__ hw,
                           size_t ncells, float* __restrict__ y) {
  const size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= ncells) return;
  const u16x8 h0 = *reinterpret_cast<const u16x8*>(d1 + 16 * v);
  const u16x8 h1 = *reinterpret_cast<const u16x8*>(d1 + 16 * v + 8);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += bf2f(f2bf(hw[c])) * bf2f(h0[c]);
#pragma unroll
  for (int c = 0; c < 8; ++c) s += bf2f(f2bf(hw[8 + c])) * bf2f(h1[c]);
  y[v] = s + hw[16];
}

// head backward: gz[v][c] = bf16(dy[v] bf16(hw[c])) (d1[v][c] > 0); block partials of
// sum_v d1[v][c] dy[v] (c < 16) and sum_v dy[v] (slot 16) over per_block cells
__global__ void __launch_bounds__(kNetThreads)
    k_head_bwd(const uint16_t* __restrict__ d1, const float* __restrict__ hw,
               const float* __restrict__ dy, size_t ncells, int per_block,
               uint16_t* __restrict__ gz, float* __restrict__ part) {
  __shared__ float red[17][kNetThreads];
  const int tid = threadIdx.x;
  float acc[17];
#pragma unroll
  for (int c = 0; c < 17; ++c) acc[c] = 0.f;
  float hr[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) hr[c] = bf2f(f2bf(hw[c]));
  const size_t v0 = (size_t)blockIdx.x * per_block;
  const size_t v1 = v0 + per_block < ncells ? v0 + per_block : ncells;
  for (size_t v = v0 + tid; v < v1; v += kNetThreads) {
    const float d = dy[v];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const u16x8 h = *reinterpret_cast<const u16x8*>(d1 + 16 * v + 8 * hh);
      u16x8 o;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const float a = bf2f(h[c]);
        acc[8 * hh + c] += a * d;
        o[c] = a > 0.f ? f2bf(d * hr[8 * hh + c]) : (uint16_t)0;
      }
      *reinterpret_cast<u16x8*>(gz + 16 * v + 8 * hh) = o;
    }
    acc[16] += d;
  }
#pragma unroll
  for (int c = 0; c < 17; ++c) red[c][tid] = acc[c];
  __syncthreads();
  for (int w = kNetThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int c = 0; c < 17; ++c) red[c][tid] += red[c][tid + w];
    __syncthreads();
  }
  if (tid < 17) part[(size_t)blockIdx.x * 17 + tid] = red[tid][0];
}

// loss per sample (one block each): e = y - mean(y) - t, L = sum e^2 / sum t^2,
// dy = 2 (e - mean e) / sum t^2 * inv_batch
__global__ void __launch_bounds__(1024)
    k_loss(const float* __restrict__ y, const float* __restrict__ t, int cells, float inv_batch,
           float* __restrict__ dy, float* __restrict__ loss) {
  __shared__ double red[3][1024];
  const int tid = threadIdx.x, b = blockIdx.x;
  const float* yb = y + (size_t)b * cells;
  const float* tb = t + (size_t)b * cells;
  double sy = 0.0, st = 0.0, stt = 0.0;
  for (int v = tid; v < cells; v += 1024) {
    sy += yb[v];
    st += tb[v];
    stt += (double)tb[v] * tb[v];
  }
  red[0][tid] = sy;
  red[1][tid] = st;
  red[2][tid] = stt;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w)
      for (int q = 0; q < 3; ++q) red[q][tid] += red[q][tid + w];
    __syncthreads();
  }
  const double my = red[0][0] / cells, den = red[2][0];
  __syncthreads();
  double se = 0.0, see = 0.0;
  for (int v = tid; v < cells; v += 1024) {
    const double e = (double)yb[v] - my - tb[v];
    se += e;
    see += e * e;
  }
  red[0][tid] = se;
  red[1][tid] = see;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w)
      for (int q = 0; q < 2; ++q) red[q][tid] += red[q][tid + w];
    __syncthreads();
  }
  const double me = red[0][0] / cells, sc = 2.0 / den * inv_batch;
  if (tid == 0) loss[b] = (float)(red[1][0] / den);
  for (int v = tid; v < cells; v += 1024)
    dy[(size_t)b * cells + v] = (float)(((double)yb[v] - my - tb[v] - me) * sc);
}

// Adam on the FP32 parameters; c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
// Training batch of step `step` (global count): sample j of the batch is sample
// idx(q), q = step * batch + j, of the `count` stored ones: q mod count in order when
// seed == 0, otherwise SplitMix64 (Steele, Lea & Flood 2014) output number q of the
// stream started at `seed`, mod count.  Copies its inputs (4 BF16 channels per cell) and
// target into the network's staging arrays; one thread per (cell, sample).
__device__ inline int64_t train_sample(uint64_t seed, int64_t q, int64_t count) {
  if (seed == 0) return q % count;
  uint64_t z = seed + (uint64_t)(q + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (int64_t)(z % (uint64_t)count);
}

__global__ void __launch_bounds__(256)
    k_gather_samples(const uint2* __restrict__ x, const float* __restrict__ t, int cells,
                     int64_t count, uint64_t seed, int64_t step, int batch,
                     uint2* __restrict__ xs, float* __restrict__ ts) {
  const int j = blockIdx.y;
  const int64_t src = train_sample(seed, step * batch + j, count);
  const size_t so = (size_t)src * cells, dof = (size_t)j * cells;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += gridDim.x * blockDim.x) {
    xs[dof + c] = x[so + c];
    ts[dof + c] = t[so + c];
  }
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, size_t np, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace mppnet
