// Red-black Gauss-Seidel sweep on the finest level with no block-wide synchronisation:
// a wave owns a whole row of cells (n = 64 C, C cells per lane, contiguous along x) and
// marches up a chunk of planes.  Same semantics and the same arithmetic, term for term,
// as the other fused sweeps:
//   x1  = x_in with every c1 cell set to (sum_f w_f x_in[nb] - h^2 b) / sum_f w_f,
//   out = x1  with every c2 cell set to (sum_f w_f x1[nb]  - h^2 b) / sum_f w_f.
// The c2 update of row j needs the c1 values of rows j - 1 and j + 1, which belong to
// other waves; instead of exchanging them through LDS behind barriers, every wave
// computes them itself from x_in rows j - 2 .. j + 2 (three times the c1 work and five
// row loads per plane, served mostly by the caches: neighbouring waves read the same
// rows at about the same time).  Neighbours along x come from the lane's own cells or,
// at its ends, from the adjacent lanes (cross-lane moves).  Every quantity of a cell
// outside the domain is zero, so the constant-coefficient update needs no wall masks
// except the face count.  The colour pattern of a lane's cells is the same on every
// lane (C is even), so neither colour phase diverges.
#pragma once

#include "rbpair.h"

namespace mpp {

constexpr int kRowWaves = 4;   // waves (rows) per workgroup

struct RowTiles {
  int nty, nkz, kz, ntiles;   // row groups, z-chunks, planes per chunk
};

inline RowTiles row_tiles(int n, int kz) {
  RowTiles t;
  t.nty = (n + kRowWaves - 1) / kRowWaves;
  t.kz = kz;
  t.nkz = (n + kz - 1) / kz;
  t.ntiles = t.nty * t.nkz;
  return t;
}
inline int row_grid(const RowTiles& t) { return 8 * ((t.ntiles + 7) / 8); }

// C consecutive values of type T at a byte offset through a buffer resource (zeros past
// the resource's end)
template <typename T, int C>
struct RowVec {
  T v[C];
};

template <typename T, int C>
__device__ inline RowVec<T, C> row_ld(__amdgpu_buffer_rsrc_t r, unsigned off) {
  RowVec<T, C> out;
  constexpr int bytes = C * (int)sizeof(T);
  static_assert(bytes == 8 || bytes == 16 || bytes == 32, "row load width");
  if constexpr (bytes == 8) {
    const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    __builtin_memcpy(out.v, &u, 8);
  } else if constexpr (bytes == 16) {
    const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    __builtin_memcpy(out.v, &u, 16);
  } else {
    const auto u0 = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    const auto u1 = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0);
    __builtin_memcpy(out.v, &u0, 16);
    __builtin_memcpy(out.v + 16 / sizeof(T), &u1, 16);
  }
  return out;
}

template <typename T, int C>
__device__ inline void row_st(const RowVec<T, C>& x, __amdgpu_buffer_rsrc_t r, unsigned off) {
  constexpr int bytes = C * (int)sizeof(T);
  if constexpr (bytes == 8) {
    u32x2 u;
    __builtin_memcpy(&u, x.v, 8);
    __builtin_amdgcn_raw_buffer_store_b64(u, r, off, 0, 0);
  } else if constexpr (bytes == 16) {
    u32x4 u;
    __builtin_memcpy(&u, x.v, 16);
    __builtin_amdgcn_raw_buffer_store_b128(u, r, off, 0, 0);
  } else {
    u32x4 u0, u1;
    __builtin_memcpy(&u0, x.v, 16);
    __builtin_memcpy(&u1, x.v + 16 / sizeof(T), 16);
    __builtin_amdgcn_raw_buffer_store_b128(u0, r, off, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b128(u1, r, off + 16, 0, 0);
  }
}

template <typename T>
__device__ inline T lane_prev(T v) {   // value of lane - 1 (lane 0: its own)
  return __shfl_up(v, 1, 64);
}
template <typename T>
__device__ inline T lane_next(T v) {   // value of lane + 1 (lane 63: its own)
  return __shfl_down(v, 1, 64);
}

// at least two workgroups (8 waves) per compute unit: up to 256 VGPRs per wave
constexpr int kRowMinBlocks = 2;

template <typename T, int MODE, int C>
__global__ void __launch_bounds__(kRowWaves * 64, kRowMinBlocks)
    k_rb_row(Faces<T> F, int n, RowTiles tl, const T* __restrict__ rhs, const T* __restrict__ xin,
             const T* __restrict__ ec, T* __restrict__ xout, int c1, Ctl ctl, int dot,
             const int* __restrict__ active) {
  using RV = RowVec<T, C>;
  constexpr unsigned TS = sizeof(T);
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int tile = xcd_tile(blockIdx.x, tl.ntiles);
  if (tile < 0) {
    if (dot && threadIdx.x == 0) ctl.partials[(size_t)b * ctl.pstride + blockIdx.x] = 0.0;
    return;
  }
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = (tile % tl.nty) * kRowWaves + w;
  const int k0 = (tile / tl.nty) * tl.kz;
  const int k1 = min(k0 + tl.kz, n);
  const bool jin = j < n;
  const size_t nn = (size_t)n * n;
  const size_t base = (size_t)b * nn * n;
  const int nc = n >> 1;
  const size_t ncc = (size_t)nc * nc;
  const size_t basec = (size_t)b * ncc * nc;
  const unsigned plane_bytes = (unsigned)nn * TS, cplane_bytes = (unsigned)ncc * TS;
  const T h2 = (T)(1.0 / ((double)n * (double)n));
  const T ir0 = F.inv_rho[2 * b], ir1 = F.inv_rho[2 * b + 1];
  const T hr0 = h2 / ir0, hr1 = h2 / ir1;
  const T sh2 = F.sig * h2;
  const bool shifted = sh2 != T(0);
  const T inv6 = T(1) / T(6), inv5 = T(1) / T(5), inv4 = T(1) / T(4), inv3 = T(1) / T(3);
  auto inv_of = [&](int walls) {
    return walls <= 0 ? inv6 : (walls == 1 ? inv5 : (walls == 2 ? inv4 : inv3));
  };
  const int i0 = lane * C;   // the lane's first cell along x

  const T* const xb = xin + base;
  const T* const bbp = rhs + base;
  const uint8_t* const cb = F.code + base;
  const T* const ecb = ec + basec;

  // byte offset of the lane's cells in row r of a plane (kOob outside the domain)
  auto row_off = [&](int r) -> unsigned { return r >= 0 && r < n ? (unsigned)(i0 + n * r) * TS : kOob; };
  // x_in of row r, plane p (zero outside the domain; MODE 1: zero)
  auto load_x = [&](int r, int p) -> RV {
    RV x;
    if (MODE == 1) {
#pragma unroll
      for (int c = 0; c < C; ++c) x.v[c] = T(0);
      return x;
    }
    const bool pl = p >= 0 && p < n;
    const auto rs = plane_rsrc(xb + (ptrdiff_t)(pl ? p : 0) * nn, pl ? plane_bytes : 0u);
    x = row_ld<T, C>(rs, row_off(r));
    if (MODE == 2) {
      // coarse correction, constant over each 2 x 2 x 2 block
      const auto re = plane_rsrc(ecb + (ptrdiff_t)(pl ? p >> 1 : 0) * ncc, pl ? cplane_bytes : 0u);
      const unsigned eo = r >= 0 && r < n ? (unsigned)((i0 >> 1) + nc * (r >> 1)) * TS : kOob;
      T e[C / 2];
      if constexpr (C / 2 == 1) {
        e[0] = buf_ld<T>(re, eo);
      } else {
        const RowVec<T, C / 2> ev = row_ld<T, C / 2>(re, eo);
#pragma unroll
        for (int c = 0; c < C / 2; ++c) e[c] = ev.v[c];
      }
#pragma unroll
      for (int c = 0; c < C; ++c) x.v[c] += e[c >> 1];
    }
    return x;
  };
  auto load_b = [&](int r, int p) -> RV {
    const bool pl = p >= 0 && p < n;
    const auto rs = plane_rsrc(bbp + (ptrdiff_t)(pl ? p : 0) * nn, pl ? plane_bytes : 0u);
    return row_ld<T, C>(rs, row_off(r));
  };
  auto load_code = [&](int r, int p) -> unsigned {
    const bool pl = p >= 0 && p < n;
    const auto rs = plane_rsrc(cb + (ptrdiff_t)(pl ? p : 0) * nn, pl ? (unsigned)nn : 0u);
    const unsigned off = r >= 0 && r < n ? (unsigned)(i0 + n * r) : kOob;
    if constexpr (C == 4) return __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
    else return __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
  };

  // Gauss-Seidel value of one cell from its six neighbour values; the coded update for a
  // cell with a crossed face (or any cell when the operator is shifted)
  auto relax = [&](unsigned cd, int ic, int jc, int kc, T xw, T xe, T xs, T xn, T xd, T xu,
                   T bb) -> T {
    const int walls = (ic == 0) + (ic == n - 1) + (jc == 0) + (jc == n - 1) + (kc == 0) + (kc == n - 1);
    const T sum = ((xw + xe) + (xs + xn)) + (xd + xu);
    const T hr = (cd & 64u) ? hr1 : hr0;
    T v = shifted ? (sum - hr * bb) / (T(6 - walls) + ((cd & 64u) ? F.sig * hr1 : F.sig * hr0))
                  : (sum - hr * bb) * inv_of(walls);
    const bool crossed = (cd & 63u) != 0u;
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(crossed) != 0, 0)) {
      if (crossed) {
        T wf[6];
        sweep_faces<T, true>(F, base + (size_t)kc * nn + (size_t)jc * n + ic, cd, ic, jc, kc, n, nn,
                             ir0, ir1, wf);
        T num = T(0);
        num += wf[0] * xw;
        num += wf[1] * xe;
        num += wf[2] * xs;
        num += wf[3] * xn;
        num += wf[4] * xd;
        num += wf[5] * xu;
        const T den = wf[0] + wf[1] + wf[2] + wf[3] + wf[4] + wf[5] + sh2;
        v = (num - h2 * bb) / den;
      }
    }
    return v;
  };

  // c1 values of row r, plane p (c1 cells only; zero outside the domain): from x_in of
  // the row (xr), the rows r - 1 / r + 1 (xs, xn) and the planes p - 1 / p + 1 (xd, xu)
  auto c1_row = [&](int r, int p, const RV& xr, const RV& xs, const RV& xn, const RV& xd,
                    const RV& xu, const RV& bv, unsigned cd) -> RV {
    RV out;
    const int o = (c1 + r + p) & 1;   // first c1 cell of the lane (wave-uniform)
    // the x neighbours beyond the lane's ends: x_in of the adjacent lanes' edge cells
    // (the cross-lane moves run on every lane; the walls are selected afterwards)
    const T from_prev = lane_prev(xr.v[C - 1]), from_next = lane_next(xr.v[0]);
    const T left = lane == 0 ? T(0) : from_prev;
    const T right = lane == 63 ? T(0) : from_next;
    const bool live = r >= 0 && r < n && p >= 0 && p < n;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      out.v[c] = T(0);
      if ((c & 1) != o) continue;
      const T xw = c > 0 ? xr.v[c - 1] : left;
      const T xe = c < C - 1 ? xr.v[c + 1] : right;
      const T v = relax((cd >> (8 * c)) & 255u, i0 + c, r, p, xw, xe, xs.v[c], xn.v[c], xd.v[c],
                        xu.v[c], bv.v[c]);
      out.v[c] = live ? v : T(0);
    }
    return out;
  };

  // ---- windows: x_in of row j on planes k .. k+2, rows j -/+ 1 on k-1 .. k+1, rows
  //      j -/+ 2 on k; b and codes of row j on k, k+1 and rows j -/+ 1 on k; c1 of row j
  //      on k-1 .. k+1 ----
  const int k = k0;
  RV xj0 = load_x(j, k), xj1 = load_x(j, k + 1), xj2 = load_x(j, k + 2);
  RV xs_m = load_x(j - 1, k - 1), xs_0 = load_x(j - 1, k), xs_p = load_x(j - 1, k + 1);
  RV xn_m = load_x(j + 1, k - 1), xn_0 = load_x(j + 1, k), xn_p = load_x(j + 1, k + 1);
  RV xs2 = load_x(j - 2, k), xn2 = load_x(j + 2, k);
  RV bj0 = load_b(j, k), bj1 = load_b(j, k + 1), bs = load_b(j - 1, k), bn = load_b(j + 1, k);
  unsigned cj0 = load_code(j, k), cj1 = load_code(j, k + 1), cs = load_code(j - 1, k),
           cn = load_code(j + 1, k);
  RV c1m, c1o;
  {
    // c1 of row j on planes k - 1 and k: x_in of row j on k - 2 and k - 1, rows j -/+ 1
    // on k - 1 (already loaded) and k (ditto)
    const RV xjm = load_x(j, k - 1), xjm2 = load_x(j, k - 2);
    const RV bjm = load_b(j, k - 1);
    const unsigned cjm = load_code(j, k - 1);
    c1m = c1_row(j, k - 1, xjm, xs_m, xn_m, xjm2, xj0, bjm, cjm);
    c1o = c1_row(j, k, xj0, xs_0, xn_0, xjm, xj1, bj0, cj0);
  }
  const char* oq = reinterpret_cast<const char*>(xout + base);
  double acc = 0.0;
  for (int kk = k0; kk < k1; ++kk) {
    // loads of the next step: x_in row j on kk+3, rows j -/+ 1 on kk+2, rows j -/+ 2 on
    // kk+1; b and codes of row j on kk+2, rows j -/+ 1 on kk+1
    const bool more = kk + 1 < k1;
    RV nxj3 = {}, nxs = {}, nxn = {}, nxs2 = {}, nxn2 = {}, nbj2 = {}, nbs = {}, nbn = {};
    unsigned ncj2 = 0u, ncs = 0u, ncn = 0u;
    if (more) {
      nxj3 = load_x(j, kk + 3);
      nxs = load_x(j - 1, kk + 2);
      nxn = load_x(j + 1, kk + 2);
      nxs2 = load_x(j - 2, kk + 1);
      nxn2 = load_x(j + 2, kk + 1);
      nbj2 = load_b(j, kk + 2);
      nbs = load_b(j - 1, kk + 1);
      nbn = load_b(j + 1, kk + 1);
      ncj2 = load_code(j, kk + 2);
      ncs = load_code(j - 1, kk + 1);
      ncn = load_code(j + 1, kk + 1);
    }
    // c1 of row j on kk + 1 and of rows j -/+ 1 on kk
    const RV c1u = c1_row(j, kk + 1, xj1, xs_p, xn_p, xj0, xj2, bj1, cj1);
    const RV c1s = c1_row(j - 1, kk, xs_0, xs2, xj0, xs_m, xs_p, bs, cs);
    const RV c1n = c1_row(j + 1, kk, xn_0, xj0, xn2, xn_m, xn_p, bn, cn);
    // c2 cells of row j on kk and the output row
    {
      const int o2 = ((c1 + j + kk) & 1) ^ 1;
      const T from_prev = lane_prev(c1o.v[C - 1]), from_next = lane_next(c1o.v[0]);
      const T left = lane == 0 ? T(0) : from_prev;
      const T right = lane == 63 ? T(0) : from_next;
      RV out;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if ((c & 1) != o2) {
          out.v[c] = c1o.v[c];
          continue;
        }
        const T xw = c > 0 ? c1o.v[c - 1] : left;
        const T xe = c < C - 1 ? c1o.v[c + 1] : right;
        out.v[c] = relax(jin ? (cj0 >> (8 * c)) & 255u : 0u, i0 + c, j, kk, xw, xe, c1s.v[c],
                         c1n.v[c], c1m.v[c], c1u.v[c], bj0.v[c]);
      }
      row_st<T, C>(out, plane_rsrc(oq + (ptrdiff_t)kk * plane_bytes, plane_bytes), row_off(j));
      if (dot && jin) {
#pragma unroll
        for (int c = 0; c < C; ++c) acc += (double)bj0.v[c] * (double)out.v[c];
      }
    }
    // rotate the windows by one plane
    c1m = c1o;
    c1o = c1u;
    xj0 = xj1;
    xj1 = xj2;
    xj2 = nxj3;
    xs_m = xs_0;
    xs_0 = xs_p;
    xs_p = nxs;
    xn_m = xn_0;
    xn_0 = xn_p;
    xn_p = nxn;
    xs2 = nxs2;
    xn2 = nxn2;
    bj0 = bj1;
    bj1 = nbj2;
    bs = nbs;
    bn = nbn;
    cj0 = cj1;
    cj1 = ncj2;
    cs = ncs;
    cn = ncn;
  }
  if (dot) block_partial(acc, ctl, b);
}

}  // namespace mpp
