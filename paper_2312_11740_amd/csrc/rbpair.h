// Red-black Gauss-Seidel sweep on the finest level, a pair of cells per thread.
//
// Same semantics as the other fused sweeps (two one-colour half sweeps, out of place):
//   x1  = x_in with every c1 cell set to (sum_f w_f x_in[nb] - h^2 b) / sum_f w_f,
//   out = x1  with every c2 cell set to (sum_f w_f x1[nb]  - h^2 b) / sum_f w_f.
// A block owns a column of TX x TY cells (TX = 2 PW) and marches up a chunk of planes
// like the z-marching kernel, but a thread owns two cells along x, one of each colour:
// with one wave per row (PW = 64) the colour of the first cell of every pair in a wave
// is the same, so neither colour phase diverges and every lane does useful work in
// both.  Each thread keeps b, the interface code and its own c1 value in registers
// between the phases; only x_in (tile + 2-cell ring) and the c1 values (tile + 1-cell
// ring) go through LDS.  Cells outside the domain hold zero in both LDS tiles, so the
// constant-coefficient update needs no wall masks: the neighbour sum is taken as is
// and divided by the number of interior faces.  Pairs are loaded and stored as one
// 8- or 16-byte access; the grid size must be even.
#pragma once

#include "rbgs.h"

namespace mpp {

template <typename T>
struct PairOf;
template <>
struct PairOf<float> {
  using V = float2;
};
template <>
struct PairOf<double> {
  using V = double2;
};

constexpr int kPrThreads = 512;
constexpr int kPrWaves = kPrThreads / 64;
constexpr int kPrRing0 = 320;   // first thread of the c1-ring items (waves 5..7)

template <int PW>
struct PrShape {
  static constexpr int TX = 2 * PW;               // cells along x
  static constexpr int TY = kPrWaves * (64 / PW); // rows
  static constexpr int XW = TX + 4, XH = TY + 4;  // x_in tile with a 2-cell ring
  static constexpr int CW = TX + 2, CH = TY + 2;  // c1 tile with a 1-cell ring
  static constexpr int NX = XW * XH, NC = CW * CH;
  static constexpr int XE = 4 * PW + 2 * XH;      // pairs of the x_in ring
  static constexpr int RE = 2 * PW + TY;          // c1 cells of the ring
  static_assert(XE <= kPrThreads && RE <= kPrThreads - kPrRing0, "ring items per thread");
};

template <int PW>
inline RbTiles pr_tiles(int n, int kz) {
  RbTiles t;
  t.ntx = (n + PrShape<PW>::TX - 1) / PrShape<PW>::TX;
  t.nty = (n + PrShape<PW>::TY - 1) / PrShape<PW>::TY;
  t.kz = kz;
  t.nkz = (n + kz - 1) / kz;
  t.ntiles = t.ntx * t.nty * t.nkz;
  return t;
}

// Buffer resource of one plane of an array (stride 0, num_records bytes): raw buffer
// accesses at offsets >= num_records read zero and drop stores, which handles cells
// outside the domain (offset kOob) and planes outside the domain (num_records = 0)
// without branches.
constexpr unsigned kOob = 0x80000000u;

__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ inline T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ inline float buf_ld<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ inline double buf_ld<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <typename T>
__device__ inline typename PairOf<T>::V buf_ld_pair(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ inline float2 buf_ld_pair<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ inline double2 buf_ld_pair<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
template <typename T>
__device__ inline void buf_st_pair(typename PairOf<T>::V v, __amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ inline void buf_st_pair<float>(float2 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                        off, 0, 0);
}
template <>
__device__ inline void buf_st_pair<double>(double2 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b128(
      __builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r, off, 0, 0);
}

// FP32: 64 VGPRs so that four blocks (32 waves) share a compute unit; FP64 is held to
// two blocks by its LDS tiles anyway
template <typename T>
struct PrWaves {
  static constexpr int value = sizeof(T) == 4 ? 6 : 4;
};

template <typename T, int MODE, int PW>
__global__ void __launch_bounds__(kPrThreads, PrWaves<T>::value)
    k_rb_pair(Faces<T> F, int n, RbTiles tl, const T* __restrict__ rhs, const T* __restrict__ xin,
              const T* __restrict__ ec, T* __restrict__ xout, int c1, Ctl ctl, int dot,
              const int* __restrict__ active) {
  using Sh = PrShape<PW>;
  using V = typename PairOf<T>::V;
  constexpr int TX = Sh::TX, TY = Sh::TY, XW = Sh::XW, CW = Sh::CW;
  constexpr unsigned TS = sizeof(T);
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int tile = xcd_tile(blockIdx.x, tl.ntiles);
  if (tile < 0) {
    if (dot && threadIdx.x == 0) ctl.partials[(size_t)b * ctl.pstride + blockIdx.x] = 0.0;
    return;
  }
  __shared__ __align__(16) T sx[3][Sh::NX];
  __shared__ __align__(16) T sc[3][Sh::NC];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i0 = (tile % tl.ntx) * TX;
  const int j0 = ((tile / tl.ntx) % tl.nty) * TY;
  const int k0 = (tile / (tl.ntx * tl.nty)) * tl.kz;
  const int k1 = min(k0 + tl.kz, n);
  const size_t nn = (size_t)n * n;
  const size_t base = (size_t)b * nn * n;
  const int nc = n >> 1;
  const size_t ncc = (size_t)nc * nc;
  const size_t basec = (size_t)b * ncc * nc;
  const unsigned plane_bytes = (unsigned)nn * TS, cplane_bytes = (unsigned)ncc * TS;
  const T h2 = (T)(1.0 / ((double)n * (double)n));
  const T ir0 = F.inv_rho[2 * b], ir1 = F.inv_rho[2 * b + 1];
  const T hr0 = h2 / ir0, hr1 = h2 / ir1;
  const T inv6 = T(1) / T(6), inv5 = T(1) / T(5), inv4 = T(1) / T(4), inv3 = T(1) / T(3);
  const V vzero = {T(0), T(0)};

  // ---- the thread's own pair: cells (i, j) and (i + 1, j) ----
  const int pp = lane % PW;
  const int jj = wave * (64 / PW) + lane / PW;
  const int i = i0 + 2 * pp, j = j0 + jj;
  const bool own_ok = i < n && j < n;
  const unsigned own_b = own_ok ? (unsigned)(i + n * j) * TS : kOob;   // byte offset in a plane
  const unsigned own_eb = own_ok ? (unsigned)((i >> 1) + nc * (j >> 1)) * TS : kOob;
  const int own_x = (jj + 2) * XW + 2 * pp + 2;   // first cell in the x_in tile
  const int own_c = (jj + 1) * CW + 2 * pp + 1;   // first cell in the c1 tile
  const int wj = (j == 0) + (j == n - 1);
  const int wx0 = (i == 0) + wj, wx1 = (i + 1 == n - 1) + wj;   // walls in x and y

  // ---- one pair of the x_in ring (threads below XE; the others read nothing) ----
  unsigned xr_b = kOob, xr_eb = kOob;
  int xr_l = 0;
  const bool xr_item = tid < Sh::XE;
  if (xr_item) {
    int xrow, xcol;
    if (tid < 4 * PW) {
      const int r = tid / PW;
      xrow = r < 2 ? r : TY + r;
      xcol = 2 * (tid % PW) + 2;
    } else {
      const int q = tid - 4 * PW;
      xrow = q >> 1;
      xcol = (q & 1) ? TX + 2 : 0;
    }
    const int gi = i0 - 2 + xcol, gj = j0 - 2 + xrow;
    if (gi >= 0 && gi < n && gj >= 0 && gj < n) {
      xr_b = (unsigned)(gi + n * gj) * TS;
      xr_eb = (unsigned)((gi >> 1) + nc * (gj >> 1)) * TS;
    }
    xr_l = xrow * XW + xcol;
  }

  // ---- one c1 cell of the ring (threads kPrRing0 .. kPrRing0 + RE - 1): rows j0 - 1
  //      and j0 + TY over the tile's pairs (one pair loaded, o picks the cell), or the
  //      cells i0 - 1 and i0 + TX of a tile row (both loaded, o picks the one of colour
  //      c1 on the plane); o = (r_oadd + L) & 1
  const int rq = tid - kPrRing0;
  const bool r_item = rq >= 0 && rq < Sh::RE;
  int r_oadd = 0, r_step = 1, r_i = 0, r_j = 0, r_c = 0, r_x = 0;
  bool r_ok0 = false, r_ok1 = false;
  unsigned r_b0 = kOob, r_b1 = kOob;   // byte offsets of the first and second value
  if (r_item) {
    if (rq < 2 * PW) {
      const int row = rq < PW ? -1 : TY;
      const int q2 = 2 * (rq % PW);
      r_j = j0 + row;
      r_i = i0 + q2;
      r_ok0 = r_ok1 = r_j >= 0 && r_j < n && r_i < n;
      r_oadd = c1 + r_j;
      r_step = 1;
      r_c = (row + 1) * CW + q2 + 1;
      r_x = (row + 2) * XW + q2 + 2;
      if (r_ok0) {
        r_b0 = (unsigned)(r_i + n * r_j) * TS;
        r_b1 = r_b0 + TS;
      }
    } else {
      const int row = rq - 2 * PW;
      r_j = j0 + row;
      r_i = i0 - 1;
      r_ok0 = i0 >= 1 && r_j < n;
      r_ok1 = i0 + TX < n && r_j < n;
      r_oadd = c1 + 1 + r_j;
      r_step = TX + 1;
      r_c = (row + 1) * CW;
      r_x = (row + 2) * XW + 1;
      if (r_ok0) r_b0 = (unsigned)(i0 - 1 + n * r_j) * TS;
      if (r_ok1) r_b1 = (unsigned)(i0 + TX + n * r_j) * TS;
    }
  }
  const int rwj = (r_j == 0) + (r_j == n - 1);

  // ---- loads: every thread issues the same instructions in every step (absent values
  //      read zero), results are consumed a step later, nothing is combined on arrival
  struct XLoad {
    V a, r;     // own pair, ring pair
    T ea, er;   // coarse corrections of the two (MODE 2)
  };
  struct BLoad {
    V bo;              // b of the own pair
    unsigned co;       // its two code bytes
    T rb0, rb1;        // b of the ring cell(s)
    unsigned rc0, rc1; // their code bytes
  };
  auto issue_x = [&](int Lx, bool live, XLoad& d) {
    if (MODE == 1) return;
    const bool pl = live && Lx >= 0 && Lx < n;
    const int Lc = pl ? Lx : 0;
    const auto rx = plane_rsrc(xin + base + (size_t)Lc * nn, pl ? plane_bytes : 0u);
    d.a = buf_ld_pair<T>(rx, own_b);
    d.r = buf_ld_pair<T>(rx, xr_b);
    if (MODE == 2) {
      const auto re = plane_rsrc(ec + basec + (size_t)(Lc >> 1) * ncc, pl ? cplane_bytes : 0u);
      d.ea = buf_ld<T>(re, own_eb);
      d.er = buf_ld<T>(re, xr_eb);
    }
  };
  auto commit_x = [&](int Lx, const XLoad& d) {
    if (MODE == 1) return;
    T* dst = sx[(Lx + 3) % 3];
    V a = d.a, r = d.r;
    if (MODE == 2) {
      a.x += d.ea;
      a.y += d.ea;
      r.x += d.er;
      r.y += d.er;
    }
    *reinterpret_cast<V*>(dst + own_x) = a;
    if (xr_item) *reinterpret_cast<V*>(dst + xr_l) = r;
  };
  auto issue_b = [&](int Lb, bool live, BLoad& d) {
    const bool pl = live && Lb >= 0 && Lb < n;
    const int Lc = pl ? Lb : 0;
    const auto rbr = plane_rsrc(rhs + base + (size_t)Lc * nn, pl ? plane_bytes : 0u);
    const auto rcr = plane_rsrc(F.code + base + (size_t)Lc * nn, pl ? (unsigned)nn : 0u);
    d.bo = buf_ld_pair<T>(rbr, own_b);
    d.co = __builtin_amdgcn_raw_buffer_load_b16(rcr, own_b / TS, 0, 0);
    d.rb0 = buf_ld<T>(rbr, r_b0);
    d.rb1 = buf_ld<T>(rbr, r_b1);
    d.rc0 = __builtin_amdgcn_raw_buffer_load_b8(rcr, r_b0 / TS, 0, 0);
    d.rc1 = __builtin_amdgcn_raw_buffer_load_b8(rcr, r_b1 / TS, 0, 0);
  };

  // Gauss-Seidel value of cell (ic, jc, kc) from its six neighbour values (zero outside
  // the domain); walls = number of its faces on the domain boundary
  auto relax = [&](unsigned cd, int ic, int jc, int kc, int walls, T xw, T xe, T xs, T xn, T xd,
                   T xu, T bb) -> T {
    if ((cd & 63u) == 0u) {
      const T sum = ((xw + xe) + (xs + xn)) + (xd + xu);
      const T inv = walls == 0 ? inv6 : (walls == 1 ? inv5 : (walls == 2 ? inv4 : inv3));
      const T hr = (cd & 64u) ? hr1 : hr0;
      return (sum - hr * bb) * inv;
    }
    T w[6];
    const size_t cell = base + (size_t)kc * nn + (size_t)jc * n + ic;
    sweep_faces<T, true>(F, cell, cd, ic, jc, kc, n, nn, ir0, ir1, w);
    T num = T(0);
    num += w[0] * xw;
    num += w[1] * xe;
    num += w[2] * xs;
    num += w[3] * xn;
    num += w[4] * xd;
    num += w[5] * xu;
    const T den = w[0] + w[1] + w[2] + w[3] + w[4] + w[5];
    return (num - h2 * bb) / den;
  };

  // c1 value of one cell on plane L (LDS indices cx in the x_in tile, cc in the c1
  // tile), zero when the cell is outside the domain
  auto c1_cell = [&](bool ok, int L, int ic, int jc, int walls, int cx, int cc, T bb,
                     unsigned cd) -> T {
    T v = T(0);
    if (ok) {
      const T* xl = sx[(L + 3) % 3];
      T xw = T(0), xe = T(0), xs = T(0), xn = T(0), xd = T(0), xu = T(0);
      if (MODE != 1) {
        xw = xl[cx - 1];
        xe = xl[cx + 1];
        xs = xl[cx - XW];
        xn = xl[cx + XW];
        xd = sx[(L + 2) % 3][cx];
        xu = sx[(L + 4) % 3][cx];
      }
      v = relax(cd, ic, jc, L, walls + (L == 0) + (L == n - 1), xw, xe, xs, xn, xd, xu, bb);
    }
    sc[(L + 3) % 3][cc] = v;
    return v;
  };

  XLoad xl = {vzero, vzero, T(0), T(0)};
  BLoad bn = {vzero, 0u, T(0), T(0), 0u, 0u}, bc = bn, bp = bn;
  T c1own = T(0), c1prev = T(0);
  double acc = 0.0;

  // prologue: x_in of planes k0 - 2 and k0 - 1 into LDS, x_in of k0 and b of k0 - 1 in
  // flight
  if (MODE != 1) {
    XLoad x0 = xl, x1 = xl;
    issue_x(k0 - 2, true, x0);
    issue_x(k0 - 1, true, x1);
    commit_x(k0 - 2, x0);
    commit_x(k0 - 1, x1);
  }
  issue_x(k0, true, xl);
  issue_b(k0 - 1, true, bn);

  for (int L = k0 - 1; L <= k1; ++L) {
    commit_x(L + 1, xl);
    bp = bc;
    bc = bn;
    // the last step loads nothing (zero-size resources) but issues the same instructions
    issue_x(L + 2, L < k1, xl);
    issue_b(L + 1, L < k1, bn);
    lds_barrier();

    // ---- c1 values of plane L: the own pair's c1 cell, then one ring cell ----
    const bool pl = L >= 0 && L < n;
    {
      const int o = (c1 + j + L) & 1;
      c1own = c1_cell(pl && own_ok, L, i + o, j, o ? wx1 : wx0, own_x + o, own_c + o,
                      o ? bc.bo.y : bc.bo.x, (bc.co >> (8 * o)) & 255u);
    }
    if (r_item) {
      const int o = (r_oadd + L) & 1;
      const int ic = r_i + o * r_step;
      const bool ok = pl && (o ? r_ok1 : r_ok0);
      const int walls = (ic == 0) + (ic == n - 1) + rwj;
      c1_cell(ok, L, ic, r_j, walls, r_x + o * r_step, r_c + o * r_step, o ? bc.rb1 : bc.rb0,
              o ? bc.rc1 : bc.rc0);
    }
    lds_barrier();

    // ---- c2 values of plane L - 1 and the output pair; the store is issued in every
    //      step and dropped outside the chunk and the domain ----
    const int k = L - 1;
    const bool kin = k >= k0 && k < k1;
    {
      const int o2 = ((c1 + j + k) & 1) ^ 1;
      const int kk = kin ? k : k0;
      const T* cl = sc[(kk + 3) % 3];
      const int q = own_c + o2;
      const T xw = o2 ? c1prev : cl[q - 1];
      const T xe = o2 ? cl[q + 1] : c1prev;
      const T bb = o2 ? bp.bo.y : bp.bo.x;
      const unsigned cd = kin ? (bp.co >> (8 * o2)) & 255u : 0u;
      const T v2 = relax(cd, i + o2, j, kk, (o2 ? wx1 : wx0) + (kk == 0) + (kk == n - 1), xw, xe,
                         cl[q - CW], cl[q + CW], sc[(kk + 2) % 3][q], sc[(kk + 4) % 3][q], bb);
      V out;
      out.x = o2 ? c1prev : v2;
      out.y = o2 ? v2 : c1prev;
      buf_st_pair<T>(out, plane_rsrc(xout + base + (size_t)kk * nn, kin ? plane_bytes : 0u), own_b);
      // b reads zero outside the domain, so those lanes add nothing
      if (dot && kin) acc += (double)bp.bo.x * (double)out.x + (double)bp.bo.y * (double)out.y;
    }
    c1prev = c1own;
  }
  if (dot) block_partial(acc, ctl, b);
}

}  // namespace mpp
