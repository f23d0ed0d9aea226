// Red-black Gauss-Seidel sweep on the finest level, a pair of cells per thread.
//
// Same semantics as the other fused sweeps (two one-colour half sweeps, out of place):
//   x1  = x_in with every c1 cell set to (sum_f w_f x_in[nb] - h^2 b) / sum_f w_f,
//   out = x1  with every c2 cell set to (sum_f w_f x1[nb]  - h^2 b) / sum_f w_f.
// A block owns a column of 128 x 8 cells and marches up a chunk of planes like the
// z-marching kernel, but each wave owns one row and each lane two cells of it along x,
// one of each colour.  The colour of a lane's first cell is then the same across the
// wave, so neither colour phase diverges, every lane works in both, and the choice of
// cell, neighbour array and LDS row is wave-uniform (scalar registers and branches).
// Each thread keeps b, the interface codes and its own c1 value in registers between
// the phases; x_in (tile + 2-cell ring) and the c1 values (tile + 1-cell ring) go
// through LDS, split by the parity of the column so that a wave reads consecutive
// words.  Cells outside the domain hold zero in both tiles, so the constant-
// coefficient update needs no wall masks: the six neighbour values are summed as they
// are and divided by the number of interior faces.  Loads and stores are raw buffer
// accesses: an offset past the end of the plane reads zero and drops the store, which
// covers cells and planes outside the domain without branches.  The grid size must be
// even (a pair never straddles the domain's edge).
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
constexpr int kPrTX = 128, kPrTY = 8;   // cells of a tile along x and y

inline RbTiles pr_tiles(int n, int kz) {
  RbTiles t;
  t.ntx = (n + kPrTX - 1) / kPrTX;
  t.nty = (n + kPrTY - 1) / kPrTY;
  t.kz = kz;
  t.nkz = (n + kz - 1) / kz;
  t.ntiles = t.ntx * t.nty * t.nkz;
  return t;
}

constexpr unsigned kOob = 0x80000000u;   // a buffer offset past the end of any plane

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
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ inline void buf_st_pair(float2 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ inline void buf_st_pair(double2 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, 0);
}

// FP32: at most 80 VGPRs, three blocks per compute unit; FP64: two (its LDS tiles)
template <typename T>
struct PrWaves {
  static constexpr int value = sizeof(T) == 4 ? 6 : 4;
};


// SH: the operator carries a diagonal shift (F.sig != 0); a compile-time switch, so that
// the unshifted sweep carries no branch on it
template <typename T, int MODE, bool SH>
__global__ void __launch_bounds__(kPrThreads, PrWaves<T>::value)
    k_rb_pair(Faces<T> F, int n, RbTiles tl, const T* __restrict__ rhs, const T* __restrict__ xin,
              const T* __restrict__ ec, T* __restrict__ xout, int c1, Ctl ctl, int dot,
              Sel sel) {
  using V = typename PairOf<T>::V;
  constexpr int TX = kPrTX, TY = kPrTY;
  constexpr int XH = TY + 4, CH = TY + 2;   // rows of the x_in and c1 tiles
  constexpr int XP = TX / 2 + 2;            // pairs per tile row (columns i0 - 2 .. i0 + TX + 1)
  constexpr int XPL = XH * XP, CPL = CH * XP;   // one parity of one plane
  constexpr int XSL = 2 * XPL, CSL = 2 * CPL;   // one plane (slot)
  constexpr unsigned TS = sizeof(T);
  const int b = sel_problem(sel, blockIdx.y);
  if (b < 0) return;
  const int tile = xcd_tile(blockIdx.x, tl.ntiles);
  if (tile < 0) {
    if (dot && threadIdx.x == 0) ctl.partials[(size_t)b * ctl.pstride + blockIdx.x] = 0.0;
    return;
  }
  // x_in and c1 tiles, three planes each: [slot][parity][row][pair]
  __shared__ __align__(16) T sx[3 * XSL];
  __shared__ __align__(16) T sc[3 * CSL];
  const int p = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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
  // diagonal shift times h^2; with a shift every cell takes the coded update
  const T sh2 = F.sig * h2;
  // shifted operator, cell without a crossed face: x = (sum - hr b) / (faces + sig hr)
  const T shr0 = F.sig * hr0, shr1 = F.sig * hr1;
  const T inv6 = T(1) / T(6), inv5 = T(1) / T(5), inv4 = T(1) / T(4), inv3 = T(1) / T(3);
  auto inv_of = [&](int walls) {   // selects, no branches
    T r = inv3;
    r = walls == 2 ? inv4 : r;
    r = walls == 1 ? inv5 : r;
    r = walls <= 0 ? inv6 : r;
    return r;
  };
  const V vzero = {T(0), T(0)};

  // ---- the lane's pair of columns (i, i + 1) and its wave's row j ----
  const int i = i0 + 2 * p;
  const int j = j0 + w;
  const bool col_ok = i < n;
  const bool wx0 = i == 0, wx1 = i + 1 == n - 1;   // x walls of the two cells
  const unsigned own_b = col_ok && j < n ? (unsigned)(i + n * j) * TS : kOob;
  const unsigned own_eb = col_ok && j < n ? (unsigned)((i >> 1) + nc * (j >> 1)) * TS : kOob;

  // ---- a second x_in pair: ring rows j0 - 2, j0 - 1, j0 + TY, j0 + TY + 1 (waves 0..3)
  //      or the ring columns i0 - 2 / i0 + TX of the 12 tile rows (wave 4, lanes 0..23)
  int xr_row = 0, xr_pair = 0;
  unsigned xr_b = kOob, xr_eb = kOob;
  if (w < 5) {
    int gi;
    bool item = true;
    if (w < 4) {
      xr_row = w < 2 ? w : TY + w;
      xr_pair = p + 1;
      gi = i;
    } else {
      item = p < 2 * XH;
      xr_row = item ? p >> 1 : 0;
      xr_pair = (p & 1) ? XP - 1 : 0;
      gi = (p & 1) ? i0 + TX : i0 - 2;
    }
    const int gj = j0 - 2 + xr_row;
    if (item && gi >= 0 && gi < n && gj >= 0 && gj < n) {
      xr_b = (unsigned)(gi + n * gj) * TS;
      xr_eb = (unsigned)((gi >> 1) + nc * (gj >> 1)) * TS;
    }
  }
  // ---- c1 ring: rows j0 - 1 (wave 5) and j0 + TY (wave 6) over the tile's pairs; the
  //      column cells i0 - 1 / i0 + TX of the tile rows (wave 7, lanes 0..TY-1; of the
  //      two, the one of colour c1 on the plane)
  const int rrow = w == 5 ? -1 : TY;    // waves 5 and 6: offset of the ring row from j0
  const int rj = j0 + rrow;
  unsigned rb0 = kOob, rb1 = kOob;      // waves 5, 6: the pair; wave 7: the two cells
  bool rok0 = false, rok1 = false;
  const int cj = j0 + p;                // wave 7: the row of the lane's column cells
  if (w == 5 || w == 6) {
    rok0 = rok1 = col_ok && rj >= 0 && rj < n;
    if (rok0) rb0 = (unsigned)(i + n * rj) * TS;
  } else if (w == 7 && p < TY) {
    rok0 = i0 >= 1 && cj < n;
    rok1 = i0 + TX < n && cj < n;
    if (rok0) rb0 = (unsigned)(i0 - 1 + n * cj) * TS;
    if (rok1) rb1 = (unsigned)(i0 + TX + n * cj) * TS;
  }

  struct XLoad {
    V a, r;     // own pair, second pair
    T ea, er;   // their coarse corrections (MODE 2)
  };
  struct BLoad {
    V bo, br;                // b of the own pair, of the ring pair or the two column cells
    unsigned co, cr0, cr1;   // code bytes: own pair (16 bits), ring pair / column cells
  };
  // every wave issues the same loads in every step (a plane outside the domain or past
  // the chunk has a zero-size resource); results are consumed a step later.  Plane
  // addresses advance by one plane per step (no multiplies in the loop).
  const unsigned code_bytes = (unsigned)nn;
  const char* xq = reinterpret_cast<const char*>(xin + base) + (ptrdiff_t)(k0 - 2) * plane_bytes;
  const char* bq = reinterpret_cast<const char*>(rhs + base) + (ptrdiff_t)(k0 - 1) * plane_bytes;
  const char* cq = reinterpret_cast<const char*>(F.code + base) + (ptrdiff_t)(k0 - 1) * code_bytes;
  char* oq = reinterpret_cast<char*>(xout + base) + (ptrdiff_t)(k0 - 2) * plane_bytes;
  const char* eb = reinterpret_cast<const char*>(ec + basec);
  // pl: plane Lx is inside the domain and needed (the callers test both at once)
  auto issue_x = [&](int Lx, bool pl, XLoad& d) {   // x_in of plane Lx at xq
    if (MODE == 1) return;
    const auto rx = plane_rsrc(xq, pl ? plane_bytes : 0u);
    d.a = buf_ld_pair<T>(rx, own_b);
    if (w < 5) d.r = buf_ld_pair<T>(rx, xr_b);
    if (MODE == 2) {
      const auto re = plane_rsrc(eb + (ptrdiff_t)(pl ? Lx >> 1 : 0) * cplane_bytes,
                                 pl ? cplane_bytes : 0u);
      d.ea = buf_ld<T>(re, own_eb);
      if (w < 5) d.er = buf_ld<T>(re, xr_eb);
    }
  };
  auto commit_x = [&](T* dst, const XLoad& d) {   // into the x_in slot at dst
    if (MODE == 1) return;
    V a = d.a, r = d.r;
    if (MODE == 2) {
      a.x += d.ea;
      a.y += d.ea;
      r.x += d.er;
      r.y += d.er;
    }
    dst[(w + 2) * XP + p + 1] = a.x;
    dst[XPL + (w + 2) * XP + p + 1] = a.y;
    if (w < 4 || (w == 4 && p < 2 * XH)) {
      dst[xr_row * XP + xr_pair] = r.x;
      dst[XPL + xr_row * XP + xr_pair] = r.y;
    }
  };
  auto issue_b = [&](int Lb, bool pl, BLoad& d) {   // b and codes of plane Lb at bq, cq
    const auto rbr = plane_rsrc(bq, pl ? plane_bytes : 0u);
    const auto rcr = plane_rsrc(cq, pl ? code_bytes : 0u);
    d.bo = buf_ld_pair<T>(rbr, own_b);
    d.co = __builtin_amdgcn_raw_buffer_load_b16(rcr, own_b / TS, 0, 0);
    if (w >= 5) {   // one test for the waves without ring work
      if (w < 7) {
        d.br = buf_ld_pair<T>(rbr, rb0);
        d.cr0 = __builtin_amdgcn_raw_buffer_load_b16(rcr, rb0 / TS, 0, 0);
      } else {
        d.br.x = buf_ld<T>(rbr, rb0);
        d.br.y = buf_ld<T>(rbr, rb1);
        d.cr0 = __builtin_amdgcn_raw_buffer_load_b8(rcr, rb0 / TS, 0, 0);
        d.cr1 = __builtin_amdgcn_raw_buffer_load_b8(rcr, rb1 / TS, 0, 0);
      }
    }
  };

  // Gauss-Seidel value of a cell with a crossed face (coefficients from the arrays);
  // pb = index of the cell's plane, off = its offset in the plane
  auto relax_coded = [&](unsigned cd, size_t pb, unsigned off, int ic, int jc, int kc, T xw, T xe,
                         T xs, T xn, T xd, T xu, T bb) -> T {
    T wf[6];
    sweep_faces<T, true>(F, pb + off, cd, ic, jc, kc, n, nn, ir0, ir1, wf);
    T num = T(0);
    num += wf[0] * xw;
    num += wf[1] * xe;
    num += wf[2] * xs;
    num += wf[3] * xn;
    num += wf[4] * xd;
    num += wf[5] * xu;
    const T den = wf[0] + wf[1] + wf[2] + wf[3] + wf[4] + wf[5] + sh2;
    return (num - h2 * bb) / den;
  };
  // Gauss-Seidel value from the six neighbour values (zero outside the domain); inv =
  // 1 / (number of interior faces) for a cell without a crossed face
  auto relax = [&](unsigned cd, size_t pb, unsigned off, int ic, int jc, int kc, T inv, T xw, T xe,
                   T xs, T xn, T xd, T xu, T bb) -> T {
    const T sum = ((xw + xe) + (xs + xn)) + (xd + xu);
    const T hr = (cd & 64u) ? hr1 : hr0;
    T v;
    if (SH) {
      // the face count from the reciprocal the caller passes (1/6, 1/5, 1/4 or 1/3)
      const T cnt = inv == inv6 ? T(6) : (inv == inv5 ? T(5) : (inv == inv4 ? T(4) : T(3)));
      v = (sum - hr * bb) / (cnt + ((cd & 64u) ? shr1 : shr0));
    } else {
      v = (sum - hr * bb) * inv;
    }
    const bool crossed = (cd & 63u) != 0u;
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(crossed) != 0, 0)) {
      if (crossed) v = relax_coded(cd, pb, off, ic, jc, kc, xw, xe, xs, xn, xd, xu, bb);
    }
    return v;
  };

  // 1 / (interior faces) of the lane's two cells on its row, without and with a z wall
  const int wy = (j == 0) + (j == n - 1);
  const T in0 = inv_of(wy + wx0), in1 = inv_of(wy + wx1);
  const T iz0 = inv_of(wy + wx0 + 1), iz1 = inv_of(wy + wx1 + 1);
  const unsigned own_off = (unsigned)(i + n * j);   // cell offset in a plane (crossed path)

  XLoad xl = {vzero, vzero, T(0), T(0)};
  BLoad bn = {vzero, vzero, 0u, 0u, 0u};
  V bprev = vzero;       // b of the own pair on plane L - 1
  unsigned cprev = 0u;   // its codes
  T c1own = T(0), c1prev = T(0);
  double acc = 0.0;
  // LDS slots (element offsets) of planes L - 1, L, L + 1 for the first step L = k0 - 1
  // (as LDS pointers, rotated every step)
  T* xm = sx + ((k0 + 1) % 3) * XSL;
  T* xl0 = sx + ((k0 + 2) % 3) * XSL;
  T* xp = sx + (k0 % 3) * XSL;
  T* cm = sc + ((k0 + 1) % 3) * CSL;
  T* cl0 = sc + ((k0 + 2) % 3) * CSL;
  T* cp = sc + (k0 % 3) * CSL;
  size_t pbL = base + (size_t)(k0 - 1) * nn;   // index of plane L's first cell

  // prologue: x_in of planes k0 - 2 and k0 - 1 into LDS, x_in of k0 and b of k0 - 1 in
  // flight
  if (MODE != 1) {
    XLoad xa = xl, xc = xl;
    issue_x(k0 - 2, (unsigned)(k0 - 2) < (unsigned)n, xa);
    xq += plane_bytes;
    issue_x(k0 - 1, (unsigned)(k0 - 1) < (unsigned)n, xc);
    xq += plane_bytes;
    commit_x(xm, xa);
    commit_x(xl0, xc);
  }
  issue_x(k0, k0 < n, xl);
  xq += plane_bytes;
  issue_b(k0 - 1, (unsigned)(k0 - 1) < (unsigned)n, bn);
  bq += plane_bytes;
  cq += code_bytes;

  const unsigned xlim = (unsigned)min(n, k1 + 2), blim = (unsigned)min(n, k1 + 1);
  // colour parity of the wave's rows on plane L (flips every step) and the LDS element
  // offsets that depend on it, relative to the lane's own x and c1 positions
  int o = (c1 + j + k0 - 1) & 1;
  const int rowx = (w + 2) * XP + p + 1, rowc = (w + 1) * XP + p + 1;
  for (int L = k0 - 1; L <= k1; ++L, o ^= 1) {
    const int x_own = o ? XPL : 0;               // own parity, same pair
    const int x_oth = o ? 0 : XPL - 1;           // other parity, west neighbour's pair
    const int c_own = o ? CPL : 0;
    const int c_oth = o ? 1 : CPL - 1;           // other parity, the x neighbour not in the pair
    commit_x(xp, xl);   // x_in of plane L + 1
    const BLoad cur = bn;
    // planes L + 2 and L + 1 while L < k1, inside the domain
    issue_x(L + 2, (unsigned)(L + 2) < xlim, xl);
    issue_b(L + 1, (unsigned)(L + 1) < blim, bn);
    xq += plane_bytes;
    bq += plane_bytes;
    cq += code_bytes;
    lds_barrier();

    // ---- c1 values of plane L: the wave's row, then the ring ----
    const bool pl = (unsigned)L < (unsigned)n;
    // plane L at a z wall: L == 0 or n - 1 (planes outside the domain also test true;
    // their values are zeroed)
    const bool zwL = (unsigned)(L - 1) >= (unsigned)(n - 2);
    {
      // o: wave-uniform, which cell of the pair
      T xw = T(0), xe = T(0), xs = T(0), xn = T(0), xd = T(0), xu = T(0);
      if (MODE != 1) {
        const T* xo = xl0 + x_oth + rowx;   // other parity, west
        xw = xo[0];
        xe = xo[1];
        const T* xs0 = xl0 + x_own + rowx;
        xs = xs0[-XP];
        xn = xs0[XP];
        xd = xm[x_own + rowx];
        xu = xp[x_own + rowx];
      }
      const T inv = o ? (zwL ? iz1 : in1) : (zwL ? iz0 : in0);
      const T bb = o ? cur.bo.y : cur.bo.x;
      const unsigned cd = (cur.co >> (8 * o)) & 255u;
      T v = relax(cd, pbL, own_off + o, i + o, j, L, inv, xw, xe, xs, xn, xd, xu, bb);
      v = pl && col_ok && j < n ? v : T(0);
      cl0[c_own + rowc] = v;
      c1own = v;
    }
    if (w >= 5) {
      // ring rows j0 - 1 and j0 + TY (waves 5, 6) over the tile's pairs, or the column
      // cells i0 - 1 / i0 + TX (wave 7, lanes 0 .. TY - 1): the cell of colour c1
      int o, ic, jc, par, pr, xr, cr;
      T bb;
      unsigned cd;
      bool ok;
      if (w < 7) {
        o = (c1 + rj + L) & 1;
        ic = i + o;
        jc = rj;
        par = o;
        pr = p + 1;
        xr = rrow + 2;
        cr = rrow + 1;
        bb = o ? cur.br.y : cur.br.x;
        cd = (cur.cr0 >> (8 * o)) & 255u;
        ok = rok0;
      } else {
        o = (c1 + 1 + cj + L) & 1;
        ic = o ? i0 + TX : i0 - 1;
        jc = cj;
        par = o ? 0 : 1;
        pr = o ? XP - 1 : 0;
        xr = p + 2;
        cr = p + 1;
        bb = o ? cur.br.y : cur.br.x;
        cd = o ? cur.cr1 : cur.cr0;
        ok = p < TY && (o ? rok1 : rok0);
      }
      T xw = T(0), xe = T(0), xs = T(0), xn = T(0), xd = T(0), xu = T(0);
      if (MODE != 1 && (w < 7 || p < TY)) {
        // west and east: the other parity, pairs pr - 1 + par and pr + par
        const T* xo = xl0 + (1 - par) * XPL + xr * XP + pr - 1 + par;
        xw = xo[0];
        xe = xo[1];
        const T* xs0 = xl0 + par * XPL + xr * XP + pr;
        xs = xs0[-XP];
        xn = xs0[XP];
        xd = xm[par * XPL + xr * XP + pr];
        xu = xp[par * XPL + xr * XP + pr];
      }
      const int walls = (ic == 0) + (ic == n - 1) + (jc == 0) + (jc == n - 1) + zwL;
      T v = relax(ok ? cd : 0u, pbL, (unsigned)(ic + n * jc), ic, jc, L, inv_of(walls), xw, xe, xs,
                  xn, xd, xu, bb);
      v = pl && ok ? v : T(0);
      if (w < 7 || p < TY) cl0[par * CPL + cr * XP + pr] = v;
    }
    lds_barrier();

    // ---- c2 values of plane L - 1 and the output pair; the store is issued in every
    //      step and dropped outside the chunk and the domain ----
    const int k = L - 1;
    const bool kin = (unsigned)(k - k0) < (unsigned)(k1 - k0);
    {
      const int o2 = o;   // wave-uniform: the c2 cell of the pair on plane k = L - 1
      const bool zwk = (unsigned)(k - 1) >= (unsigned)(n - 2);   // as zwL (k outside: dropped)
      // slot(k) = cm, slot(k - 1) = cp, slot(k + 1) = cl0
      const T* cl = cm + c_own + rowc;
      // the c1 neighbour along x that is not the lane's own c1 cell
      const T xo = cm[c_oth + rowc];
      const T xw = o2 ? c1prev : xo;
      const T xe = o2 ? xo : c1prev;
      const T inv = o2 ? (zwk ? iz1 : in1) : (zwk ? iz0 : in0);
      const T bb = o2 ? bprev.y : bprev.x;
      const unsigned cd = kin ? (cprev >> (8 * o2)) & 255u : 0u;
      const T v2 = relax(cd, pbL - nn, own_off + o2, i + o2, j, k, inv, xw, xe, cl[-XP], cl[XP],
                         cp[c_own + rowc], cl0[c_own + rowc], bb);
      V out;
      out.x = o2 ? c1prev : v2;
      out.y = o2 ? v2 : c1prev;
      buf_st_pair(out, plane_rsrc(oq, kin ? plane_bytes : 0u), own_b);
      // b reads zero outside the domain, so those lanes add nothing
      if (dot && kin) acc += (double)bprev.x * (double)out.x + (double)bprev.y * (double)out.y;
    }
    bprev = cur.bo;
    cprev = cur.co;
    c1prev = c1own;
    oq += plane_bytes;
    pbL += nn;
    // rotate: L - 1 <- L, L <- L + 1, L + 1 <- L + 2
    T* const tx = xm;
    T* const tc = cm;
    xm = xl0;
    xl0 = xp;
    xp = tx;
    cm = cl0;
    cl0 = cp;
    cp = tc;
  }
  if (dot) block_partial(acc, ctl, b);
}

}  // namespace mpp
