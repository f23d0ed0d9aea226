// Host side of the gfx950 pressure-projection library: the C ABI of include/mpp.h,
// workspace layout, the multigrid hierarchy and the preconditioned CG drivers.
//
// All device memory lives in the caller's workspace; the host keeps only the
// operator handle and a few polling mirrors.  Control returns to the host every
// `check_every` CG iterations to read the per-problem `active` flags, which the
// kernels themselves maintain (convergence, iteration cap and breakdown are decided
// on the device by the last block of each reduction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "guess.h"
#include "levelset.h"
#include "heat.h"
#include "amr.h"
#include "blocks.h"
#include "deflate.h"
#include "kernels.h"
#include "net_internal.h"
#include "project.h"
#include "rbgs.h"
#include "rbgs3d.h"
#include "rbpair.h"
#include "stencil.h"

using namespace mpp;

namespace {

struct HipError {
  hipError_t e;
};

inline void ck(hipError_t e) {
  if (e != hipSuccess) throw HipError{e};
}

inline void ck_launch() { ck(hipGetLastError()); }

// multigrid level sizes: halve while even and > 4
int level_sizes(int n, int* sizes) {
  int L = 0;
  sizes[L++] = n;
  while (n % 2 == 0 && n > 4 && L < kMaxLevels) {
    n /= 2;
    sizes[L++] = n;
  }
  return L;
}

bool desc_ok(const mpp_desc* d) {
  if (!d || d->n < 2 || d->n > 1024 || d->batch < 1 || d->batch > 65535 ||
      (d->flags & ~(uint32_t)MPP_FLAG_NO_GRAPHS) != 0)
    return false;
  int sizes[kMaxLevels];
  const int L = level_sizes(d->n, sizes);
  const int nc = sizes[L - 1];
  if (nc * nc * nc > kMaxCoarse) return false;
  return true;
}

int blocks_per_problem(size_t cells, int B) {
  const size_t need = (cells + kBlock - 1) / kBlock;
  const size_t cap = std::max<size_t>(1, 8192 / (size_t)B);
  return (int)std::max<size_t>(1, std::min(need, cap));
}

// Sequential carve-out of the workspace, 256-byte aligned pieces.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Lays out every device buffer of an operator; with base == nullptr only sizes.
size_t layout(mpp_op_s* op, const mpp_desc* d, char* base) {
  Carver cv{base};
  const int B = d->batch;
  int sizes[kMaxLevels];
  const int L = level_sizes(d->n, sizes);
  op->n = d->n;
  op->batch = B;
  op->nlev = L;
  op->cells = (size_t)d->n * d->n * d->n;
  const size_t C = op->cells * B;
  op->pstride = 0;
  for (int l = 0; l < L; ++l) {
    Level& lv = op->lev[l];
    lv.n = sizes[l];
    lv.cells = (size_t)sizes[l] * sizes[l] * sizes[l];
    const size_t cl = lv.cells * B;
    lv.bpp = blocks_per_problem(lv.cells, B);
    op->pstride = std::max(op->pstride, lv.bpp);
    if (l == 0) lv.code = cv.take<uint8_t>(cl);
    for (int a = 0; a < 3; ++a) lv.f64[a] = cv.take<double>(cl + 64);
    for (int a = 0; a < 3; ++a) lv.f32[a] = cv.take<float>(cl + 64);
    if (l > 0) {
      lv.b64 = cv.take<double>(cl);
      lv.x64 = cv.take<double>(cl);
      lv.t64 = cv.take<double>(cl);
      lv.b32 = cv.take<float>(cl);
      lv.x32 = cv.take<float>(cl);
      lv.t32 = cv.take<float>(cl);
    }
  }
  const int m = sizes[L - 1] * sizes[L - 1] * sizes[L - 1];
  op->coarse_m = m;
  op->coarse_inv = cv.take<double>((size_t)B * m * m);
  op->coarse_work = cv.take<double>((size_t)B * m * m);
  op->rho = cv.take<double>((size_t)B * 3);
  op->inv_rho64 = cv.take<double>((size_t)B * 2);
  op->inv_rho32 = cv.take<float>((size_t)B * 2);
  op->kappa = cv.take<double>(C);
  op->jterm = cv.take<double>(C);
  op->x = cv.take<double>(C);
  op->b = cv.take<double>(C);
  op->r = cv.take<double>(C);
  op->z = cv.take<double>(C);
  op->p = cv.take<double>(C);
  op->q = cv.take<double>(C);
  op->r32 = cv.take<float>(C);
  op->z32 = cv.take<float>(C);
  op->p32 = cv.take<float>(C);
  op->q32 = cv.take<float>(C);
  op->d32 = cv.take<float>(C);
  for (int l = 0; l < L; ++l) {   // every sweep kernel the tuner may pick
    for (int kz = 2; kz <= 2 * kRbKZ; kz *= 2)
      op->pstride = std::max(op->pstride, rb_grid(rb_tiles(sizes[l], B, kz)));
    for (int shape = 0; shape < k3Shapes; ++shape)
      op->pstride = std::max(op->pstride, grid3(tiles3(sizes[l], shape)));
    for (int kz = 2; kz <= 2 * kRbKZ; kz *= 2) {
      op->pstride = std::max(op->pstride, rb_grid(pr_tiles(sizes[l], kz)));
    }
  }
  for (int kz = 2; kz <= kStKZ; kz *= 2)   // every chunk size st_kz may pick
    op->pstride = std::max(op->pstride, st_grid(st_tiles(sizes[0], kz)));
  // the learned guess's sum and dot share a pass: two sets of finest-level partials
  op->pstride = std::max(op->pstride, 2 * op->lev[0].bpp);
  // the band correction of a deflated CG appends its partials after a producer's
  op->pstride += kDefBandBlocks;
  op->partials = cv.take<double>((size_t)B * op->pstride);
  // deflation: region ids, the band (capacity one eighth of the cells), E and its inverse
  {
    Defl& D = op->defl;
    D.cap = (int)(op->cells / 8 + 64);
    D.lcap = (int)(op->cells / 4 + 64);
    D.pcap = std::max(kDefBandBlocks, kDefRegionBlocks);
    D.lab = cv.take<uint8_t>(C);
    D.light = cv.take<int>((size_t)B * D.lcap);
    D.lcount = cv.take<int>((size_t)B);
    D.bcell = cv.take<int>((size_t)B * D.cap);
    D.blab = cv.take<uint32_t>((size_t)B * D.cap);
    D.bval = cv.take<double>((size_t)B * D.cap * kDefPairs);
    D.bcount = cv.take<int>((size_t)B);
    D.k = cv.take<int>((size_t)B);
    D.einv = cv.take<double>((size_t)B * kDefMax * kDefMax);
    D.zb = cv.take<double>((size_t)B * kDefMax);
    D.coef = cv.take<double>((size_t)B * kDefMax);
    D.part = cv.take<double>((size_t)B * D.pcap * kDefMax);
    op->defl_e = cv.take<double>((size_t)B * kDefMax * kDefMax);
    op->defl_light = cv.take<int>((size_t)B);
    op->defl_flag = cv.take<int>((size_t)kCclBatch * B);
    op->defl_total = cv.take<int>((size_t)B);
    op->defl_over = cv.take<int>((size_t)B);
  }
  op->tail_mask = cv.take<int>((size_t)B);
  op->live = cv.take<int>((size_t)B + 1);
  op->rows = B;
  op->counters = cv.take<unsigned>((size_t)B);
  for (Ctl* c : {&op->outer, &op->inner}) {
    c->scal = cv.take<double>((size_t)B * kSlots);
    c->active = cv.take<int>((size_t)B);
    c->iters = cv.take<int>((size_t)B);
    c->status = cv.take<int>((size_t)B);
    c->partials = op->partials;
    c->counters = op->counters;
    c->pstride = op->pstride;
    c->list = nullptr;
  }
  return cv.off + 256;
}

template <typename T>
Faces<T> faces_of(const mpp_op_s* op, int l);

// The shift halves per coarser level: with mean restriction and piecewise-constant
// prolongation the coarse operator (faces = means of the fine ones at twice the spacing)
// is half the Galerkin product, and the Galerkin product keeps a shift unchanged.
inline double level_shift(const mpp_op_s* op, int l) { return std::ldexp(op->shift, -l); }

template <>
Faces<double> faces_of<double>(const mpp_op_s* op, int l) {
  const Level& lv = op->lev[l];
  return Faces<double>{l == 0 ? lv.code : nullptr, lv.f64[0], lv.f64[1], lv.f64[2], op->inv_rho64,
                       level_shift(op, l)};
}
template <>
Faces<float> faces_of<float>(const mpp_op_s* op, int l) {
  const Level& lv = op->lev[l];
  return Faces<float>{l == 0 ? lv.code : nullptr, lv.f32[0], lv.f32[1], lv.f32[2], op->inv_rho32,
                      (float)level_shift(op, l)};
}

template <typename T> T* lvl_b(Level& L);
template <typename T> T* lvl_x(Level& L);
template <> double* lvl_b<double>(Level& L) { return L.b64; }
template <> double* lvl_x<double>(Level& L) { return L.x64; }
template <typename T> T* lvl_t(Level& L);
template <> double* lvl_t<double>(Level& L) { return L.t64; }
template <> float* lvl_t<float>(Level& L) { return L.t32; }
template <> float* lvl_b<float>(Level& L) { return L.b32; }
template <> float* lvl_x<float>(Level& L) { return L.x32; }

inline dim3 grid_of(const Level& lv, int B) { return dim3(lv.bpp, B); }

// block rows of a launch: every problem's, or with a list the rows of the CG iterations
inline int rows_of(const mpp_op_s* op, const int* list) { return list ? op->rows : op->batch; }

EpiArgs epi(int kind) {
  EpiArgs e{};
  e.kind = kind;
  e.only_active = (kind == E_RZ || kind == E_PQ || kind == E_RR_ITER) ? 1 : 0;
  return e;
}

// Adds the block partials of the preceding producer launch per problem and runs the
// epilogue (one block per problem).
void finish_sums(mpp_op_s* op, const Ctl& ctl, const EpiArgs& e, int nparts, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(rows_of(op, ctl.list)), dim3(1024), 0, s, ctl, nparts, e);
  ck_launch();
}

// ------------------------------------------------------------------------------
// finest-level streaming kernels (grid = XCD-ordered tiles of 64 x 4 columns)
// ------------------------------------------------------------------------------
// y = A x on the finest level, with x.y block partials when dot; returns the number
// of partials written (0 without dot).
// z-chunk of the column-marching stencil kernels: 16 planes, shorter (down to 2) while
// the grid would have fewer than 2048 blocks (small grids are latency-bound and want
// every compute unit)
int st_kz(int n, int batch) {
  int kz = kStKZ;
  while (kz > 2 && (long)st_tiles(n, kz).ntiles * batch < 2048) kz /= 2;
  return kz;
}

template <typename T>
int launch_apply(const mpp_op_s* op, Faces<T> F, const T* x, T* y, const Ctl& ctl, int dot,
                 Sel sel, hipStream_t s) {
  const int n = op->lev[0].n, rows = rows_of(op, sel.list);
  const int kz = st_kz(n, rows);
  const StTiles tl = st_tiles(n, kz);
  const dim3 grid(st_grid(tl), rows);
  hipLaunchKernelGGL((k_stencil_z<T, 0>), grid, dim3(kStThreads), 0, s, F, n, tl, kz, x,
                     (const T*)nullptr, y, ctl, dot, 0, sel);
  return dot ? (int)grid.x : 0;
}

// r = rhs - A x (x = 0 when xzero) with ||r||^2 block partials; returns their number.
template <typename T>
int launch_residual(const mpp_op_s* op, Faces<T> F, const T* rhs, const T* x, T* r,
                    const Ctl& ctl, int xzero, hipStream_t s) {
  if (xzero) {   // r = rhs: a streaming copy
    const Level& L0 = op->lev[0];
    hipLaunchKernelGGL(k_copy_sq<T>, grid_of(L0, op->batch), dim3(kBlock), 0, s, rhs, r,
                       (int)L0.cells, ctl);
    return L0.bpp;
  }
  const int n = op->lev[0].n;
  const int kz = st_kz(n, op->batch);
  const StTiles tl = st_tiles(n, kz);
  const dim3 grid(st_grid(tl), op->batch);
  hipLaunchKernelGGL((k_stencil_z<T, 1>), grid, dim3(kStThreads), 0, s, F, n, tl, kz, x, rhs,
                     r, ctl, 1, xzero, Sel{});
  return (int)grid.x;
}

// coarse rhs of level l+1 from the residual of level l
template <typename T>
void launch_resid_restrict(const mpp_op_s* op, int l, Faces<T> F, const T* rhs, const T* x, T* bc,
                           Sel sel, hipStream_t s) {
  const int n = op->lev[l].n, rows = rows_of(op, sel.list);
  const int kz = st_kz(n, rows);
  const StTiles tl = st_tiles(n, kz);
  const dim3 grid(st_grid(tl), rows);
  if (l == 0)
    hipLaunchKernelGGL((k_resid_restrict_z<T, true>), grid, dim3(kStThreads), 0, s, F, n, tl, kz,
                       rhs, x, bc, sel);
  else
    hipLaunchKernelGGL((k_resid_restrict_z<T, false>), grid, dim3(kStThreads), 0, s, F, n, tl, kz,
                       rhs, x, bc, sel);
}

// ------------------------------------------------------------------------------
// profiler: HIP events around launches
// ------------------------------------------------------------------------------
const char* kKernelNames[kKernelIds] = {
    "apply_dot", "residual", "smooth_colour", "resid_restrict", "prolong_add",  "dot",
    "update_p",  "update_xr", "coarse_vcycle", "apply",        "rb_sweep_zero", "rb_sweep",
    "rb_sweep_prolong", "heat_apply", "heat_residual", "heat_jacobi", "deflation"};

hipEvent_t prof_event(Prof& P) {
  if (P.used == P.pool.size()) {
    hipEvent_t e;
    ck(hipEventCreate(&e));
    P.pool.push_back(e);
  }
  return P.pool[P.used++];
}

// Folds finished records into the totals (the stream must be synchronised).
void prof_collect(Prof& P) {
  for (const ProfRec& r : P.recs) {
    float ms = 0.f;
    ck(hipEventElapsedTime(&ms, r.a, r.b));
    P.ms[r.kid] += ms;
    P.bytes[r.kid] += r.bytes;
    P.launches[r.kid] += 1;
  }
  P.recs.clear();
  P.used = 0;
}

template <class F>
void timed(mpp_op_s* op, int kid, double bytes, hipStream_t s, F&& launch) {
  Prof& P = op->prof;
  if (!P.on) {
    launch();
    return;
  }
  hipEvent_t a = prof_event(P), b = prof_event(P);
  ck(hipEventRecord(a, s));
  launch();
  ck(hipEventRecord(b, s));
  P.recs.push_back(ProfRec{kid, a, b, bytes});
}

// Algorithmic bytes of one launch on the finest level: every array the kernel must
// touch, once; S = bytes per value, per cell of every problem.
double alg_bytes(const mpp_op_s* op, int kid, size_t S) {
  const double cells = (double)op->cells * op->batch;
  const double s = (double)S;
  switch (kid) {
    case K_APPLY_DOT: case K_APPLY: return cells * (2 * s + 1);   // x, y, code
    case K_RESIDUAL: return cells * (3 * s + 1);                  // b, x, r, code
    case K_SMOOTH: return cells * (2.5 * s + 1);                  // x, b, half of x, code
    case K_RESID_RESTRICT: return cells * (2 * s + s / 8 + 1);    // b, x, coarse b, code
    case K_PROLONG: return cells * (2 * s + s / 8);               // x (r+w), coarse x
    case K_DOT: return cells * 2 * s;
    case K_UPDATE_P: return cells * 3 * s;
    case K_UPDATE_XR: return cells * 6 * s;
    case K_RB_ZERO: return cells * (2 * s + 1);                   // b, code, out
    case K_RB: return cells * (3 * s + 1);                        // x_in, b, code, out
    case K_RB_PROLONG: return cells * (3 * s + s / 8 + 1);        // + coarse correction
    case K_HEAT_APPLY: return cells * (2 * s + 1);                // p, q, code
    case K_HEAT_RESIDUAL: return cells * (3 * s + 1);             // b, x, r, code
    case K_HEAT_JACOBI: return cells * (2 * s + 1);               // r, z, code
    default: return 0.0;
  }
}

template <typename T> const T* lvl_f(const Level& L, int a);
template <> const double* lvl_f<double>(const Level& L, int a) { return L.f64[a]; }
template <> const float* lvl_f<float>(const Level& L, int a) { return L.f32[a]; }

// ------------------------------------------------------------------------------
// V-cycle: z ~= A^{-1} r, zero initial guess
// ------------------------------------------------------------------------------
template <typename T> T* level0_tmp(mpp_op_s* op);
template <> double* level0_tmp<double>(mpp_op_s* op) { return op->q; }
template <> float* level0_tmp<float>(mpp_op_s* op) { return op->q32; }

template <typename T>
void vcycle(mpp_op_s* op, int l, const T* rhs, T* x, int nu, Sel sel, hipStream_t s,
            const Ctl* dctl = nullptr, int* dot_parts = nullptr);

// One fused sweep on level l with the kernel the tuner picked for it: kz > 0 the
// z-marching kernel with chunks of kz planes (0: its default), kz = -1, -2, -3 the
// 3D-tile kernel with tile shape 0, 1, 2, kz <= -4 the pair-per-thread kernel with
// chunks of -kz planes (finest level, even n).  Returns the grid size (the number of dot
// partials).
template <typename T, int MODE, bool FINE>
int launch_rb(const mpp_op_s* op, int l, int kz, const Faces<T>& F, const T* rhs, const T* in,
              const T* ec, T* out, int c1, const Ctl& ctl, int dot, Sel sel,
              hipStream_t s) {
  const int n = op->lev[l].n, B = rows_of(op, sel.list);
  if (kz <= -4) {
    if constexpr (FINE) {
      if (n % 2 == 0) {
        const RbTiles tl = pr_tiles(n, -kz);
        const dim3 grid(rb_grid(tl), B);
        if (F.sig != T(0))
          hipLaunchKernelGGL((k_rb_pair<T, MODE, true>), grid, dim3(kPrThreads), 0, s, F, n, tl,
                             rhs, in, ec, out, c1, ctl, dot, sel);
        else
          hipLaunchKernelGGL((k_rb_pair<T, MODE, false>), grid, dim3(kPrThreads), 0, s, F, n, tl,
                             rhs, in, ec, out, c1, ctl, dot, sel);
        return (int)grid.x;
      }
    }
    throw HipError{hipErrorInvalidValue};   // the pair kernel only runs on an even finest level
  }
  if (kz < 0) {
    const int shape = -kz - 1;
    const Tiles3 t3 = tiles3(n, shape);
    const dim3 grid(grid3(t3), B);
    if (shape == 0)
      hipLaunchKernelGGL((k_rb_sweep3d<T, MODE, FINE, 0>), grid, dim3(Shape3<0>::Threads), 0, s,
                         F, n, t3, rhs, in, ec, out, c1, ctl, dot, sel);
    else if (shape == 1)
      hipLaunchKernelGGL((k_rb_sweep3d<T, MODE, FINE, 1>), grid, dim3(Shape3<1>::Threads), 0, s,
                         F, n, t3, rhs, in, ec, out, c1, ctl, dot, sel);
    else
      hipLaunchKernelGGL((k_rb_sweep3d<T, MODE, FINE, 2>), grid, dim3(Shape3<2>::Threads), 0, s,
                         F, n, t3, rhs, in, ec, out, c1, ctl, dot, sel);
    return (int)grid.x;
  }
  const RbTiles tl = rb_tiles(n, op->batch, kz);
  const dim3 grid(rb_grid(tl), B);
  hipLaunchKernelGGL((k_rb_sweep<T, MODE, FINE>), grid, dim3(kRbThreads), 0, s, F, n, tl, rhs, in,
                     ec, out, c1, ctl, dot, sel);
  return (int)grid.x;
}

// A level with fused sweeps: 2 nu out-of-place sweeps alternate between x and a
// scratch array so that the last one lands in x; the prolongation is folded into the
// first post-smoothing sweep and r.z (b.x) into the last one when dot_parts is given.
template <typename T>
void vcycle_fused(mpp_op_s* op, int l, const T* rhs, T* x, int nu, Sel sel,
                  hipStream_t s, const Ctl* dctl, int* dot_parts) {
  Level& L = op->lev[l];
  Level& Lc = op->lev[l + 1];
  const Faces<T> F = faces_of<T>(op, l);
  T* tmp = l == 0 ? level0_tmp<T>(op) : lvl_t<T>(L);
  const int kz = op->tail ? op->kz_tail[sizeof(T) == 4][l] : op->kz[sizeof(T) == 4][l];
  const Ctl ctl = dctl ? *dctl : op->outer;
  const bool fine = l == 0;
  int nparts = 0;
  auto dst = [&](int sw) { return ((2 * nu - 1 - sw) % 2 == 0) ? x : tmp; };
  auto launch = [&](int sw, const T* in, int c1, int mode, int dot) {
    const T* ecv = lvl_x<T>(Lc);
#define MPP_RB(MD, FN) \
  nparts = launch_rb<T, MD, FN>(op, l, kz, F, rhs, in, ecv, dst(sw), c1, ctl, dot, sel, s)
    if (fine) {
      if (mode == 1) MPP_RB(1, true); else if (mode == 2) MPP_RB(2, true); else MPP_RB(0, true);
    } else {
      if (mode == 1) MPP_RB(1, false); else if (mode == 2) MPP_RB(2, false); else MPP_RB(0, false);
    }
#undef MPP_RB
  };
  auto sweep = [&](int sw, const T* in, int c1, int mode, int dot) {
    const int kid = mode == 1 ? K_RB_ZERO : (mode == 2 ? K_RB_PROLONG : K_RB);
    if (fine)
      timed(op, kid, alg_bytes(op, kid, sizeof(T)), s, [&] { launch(sw, in, c1, mode, dot); });
    else
      launch(sw, in, c1, mode, dot);
    ck_launch();
  };
  sweep(0, nullptr, 0, 1, 0);
  for (int q = 1; q < nu; ++q) sweep(q, dst(q - 1), 0, 0, 0);
  const T* xpre = dst(nu - 1);
  auto restrict_ = [&] { launch_resid_restrict<T>(op, l, F, rhs, xpre, lvl_b<T>(Lc), sel, s); };
  if (fine)
    timed(op, K_RESID_RESTRICT, alg_bytes(op, K_RESID_RESTRICT, sizeof(T)), s, restrict_);
  else
    restrict_();
  ck_launch();
  if (fine)
    timed(op, K_COARSE_VCYCLE, 0.0, s,
          [&] { vcycle<T>(op, 1, lvl_b<T>(Lc), lvl_x<T>(Lc), op->nu_c, sel, s); });
  else
    vcycle<T>(op, l + 1, lvl_b<T>(Lc), lvl_x<T>(Lc), op->nu_c, sel, s);
  const int want = dot_parts ? 1 : 0;
  sweep(nu, xpre, 1, 2, (nu == 1) ? want : 0);
  for (int q = nu + 1; q < 2 * nu; ++q) sweep(q, dst(q - 1), 1, 0, (q == 2 * nu - 1) ? want : 0);
  if (dot_parts) *dot_parts = nparts;
}

template <typename T>
void vcycle(mpp_op_s* op, int l, const T* rhs, T* x, int nu, Sel sel, hipStream_t s,
            const Ctl* dctl, int* dot_parts) {
  Level& L = op->lev[l];
  const int B = rows_of(op, sel.list);
  if (dot_parts) *dot_parts = 0;
  if (l < op->nlev - 1 && L.cells > (size_t)kSmallCells) {
    vcycle_fused<T>(op, l, rhs, x, nu, sel, s, l == 0 ? dctl : nullptr,
                    l == 0 ? dot_parts : nullptr);
    return;
  }
  // this level and everything below: one workgroup per problem, one launch
  SmallCycle<T> S{};
  S.nlev = op->nlev - l;
  for (int q = 0; q < S.nlev; ++q) {
    Level& Lq = op->lev[l + q];
    S.lv[q] = SmallLevel<T>{Lq.n, lvl_f<T>(Lq, 0), lvl_f<T>(Lq, 1), lvl_f<T>(Lq, 2),
                            q == 0 ? const_cast<T*>(rhs) : lvl_b<T>(Lq), q == 0 ? x : lvl_x<T>(Lq),
                            (T)level_shift(op, l + q)};
  }
  S.inv = op->coarse_inv;
  S.m = op->coarse_m;
  S.nu = l == 0 ? nu : op->nu_c;
  // x, b, reciprocal diagonals and one residual scratch always fit (<= 4681 cells in at
  // most 3 levels, 16^3 first level: 145 KB in FP64); the faces too in FP32
  size_t fixed = 0, fb = 0;
  small_lds_bytes(S, fixed, fb);
  if (fixed > (size_t)kSmallLdsBytes || S.nlev > 3 || S.m > kSmallBlock)
    throw HipError{hipErrorInvalidValue};
  if (fixed + fb <= (size_t)kSmallLdsBytes)
    hipLaunchKernelGGL((k_small_cycle<T, true>), dim3(B), dim3(kSmallBlock), 0, s, S, sel);
  else
    hipLaunchKernelGGL((k_small_cycle<T, false>), dim3(B), dim3(kSmallBlock), 0, s, S, sel);
  ck_launch();
}

// ------------------------------------------------------------------------------
// tile autotuning: the sweep kernel of each level (z-marching with a z-chunk of 2 .. 32
// planes, or 3D tiles loaded at once) is timed with HIP events the first time a shape
// is solved in a precision, and cached for the process by (n, batch, precision, level
// size)
// ------------------------------------------------------------------------------
struct TuneKey {
  int n, batch, tsize, nl, tail;
  bool operator<(const TuneKey& o) const {
    if (n != o.n) return n < o.n;
    if (batch != o.batch) return batch < o.batch;
    if (tsize != o.tsize) return tsize < o.tsize;
    if (nl != o.nl) return nl < o.nl;
    return tail < o.tail;
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;

template <typename T>
void ensure_tuned(mpp_op_s* op, hipStream_t s) {
  const int w = sizeof(T) == 4;
  if (op->tuned[w]) return;
  op->tuned[w] = true;
  const char* env = std::getenv("MPP_AUTOTUNE");
  if (env && env[0] == '0') {
    for (int l = 0; l < op->nlev; ++l) op->kz_tail[w][l] = op->kz[w][l];
    return;
  }
  // MPP_SWEEP=march, =tile[S] or =pair[K] fixes the sweep kernel of every level (no
  // timing; tile: the 3D-tile kernel with tile shape S (default 0); pair: the pair kernel
  // with K-plane chunks (default 16) on an even finest level, z-marching below)
  const char* force = std::getenv("MPP_SWEEP");
  if (force && (std::strcmp(force, "march") == 0 || std::strncmp(force, "tile", 4) == 0 ||
                std::strncmp(force, "pair", 4) == 0)) {
    const int shape = force[0] == 't' ? std::min(std::max(std::atoi(force + 4), 0), k3Shapes - 1)
                                      : 0;
    for (int l = 0; l < op->nlev; ++l) op->kz[w][l] = force[0] == 't' ? -1 - shape : 0;
    if (force[0] == 'p' && op->lev[0].n % 2 == 0) {
      const int kz = std::atoi(force + 4);
      op->kz[w][0] = -(kz >= 4 && kz <= 2 * kRbKZ ? kz : 16);
    }
    for (int l = 0; l < op->nlev; ++l) op->kz_tail[w][l] = op->kz[w][l];
    return;
  }
  const int B = op->batch;
  // the tail schedule is timed with problem 0 alone active, listed on one row
  if (B > 1) {
    hipLaunchKernelGGL(k_int_fill, dim3((B + 255) / 256), dim3(256), 0, s, op->tail_mask, B, 0);
    hipLaunchKernelGGL(k_int_fill, dim3(1), dim3(1), 0, s, op->tail_mask, 1, 1);
    hipLaunchKernelGGL(k_live_list, dim3(1), dim3(1024), 0, s, (const int*)op->tail_mask, B,
                       op->live);
    ck_launch();
  }
  hipEvent_t e0, e1;
  ck(hipEventCreate(&e0));
  ck(hipEventCreate(&e1));
  for (int l = 0; l + 1 < op->nlev; ++l)
   for (int tail = 0; tail < (B > 1 ? 2 : 1); ++tail) {
    Level& L = op->lev[l];
    if (L.cells <= (size_t)kSmallCells) break;
    int* slot = tail ? &op->kz_tail[w][l] : &op->kz[w][l];
    const Sel mask = tail ? Sel{op->tail_mask, op->live} : Sel{};
    op->rows = tail ? 1 : B;
    const TuneKey key{op->n, B, (int)sizeof(T), L.n, tail};
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        *slot = it->second;
        continue;
      }
    }
    // time MODE-0 sweeps on zeroed level buffers (contents do not change the cost)
    T* in = l == 0 ? (T*)(w ? (void*)op->z32 : (void*)op->z) : lvl_x<T>(L);
    T* out = l == 0 ? level0_tmp<T>(op) : lvl_t<T>(L);
    const T* rhs = l == 0 ? (const T*)(w ? (void*)op->r32 : (void*)op->r) : lvl_b<T>(L);
    const dim3 g1 = grid_of(L, B);
    hipLaunchKernelGGL(k_fill<T>, g1, dim3(kBlock), 0, s, in, (int)L.cells, T(0));
    hipLaunchKernelGGL(k_fill<T>, g1, dim3(kBlock), 0, s, const_cast<T*>(rhs), (int)L.cells, T(0));
    ck_launch();
    // timed on the unshifted operator, whatever the operator's current use: the choice
    // is cached per shape and shared by pressure and heat solves
    Faces<T> F = faces_of<T>(op, l);
    F.sig = T(0);
    float best = 1e30f;
    int best_kz = 0;
    // candidates: the z-marching kernel with chunks of 2 .. 32 planes, the 3D-tile kernel
    // in its three tile shapes, on an even finest level the pair kernel with chunks of
    // 4 .. 32 planes
    std::vector<int> cands;
    for (int kz = 2; kz <= 2 * kRbKZ && kz <= L.n; kz *= 2) cands.push_back(kz);
    for (int shape = 0; shape < k3Shapes; ++shape) cands.push_back(-1 - shape);
    if (l == 0 && L.n % 2 == 0)
      for (int kz = 4; kz <= 2 * kRbKZ && kz <= L.n; kz *= 2) cands.push_back(-kz);
    // two rounds over the candidates, each candidate's better round counts (a single
    // round of three launches let clock and cache noise pick a slower chunk size)
    std::vector<float> cand_ms(cands.size(), 1e30f);
    for (int round = 0; round < 2; ++round)
      for (size_t ci = 0; ci < cands.size(); ++ci) {
        const int kz = cands[ci];
        auto launch = [&] {
          if (l == 0)
            launch_rb<T, 0, true>(op, l, kz, F, rhs, in, (const T*)nullptr, out, 0, op->outer, 0,
                                  mask, s);
          else
            launch_rb<T, 0, false>(op, l, kz, F, rhs, in, (const T*)nullptr, out, 0, op->outer,
                                   0, mask, s);
        };
        launch();
        ck(hipEventRecord(e0, s));
        for (int q = 0; q < 3; ++q) launch();
        ck(hipEventRecord(e1, s));
        ck_launch();
        ck(hipEventSynchronize(e1));
        float ms = 0.f;
        ck(hipEventElapsedTime(&ms, e0, e1));
        cand_ms[ci] = std::min(cand_ms[ci], ms);
      }
    for (size_t ci = 0; ci < cands.size(); ++ci)
      if (cand_ms[ci] < best) {
        best = cand_ms[ci];
        best_kz = cands[ci];
      }
    *slot = best_kz;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune.emplace(key, best_kz);   // the first tuning of a shape wins
    *slot = g_tune[key];
  }
  op->rows = B;
  if (B == 1)
    for (int l = 0; l < op->nlev; ++l) op->kz_tail[w][l] = op->kz[w][l];
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

bool any_active(mpp_op_s* op, const Ctl& ctl, hipStream_t s) {
  ck(hipMemcpyAsync(op->h_active, ctl.active, sizeof(int) * op->batch, hipMemcpyDeviceToHost, s));
  ck(hipStreamSynchronize(s));
  if (op->prof.on) prof_collect(op->prof);
  for (int b = 0; b < op->batch; ++b)
    if (op->h_active[b]) return true;
  return false;
}


// ------------------------------------------------------------------------------
// launch graphs: a block of CG iterations is captured once per operator and
// argument set and replayed (no memset nodes: every buffer a replay relies on is
// written by kernels)
// ------------------------------------------------------------------------------
template <class F>
void run_graph(mpp_op_s* op, const GraphKey& key, hipStream_t s, F&& enqueue) {
  for (GraphEntry& g : op->graphs)
    if (g.key == key) {
      ck(hipGraphLaunch(g.exec, s));
      return;
    }
  if (!op->cap_stream) ck(hipStreamCreateWithFlags(&op->cap_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  ck(hipStreamBeginCapture(op->cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    enqueue(op->cap_stream);
  } catch (...) {
    hipGraph_t g2 = nullptr;
    (void)hipStreamEndCapture(op->cap_stream, &g2);
    if (g2) (void)hipGraphDestroy(g2);
    throw;
  }
  ck(hipStreamEndCapture(op->cap_stream, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    throw HipError{e};
  }
  op->graphs.push_back(GraphEntry{key, graph, exec});
  ck(hipGraphLaunch(exec, s));
}

// ------------------------------------------------------------------------------
// deflation of the light-phase regions (deflate.h): built at the first deflated solve
// after a build or update, from the operator's faces; host syncs are part of the build
// ------------------------------------------------------------------------------
void build_deflation(mpp_op_s* op, hipStream_t s) {
  op->defl_ready = true;
  op->defl_any = false;
  const int B = op->batch;
  op->h_defl_k.assign(B, 0);
  Defl& D = op->defl;
  const dim3 gb((B + 255) / 256);
  hipLaunchKernelGGL(k_int_fill, gb, dim3(256), 0, s, D.k, B, 0);
  hipLaunchKernelGGL(k_int_fill, gb, dim3(256), 0, s, D.bcount, B, 0);
  hipLaunchKernelGGL(k_int_fill, gb, dim3(256), 0, s, D.lcount, B, 0);
  ck_launch();
  bool want = false;
  for (int b = 0; b < B; ++b) want = want || op->h_defl_light[b] >= 0;
  if (!want) return;
  const Level& L0 = op->lev[0];
  const int n = op->n, cells = (int)L0.cells;
  // the CG vectors are free between solves: labels and compaction counts live there
  int* lab = reinterpret_cast<int*>(op->q);
  int* counts = reinterpret_cast<int*>(op->z);
  std::vector<int> h(B);
  auto to_host = [&](const int* d) {
    ck(hipMemcpyAsync(h.data(), d, sizeof(int) * B, hipMemcpyDeviceToHost, s));
    ck(hipStreamSynchronize(s));
  };
  ck(hipMemcpyAsync(op->defl_light, op->h_defl_light.data(), sizeof(int) * B,
                    hipMemcpyHostToDevice, s));
  // Counts stay on the device: kernels over the light list read its length there and
  // are launched for the largest list the workspace holds (grid-stride loops, or chunks
  // past the end that do nothing), so the host waits only for the labelling rounds and
  // once at the end.
  // the light cells in cell order (a problem with more than lcap of them: not deflated)
  const int nblk = (cells + kDefChunk - 1) / kDefChunk;
  hipLaunchKernelGGL(k_light_count, dim3(nblk, B), dim3(kDefThreads), 0, s, L0.code, cells,
                     op->defl_light, counts, nblk);
  hipLaunchKernelGGL(k_scan_counts, dim3(B), dim3(1024), 0, s, counts, nblk, op->defl_total);
  hipLaunchKernelGGL(k_light_write, dim3(nblk, B), dim3(kDefThreads), 0, s, L0.code, cells,
                     op->defl_light, counts, op->defl_total, nblk, D.light, D.lcap);
  hipLaunchKernelGGL(k_light_done, gb, dim3(256), 0, s, D.lcount, op->defl_total, op->defl_light,
                     D.lcap, B);
  ck_launch();
  const int lblk = std::min(512, (D.lcap + 255) / 256);
  op->defl_rblk = std::min(kDefRegionBlocks, (D.lcap + 255) / 256);
  // propagation rounds over the light cells in batches of kCclBatch, each round with its
  // own changed flag, until the last round of a batch changed nothing (labels only
  // decrease, so this ends; the cap is a guard)
  hipLaunchKernelGGL(k_ccl_init, dim3(lblk, B), dim3(256), 0, s, D.light, D.lcount, D.lcap, cells,
                     lab);
  ck_launch();
  const dim3 gf((kCclBatch * B + 255) / 256);
  for (int round = 0; round < 65536; round += kCclBatch) {
    hipLaunchKernelGGL(k_int_fill, gf, dim3(256), 0, s, op->defl_flag, kCclBatch * B, 0);
    for (int t = 0; t < kCclBatch; ++t)
      hipLaunchKernelGGL(k_ccl_round, dim3(lblk, B), dim3(256), 0, s, n, L0.code, op->defl_light,
                         D.light, D.lcount, D.lcap, lab,
                         t ? (const int*)op->defl_flag + (size_t)(t - 1) * B : (const int*)nullptr,
                         op->defl_flag + (size_t)t * B);
    ck_launch();
    to_host(op->defl_flag + (size_t)(kCclBatch - 1) * B);
    bool changed = false;
    for (int b = 0; b < B; ++b) changed = changed || h[b] != 0;
    if (!changed) break;
  }
  // the first kDefMax components of each problem (by smallest cell index) become
  // regions 1..k
  const int nblk_l = (D.lcap + kDefChunk - 1) / kDefChunk;
  hipLaunchKernelGGL(k_root_count, dim3(nblk_l, B), dim3(kDefThreads), 0, s, lab, cells, D.light,
                     D.lcount, D.lcap, counts, nblk_l);
  hipLaunchKernelGGL(k_scan_counts, dim3(B), dim3(1024), 0, s, counts, nblk_l, op->defl_total);
  hipLaunchKernelGGL(k_root_mark, dim3(nblk_l, B), dim3(kDefThreads), 0, s, lab, cells, D.light,
                     D.lcount, D.lcap, counts, nblk_l);
  hipLaunchKernelGGL(k_u8_fill, dim3(1024), dim3(256), 0, s, D.lab, op->cells * B);
  hipLaunchKernelGGL(k_region_ids, dim3(lblk, B), dim3(256), 0, s, lab, cells, D.light, D.lcount,
                     D.lcap, D.lab);
  hipLaunchKernelGGL(k_regions_done, gb, dim3(256), 0, s, D.k, op->defl_total, D.lcount, B);
  hipLaunchKernelGGL(k_int_fill, gb, dim3(256), 0, s, op->defl_over, B, 0);
  ck_launch();
  // the band in cell order, E = Z^T A Z, its inverse; a problem that does not fit is
  // not deflated
  const Faces<double> F = faces_of<double>(op, 0);
  // (the labels of the propagation are done with: their array holds the band mask)
  uint8_t* mask = reinterpret_cast<uint8_t*>(lab);
  hipLaunchKernelGGL(k_u8_fill, dim3(1024), dim3(256), 0, s, mask, op->cells * B);
  hipLaunchKernelGGL(k_band_mark, dim3(lblk, B), dim3(256), 0, s, D.lab, n, D.light, D.lcount,
                     D.lcap, D.k, mask);
  hipLaunchKernelGGL(k_band_count, dim3(nblk, B), dim3(kDefThreads), 0, s, mask, n, D.k, counts,
                     nblk);
  hipLaunchKernelGGL(k_scan_counts, dim3(B), dim3(1024), 0, s, counts, nblk, op->defl_total);
  hipLaunchKernelGGL(k_band_write, dim3(nblk, B), dim3(kDefThreads), 0, s, F, D.lab, mask, n, D.k,
                     counts, nblk, D, op->defl_over);
  hipLaunchKernelGGL(k_band_done, gb, dim3(256), 0, s, D.bcount, op->defl_total, D.cap, B);
  ck_launch();
  hipLaunchKernelGGL(k_defl_e, dim3(kDefMax, B), dim3(kDefThreads), 0, s, D, op->defl_e);
  hipLaunchKernelGGL(k_defl_inverse, dim3(B), dim3(kDefMax * kDefMax), 0, s, op->defl_e, D,
                     op->defl_over);
  hipLaunchKernelGGL(k_defl_off, gb, dim3(256), 0, s, D, op->defl_over, B);
  ck_launch();
  to_host(D.k);
  for (int b = 0; b < B; ++b) {
    op->h_defl_k[b] = h[b];
    op->defl_any = op->defl_any || h[b] > 0;
  }
}

// Start of a deflated CG: zb = Z^T rhs, coef = E^{-1} (zb - (A Z)^T x) and r -= A Z coef on
// the band, the change of ||r||^2 appended to the residual's partials (at `off`)
template <typename T>
void defl_start(mpp_op_s* op, Ctl& ctl, const T* rhs, const T* x, T* r, int xzero, int off,
                hipStream_t s) {
  const Defl& D = op->defl;
  const int B = op->batch, cells = (int)op->lev[0].cells;
  hipLaunchKernelGGL(k_region_sums<T>, dim3(op->defl_rblk, B), dim3(kDefThreads), 0, s, rhs, D.lab,
                     cells, D, (const int*)nullptr);
  hipLaunchKernelGGL(k_defl_zb, dim3(B), dim3(64), 0, s, D, op->defl_rblk, (const int*)nullptr);
  if (!xzero)
    hipLaunchKernelGGL(k_band_sums<T>, dim3(kDefBandBlocks, B), dim3(kDefThreads), 0, s, x, cells,
                       D, Sel{});
  hipLaunchKernelGGL(k_defl_coef, dim3(B), dim3(64), 0, s, D, xzero ? 0 : 1, (const int*)nullptr);
  hipLaunchKernelGGL(k_band_fix<T>, dim3(kDefBandBlocks, B), dim3(kDefThreads), 0, s, r, cells, D,
                     ctl, -1, off, Sel{});
  ck_launch();
}

// z <- P^T z = z - Z E^{-1} (A Z)^T z for the active problems
template <typename T>
void defl_project(mpp_op_s* op, const Ctl& ctl, T* z, hipStream_t s) {
  const Defl& D = op->defl;
  const int rows = rows_of(op, ctl.list), cells = (int)op->lev[0].cells;
  timed(op, K_DEFL, 0.0, s, [&] {
    hipLaunchKernelGGL(k_band_sums<T>, dim3(kDefBandBlocks, rows), dim3(kDefThreads), 0, s, z,
                       cells, D, sel_of(ctl));
    hipLaunchKernelGGL(k_region_add<T>, dim3(op->defl_rblk, rows), dim3(kDefThreads), 0, s, z,
                       D.lab, cells, D, 1, sel_of(ctl));
  });
  ck_launch();
}

// End of a deflated CG: x += Z E^{-1} Z^T (rhs - A x) (zb of the start, the band sums of x)
template <typename T>
void defl_end(mpp_op_s* op, T* x, hipStream_t s) {
  const Defl& D = op->defl;
  const int B = op->batch, cells = (int)op->lev[0].cells;
  hipLaunchKernelGGL(k_band_sums<T>, dim3(kDefBandBlocks, B), dim3(kDefThreads), 0, s, x, cells, D,
                     Sel{});
  hipLaunchKernelGGL(k_defl_coef, dim3(B), dim3(64), 0, s, D, 1, (const int*)nullptr);
  hipLaunchKernelGGL(k_region_add<T>, dim3(op->defl_rblk, B), dim3(kDefThreads), 0, s, x, D.lab,
                     cells, D, 0, Sel{});
  ck_launch();
}

// ------------------------------------------------------------------------------
// Preconditioned CG on -A for every problem whose ctl.active flag is set by the
// start epilogue.  Uses ctl.scal[S_TOL2] as the per-problem target on ||r||^2.
// ------------------------------------------------------------------------------
// z = V(r) and the r.z epilogue (the dot is folded into the last sweep when the
// finest level uses the fused sweeps)
template <typename T>
void vcycle_dot(mpp_op_s* op, Ctl& ctl, const T* r, T* z, int nu, const EpiArgs& erz,
                hipStream_t s) {
  const Level& L0 = op->lev[0];
  int parts = 0;
  vcycle<T>(op, 0, r, z, nu, sel_of(ctl), s, &ctl, &parts);
  if (parts == 0) {
    timed(op, K_DOT, alg_bytes(op, K_DOT, sizeof(T)), s, [&] {
      hipLaunchKernelGGL(k_dot<T>, grid_of(L0, rows_of(op, ctl.list)), dim3(kBlock), 0, s, r, z,
                         (int)L0.cells, ctl, erz, sel_of(ctl));
    });
    ck_launch();
    parts = L0.bpp;
  }
  finish_sums(op, ctl, erz, parts, s);
}

// `iters` CG iterations, each from z = V(r) to the convergence test on the updated
// residual, so that a block of iterations ends with the test the host polls (a block
// launched after the last useful test would run only kernels with nothing to do).
// first: the block starts the CG (p = z, no beta).
template <typename T>
void pcg_iterations(mpp_op_s* op, Ctl& ctl, T* x, T* r, T* z, T* p, T* q, int nu, int iters,
                    bool first, hipStream_t s) {
  Level& L0 = op->lev[0];
  const int rows = rows_of(op, ctl.list);
  const dim3 g = grid_of(L0, rows);
  const Faces<T> F = faces_of<T>(op, 0);
  const int cells = (int)L0.cells;
  const EpiArgs epq = epi(E_PQ), err = epi(E_RR_ITER);
  const bool defl = op->defl_use;
  // the row map of this block of iterations from the flags as they stand
  if (ctl.list) {
    hipLaunchKernelGGL(k_live_list, dim3(1), dim3(1024), 0, s, (const int*)ctl.active, op->batch,
                       op->live);
    ck_launch();
  }
  for (int it = 0; it < iters; ++it) {
    const int f1 = (first && it == 0) ? 1 : 0;
    EpiArgs erz = epi(E_RZ);
    erz.first = f1;
    vcycle_dot<T>(op, ctl, r, z, nu, erz, s);
    if (defl) defl_project<T>(op, ctl, z, s);
    timed(op, K_UPDATE_P, alg_bytes(op, K_UPDATE_P, sizeof(T)), s, [&] {
      hipLaunchKernelGGL(k_update_p<T>, g, dim3(kBlock), 0, s, z, p, cells, ctl, f1);
    });
    ck_launch();
    int parts = 0;
    timed(op, K_APPLY_DOT, alg_bytes(op, K_APPLY_DOT, sizeof(T)), s,
          [&] { parts = launch_apply<T>(op, F, p, q, ctl, 1, sel_of(ctl), s); });
    ck_launch();
    if (defl) {   // p.(P q) = p.q - a.s, s = (A Z)^T p over the band, a = E^{-1} s
      timed(op, K_DEFL, 0.0, s, [&] {
        hipLaunchKernelGGL(k_band_sums<T>, dim3(kDefBandBlocks, rows), dim3(kDefThreads), 0, s, p,
                           cells, op->defl, sel_of(ctl));
        hipLaunchKernelGGL(k_finish_pq_defl, dim3(rows), dim3(1024), 0, s, ctl, parts, epq,
                           op->defl);
      });
      ck_launch();
    } else {
      finish_sums(op, ctl, epq, parts, s);
    }
    timed(op, K_UPDATE_XR, alg_bytes(op, K_UPDATE_XR, sizeof(T)), s, [&] {
      hipLaunchKernelGGL(k_update_xr<T>, g, dim3(kBlock), 0, s, x, r, p, q, cells, ctl, err);
    });
    ck_launch();
    if (defl) {   // r += alpha (A Z) a on the band (r -= alpha P q), ||r||^2 corrected
      timed(op, K_DEFL, 0.0, s, [&] {
        hipLaunchKernelGGL(k_band_fix<T>, dim3(kDefBandBlocks, rows), dim3(kDefThreads), 0, s, r,
                           cells, op->defl, ctl, (int)S_ALPHA, L0.bpp, sel_of(ctl));
      });
      ck_launch();
      finish_sums(op, ctl, err, L0.bpp + kDefBandBlocks, s);
    } else {
      finish_sums(op, ctl, err, L0.bpp, s);
    }
  }
}

// known_active: the caller knows some problem is active at the start (no start poll).
// given_parts > 0: the caller has r = rhs (x = 0) and that many ||r||^2 block partials in
// place (no residual launch).
template <typename T>
void pcg(mpp_op_s* op, Ctl& ctl, const T* rhs, T* x, T* r, T* z, T* p, T* q, int nu,
         int check_every, int xzero, const EpiArgs& start, hipStream_t s,
         bool known_active = false, int given_parts = 0) {
  const Faces<T> F = faces_of<T>(op, 0);
  int parts = given_parts;
  if (parts == 0) {
    timed(op, K_RESIDUAL, alg_bytes(op, K_RESIDUAL, sizeof(T)), s,
          [&] { parts = launch_residual<T>(op, F, rhs, x, r, ctl, xzero, s); });
    ck_launch();
  }
  const bool defl = op->defl_use;
  EpiArgs start_ = start;
  if (defl) {   // CG on the deflated system: r <- P r
    // a relative target stays relative to ||r|| before deflation: the jump term, which
    // dominates b, is almost entirely A times a constant per region, so P r can be tiny
    EpiArgs eb = epi(E_STORE_MEAN);
    eb.slot = S_SUM;
    eb.inv_cells = 1.0;
    finish_sums(op, ctl, eb, parts, s);
    start_.rel_base = 1;
    defl_start<T>(op, ctl, rhs, x, r, xzero, parts, s);
    parts += kDefBandBlocks;
  }
  finish_sums(op, ctl, start_, parts, s);
  // the row map and the schedule of the iterations end with them, however pcg is left
  struct Unlist {
    mpp_op_s* op;
    Ctl& c;
    ~Unlist() {
      c.list = nullptr;
      op->rows = op->batch;
      op->tail = false;
    }
  } unlist{op, ctl};
  // the iterate of a deflated CG takes its component in the regions at the end
  auto done_ = [&] {
    ctl.list = nullptr;
    op->tail = false;
    if (defl) defl_end<T>(op, x, s);
  };
  if (!known_active && !any_active(op, ctl, s)) {
    done_();
    return;
  }
  // Once the live count of the last poll rounded up to a power of two is below the batch,
  // the iterations serve the problems listed in op->live (rebuilt from the active flags
  // at the start of every block of iterations) on that many block rows: the list never
  // holds more, since problems only leave.  Before that every problem keeps its row (a
  // list would launch as many rows and add a load to every block's start).  Few live
  // problems of a batch also take the tail schedule (more, smaller tiles per problem).
  // MPP_COMPACT=0 keeps every problem's row throughout, MPP_TAIL=0 the full-batch tiles.
  const int B = op->batch;
  const char* tail_env = std::getenv("MPP_TAIL");
  const bool tail_ok = B > 1 && !(tail_env && tail_env[0] == '0');
  const char* compact_env = std::getenv("MPP_COMPACT");
  const bool compact = !(compact_env && compact_env[0] == '0');
  auto set_sched = [&] {
    int live = 0;
    for (int b = 0; b < B; ++b) live += op->h_active[b] != 0;
    int rows = 1;
    while (rows < live) rows *= 2;
    op->rows = compact ? std::min(rows, B) : B;
    op->tail = tail_ok && live <= std::max(1, B / 8);
    ctl.list = op->rows < B ? op->live : nullptr;
  };
  set_sched();
  // iterations in blocks of check_every; the kernels themselves stop working on a
  // problem once it has converged, so a block may overrun the last useful iteration
  // (measured: spacing the polls by a prediction of the remaining iterations gains
  // nothing on one problem and loses on a batch)
  const bool graphs = op->use_graphs && !op->prof.on;
  for (int done = 0; done <= ctl.max_iter; done += check_every) {
    const bool first = done == 0;
    const GraphKey key{(int)sizeof(T), nu, op->nu_c, check_every, ctl.max_iter, defl ? 1 : 0,
                       op->tail ? 1 : 0, op->rows, first ? 1 : 0,
                       {(const void*)ctl.scal, x, r, z, p, q}, op->shift};
    if (graphs)
      run_graph(op, key, s, [&](hipStream_t cs) {
        pcg_iterations<T>(op, ctl, x, r, z, p, q, nu, check_every, first, cs);
      });
    else
      pcg_iterations<T>(op, ctl, x, r, z, p, q, nu, check_every, first, s);
    if (!any_active(op, ctl, s)) break;
    set_sched();
  }
  done_();
}

void reset_ctl(mpp_op_s* op, Ctl& ctl, int max_iter, hipStream_t s) {
  const int B = op->batch;
  ctl.list = nullptr;
  hipLaunchKernelGGL(k_ctl_reset, dim3((B * kSlots + 255) / 256), dim3(256), 0, s, ctl, B);
  ck_launch();
  ctl.max_iter = max_iter;
}

// b = f + jterm - mean, into `out`; S_MEAN of ctl
void make_rhs(mpp_op_s* op, Ctl& ctl, const double* f, double* out, hipStream_t s,
              double rtol, bool want_bb, float* out32 = nullptr) {
  const Level& L0 = op->lev[0];
  const dim3 g = grid_of(L0, op->batch);
  const int cells = (int)L0.cells;
  EpiArgs em = epi(E_MEAN);
  em.inv_cells = 1.0 / (double)L0.cells;
  hipLaunchKernelGGL(k_rhs_sum, g, dim3(kBlock), 0, s, f, op->jterm, out, cells, ctl, em);
  ck_launch();
  finish_sums(op, ctl, em, L0.bpp, s);
  EpiArgs eb = epi(E_BB);
  eb.rtol2 = rtol * rtol;
  hipLaunchKernelGGL(k_sub_mean_sq, g, dim3(kBlock), 0, s, out, cells, ctl, eb, (int)S_MEAN,
                     want_bb ? 1 : 0, out32);
  ck_launch();
  if (want_bb) finish_sums(op, ctl, eb, L0.bpp, s);
}

// x -= mean(x)
void remove_mean(mpp_op_s* op, Ctl& ctl, double* x, hipStream_t s) {
  const Level& L0 = op->lev[0];
  const dim3 g = grid_of(L0, op->batch);
  const int cells = (int)L0.cells;
  EpiArgs e = epi(E_STORE_MEAN);
  e.slot = S_SUM;
  e.inv_cells = 1.0 / (double)L0.cells;
  hipLaunchKernelGGL(k_sum<double>, g, dim3(kBlock), 0, s, x, cells, ctl, e);
  ck_launch();
  finish_sums(op, ctl, e, L0.bpp, s);
  hipLaunchKernelGGL(k_sub_mean_sq, g, dim3(kBlock), 0, s, x, cells, ctl, e, (int)S_SUM, 0,
                     (float*)nullptr);
  ck_launch();
}

// EINVAL before EBREAKDOWN before ENOTCONVERGED before OK
int worse(int a, int b) {
  auto rank = [](int st) {
    switch (st) {
      case MPP_OK: return 0;
      case MPP_ENOTCONVERGED: return 1;
      case MPP_EBREAKDOWN: return 2;
      default: return 3;
    }
  };
  return rank(b) > rank(a) ? b : a;
}

int status_of(hipError_t e) {
  (void)e;
  return MPP_EDEVICE;
}

// ------------------------------------------------------------------------------
// implicit heat diffusion: CG on (dt A - I) with the inverse diagonal as the
// preconditioner, on the operator's finest-level faces
// ------------------------------------------------------------------------------
dim3 heat_grid(const mpp_op_s* op, StTiles& tl) {
  tl = st_tiles(op->lev[0].n, kStKZ);
  return dim3(st_grid(tl), op->batch);
}

int heat_apply(mpp_op_s* op, const double* p, double* q, const Ctl& ctl, hipStream_t s) {
  StTiles tl;
  const dim3 grid = heat_grid(op, tl);
  timed(op, K_HEAT_APPLY, alg_bytes(op, K_HEAT_APPLY, 8), s, [&] {
    hipLaunchKernelGGL(k_heat_z<0>, grid, dim3(kStThreads), 0, s, faces_of<double>(op, 0),
                       op->lev[0].n, tl, kStKZ, p, (const double*)nullptr, q, ctl, ctl.active);
  });
  ck_launch();
  return (int)grid.x;
}

int heat_residual(mpp_op_s* op, const double* b, const double* x, double* r, const Ctl& ctl,
                  hipStream_t s) {
  StTiles tl;
  const dim3 grid = heat_grid(op, tl);
  timed(op, K_HEAT_RESIDUAL, alg_bytes(op, K_HEAT_RESIDUAL, 8), s, [&] {
    hipLaunchKernelGGL(k_heat_z<1>, grid, dim3(kStThreads), 0, s, faces_of<double>(op, 0),
                       op->lev[0].n, tl, kStKZ, x, b, r, ctl, (const int*)nullptr);
  });
  ck_launch();
  return (int)grid.x;
}

int heat_jacobi(mpp_op_s* op, const double* r, double* z, const Ctl& ctl, hipStream_t s) {
  StTiles tl;
  const dim3 grid = heat_grid(op, tl);
  timed(op, K_HEAT_JACOBI, alg_bytes(op, K_HEAT_JACOBI, 8), s, [&] {
    hipLaunchKernelGGL(k_heat_jacobi, grid, dim3(kStThreads), 0, s, faces_of<double>(op, 0),
                       op->lev[0].n, tl, kStKZ, r, z, ctl, ctl.active);
  });
  ck_launch();
  return (int)grid.x;
}

void heat_iterations(mpp_op_s* op, Ctl& ctl, double* x, int iters, hipStream_t s) {
  const Level& L0 = op->lev[0];
  const dim3 g = grid_of(L0, op->batch);
  const int cells = (int)L0.cells;
  const EpiArgs erz = epi(E_RZ), epq = epi(E_PQ), err = epi(E_RR_ITER);
  for (int it = 0; it < iters; ++it) {
    finish_sums(op, ctl, epq, heat_apply(op, op->p, op->q, ctl, s), s);
    timed(op, K_UPDATE_XR, alg_bytes(op, K_UPDATE_XR, 8), s, [&] {
      hipLaunchKernelGGL(k_update_xr<double>, g, dim3(kBlock), 0, s, x, op->r, op->p, op->q,
                         cells, ctl, err);
    });
    ck_launch();
    finish_sums(op, ctl, err, L0.bpp, s);
    finish_sums(op, ctl, erz, heat_jacobi(op, op->r, op->z, ctl, s), s);
    timed(op, K_UPDATE_P, alg_bytes(op, K_UPDATE_P, 8), s, [&] {
      hipLaunchKernelGGL(k_update_p<double>, g, dim3(kBlock), 0, s, op->z, op->p, cells, ctl, 0);
    });
    ck_launch();
  }
}

// CG from the true residual of x until every problem has converged, broken down or
// used ctl.max_iter iterations
void heat_pcg(mpp_op_s* op, Ctl& ctl, double* x, int check_every, hipStream_t s) {
  const Level& L0 = op->lev[0];
  const dim3 g = grid_of(L0, op->batch);
  const int cells = (int)L0.cells;
  finish_sums(op, ctl, epi(E_START), heat_residual(op, op->b, x, op->r, ctl, s), s);
  if (!any_active(op, ctl, s)) return;
  EpiArgs erz = epi(E_RZ);
  erz.first = 1;
  finish_sums(op, ctl, erz, heat_jacobi(op, op->r, op->z, ctl, s), s);
  hipLaunchKernelGGL(k_update_p<double>, g, dim3(kBlock), 0, s, op->z, op->p, cells, ctl, 1);
  ck_launch();
  // nu = 0 marks these graphs apart from the pressure solve's (nu >= 1)
  const bool graphs = op->use_graphs && !op->prof.on;
  const GraphKey key{8, 0, 0, check_every, ctl.max_iter, 0, 0, op->batch, 0,
                     {(const void*)ctl.scal, x, op->r, op->z, op->p, op->q}};
  for (int done = 0; done < ctl.max_iter; done += check_every) {
    if (graphs)
      run_graph(op, key, s, [&](hipStream_t cs) { heat_iterations(op, ctl, x, check_every, cs); });
    else
      heat_iterations(op, ctl, x, check_every, s);
    if (!any_active(op, ctl, s)) return;
  }
}

}  // namespace

// ==============================================================================
// C ABI
// ==============================================================================
extern "C" {

void mpp_default_opts(mpp_solve_opts* o) {
  if (!o) return;
  o->rtol = 1e-10;
  o->max_iter = 500;
  o->mode = MPP_MODE_FP64;
  o->guess = MPP_GUESS_ZERO;
  o->nu = 2;
  o->nu_coarse = 0;
  o->check_every = 2;
  o->inner_rtol = 1e-5;
  o->deflate = 1;
  o->reuse_rhs = 0;
}

size_t mpp_workspace_bytes(const mpp_desc* desc) {
  if (!desc_ok(desc)) return 0;
  mpp_op_s tmp;
  return layout(&tmp, desc, nullptr);
}

const char* mpp_strerror(int st) {
  switch (st) {
    case MPP_OK: return "ok";
    case MPP_EINVAL: return "invalid argument";
    case MPP_ENOMEM: return "workspace too small";
    case MPP_EDEVICE: return "HIP runtime error";
    case MPP_ENOTCONVERGED: return "not converged within max_iter";
    case MPP_EBREAKDOWN: return "conjugate-gradient breakdown";
    default: return "unknown status";
  }
}

}  // extern "C"

namespace {

// Dense inverse of the coarsest level for the current shift.
void factor_coarsest(mpp_op_s* op, hipStream_t s) {
  const Level& Lc = op->lev[op->nlev - 1];
  const double sc = level_shift(op, op->nlev - 1);
  hipLaunchKernelGGL(k_coarse_factor, dim3(op->batch), dim3(1024), 0, s, Lc.f64[0], Lc.f64[1],
                     Lc.f64[2], Lc.n, sc, op->coarse_work, op->coarse_inv);
  ck_launch();
  op->coarse_shift = sc;
}

// Makes A - shift I (on the finest level; halved per coarser level) the operator every
// kernel applies; the coarsest inverse is rebuilt when its shift changes.
void use_shift(mpp_op_s* op, double shift, hipStream_t s) {
  op->shift = shift;
  if (level_shift(op, op->nlev - 1) != op->coarse_shift) factor_coarsest(op, s);
}

bool opts_valid(const mpp_solve_opts& o) {
  if (!(o.rtol > 0.0) || o.max_iter < 1 || o.nu < 1 || o.check_every < 1 || o.nu_coarse < 0 ||
      (o.mode != MPP_MODE_FP64 && o.mode != MPP_MODE_MIXED) ||
      (o.guess != MPP_GUESS_ZERO && o.guess != MPP_GUESS_GIVEN))
    return false;
  if (o.mode == MPP_MODE_MIXED && !(o.inner_rtol > 0.0 && o.inner_rtol < 1.0)) return false;
  if (o.deflate != 0 && o.deflate != 1) return false;
  if (o.reuse_rhs != 0 && o.reuse_rhs != 1) return false;
  return true;
}

// MG-PCG on op->b (S_BB and S_TOL2 of op->outer set) from the caller's p or from zero,
// in FP64 or as FP64 refinement around FP32 MG-PCG; the iterate ends in op->x.
void solve_core(mpp_op_s* op, const mpp_solve_opts& o, const double* user_p,
                std::vector<int>& outer_count, std::vector<int>& istatus, hipStream_t s) {
  const int B = op->batch;
  const Level& L0 = op->lev[0];
  const dim3 g = grid_of(L0, B);
  const int cells = (int)L0.cells;
  ensure_tuned<double>(op, s);
  if (o.mode == MPP_MODE_MIXED) ensure_tuned<float>(op, s);
  op->nu_c = o.nu_coarse > 0 ? o.nu_coarse : o.nu;
  // deflation of the light-phase regions: pressure solves only (a shifted operator has no
  // such slow modes)
  op->defl_use = false;
  if (o.deflate && op->shift == 0.0) {
    if (!op->defl_ready) build_deflation(op, s);
    op->defl_use = op->defl_any;
  }
  Ctl& oc = op->outer;
  // the iterate lives in the workspace (captured launch graphs refer to it); the
  // caller's p is copied in and out
  double* const p = op->x;
  // from zero the first residual is b itself (no reads of the iterate)
  const bool zero_start = o.guess == MPP_GUESS_ZERO;
  if (zero_start) {
    hipLaunchKernelGGL(k_fill<double>, g, dim3(kBlock), 0, s, p, cells, 0.0);
    ck_launch();
  } else {
    ck(hipMemcpyAsync(p, user_p, sizeof(double) * op->cells * B, hipMemcpyDeviceToDevice, s));
  }
  EpiArgs start = epi(E_START);
  if (o.mode == MPP_MODE_FP64) {
    for (int restart = 0; restart < 4; ++restart) {
      pcg<double>(op, oc, op->b, p, op->r, op->z, op->p, op->q, o.nu, o.check_every,
                  (restart == 0 && zero_start) ? 1 : 0, start, s);
      // true residual; re-arms the problems that are not there yet
      finish_sums(op, oc, start,
                  launch_residual<double>(op, faces_of<double>(op, 0), op->b, p, op->r, oc, 0, s), s);
      ck_launch();
      for (int b = 0; b < B; ++b) outer_count[b] += 1;
      if (!any_active(op, oc, s)) break;
    }
    return;
  }
  Ctl& ic = op->inner;
  reset_ctl(op, ic, o.max_iter, s);
  EpiArgs istart = epi(E_START_REL);
  istart.rtol2 = o.inner_rtol * o.inner_rtol;
  istart.gate = oc.active;
  istart.outer_scal = oc.scal;
  istart.outer_rtol = o.rtol;
  bool settled = false;
  for (int outer = 0; outer < 40; ++outer) {
    const int xzero = (outer == 0 && zero_start) ? 1 : 0;
    int parts = launch_residual<double>(op, faces_of<double>(op, 0), op->b, p, op->r, oc, xzero, s);
    ck_launch();
    if (op->defl_use) {
      // the regions' share of the correction in FP64: x += Z E^{-1} Z^T (b - A x) and
      // r -= A Z E^{-1} Z^T r, so that the FP32 inner solve never carries the large
      // per-region constants of the solution (in FP32 they would limit the true
      // residual reduction of a refinement step to about 1e-4)
      timed(op, K_DEFL, 0.0, s, [&] {
        defl_start<double>(op, oc, op->b, p, op->r, xzero, parts, s);
        hipLaunchKernelGGL(k_region_add<double>, dim3(op->defl_rblk, B), dim3(kDefThreads), 0, s,
                           p, op->defl.lab, cells, op->defl, 0, Sel{});
      });
      ck_launch();
      parts += kDefBandBlocks;
    }
    finish_sums(op, oc, start, parts, s);
    if (!any_active(op, oc, s)) {
      settled = true;
      break;
    }
    for (int b = 0; b < B; ++b) outer_count[b] += op->h_active[b];
    hipLaunchKernelGGL(k_scale_down, g, dim3(kBlock), 0, s, op->r, op->r32, op->d32, cells,
                       oc.scal, oc.active, ic);
    ck_launch();
    // every problem still active in the refinement has work in its inner solve, which
    // starts from d32 = 0 with the partials of ||r32||^2 in place
    pcg<float>(op, ic, op->r32, op->d32, op->r32, op->z32, op->p32, op->q32, o.nu,
               o.check_every, 1, istart, s, true, (int)L0.bpp);
    hipLaunchKernelGGL(k_correct, g, dim3(kBlock), 0, s, p, op->d32, cells, oc.scal, oc.active);
    ck_launch();
    // an inner breakdown or an exhausted iteration budget ends the refinement of that
    // problem only
    hipLaunchKernelGGL(k_stop_failed, dim3((B + 255) / 256), dim3(256), 0, s, B, ic.status,
                       oc.status, oc.active);
    ck_launch();
  }
  if (!settled) {   // 40 refinement steps: true residual of the returned iterate
    finish_sums(op, oc, start,
                launch_residual<double>(op, faces_of<double>(op, 0), op->b, p, op->r, oc, 0, s), s);
    ck_launch();
  }
  ck(hipMemcpyAsync(istatus.data(), ic.status, sizeof(int) * B, hipMemcpyDeviceToHost, s));
}

// op->x to the caller and the scalars, statuses and iteration counts to the host
// (inner: the iteration counts are those of the FP32 inner solves)
void finish_solve(mpp_op_s* op, bool inner, double* user_p, hipStream_t s) {
  const int B = op->batch;
  Ctl& oc = op->outer;
  ck(hipMemcpyAsync(user_p, op->x, sizeof(double) * op->cells * B, hipMemcpyDeviceToDevice, s));
  ck(hipMemcpyAsync(op->h_scal, oc.scal, sizeof(double) * B * kSlots, hipMemcpyDeviceToHost, s));
  ck(hipMemcpyAsync(op->h_status, oc.status, sizeof(int) * B, hipMemcpyDeviceToHost, s));
  ck(hipMemcpyAsync(op->h_iters, inner ? op->inner.iters : oc.iters, sizeof(int) * B,
                    hipMemcpyDeviceToHost, s));
  ck(hipMemcpyAsync(op->h_active, oc.active, sizeof(int) * B, hipMemcpyDeviceToHost, s));
  ck(hipStreamSynchronize(s));
}

int fill_info(mpp_op_s* op, const mpp_solve_opts& o, const std::vector<int>& outer_count,
              const std::vector<int>& istatus, mpp_solve_info* info) {
  int worst = MPP_OK;
  for (int b = 0; b < op->batch; ++b) {
    const double* sc = op->h_scal + (size_t)b * kSlots;
    mpp_solve_info& in = info[b];
    in.status = op->h_status[b];
    in.iters = op->h_iters[b];
    in.outer_iters = outer_count[b];
    in.reserved = 0;
    in.bnorm = std::sqrt(sc[S_BB]);
    in.removed_mean = sc[S_MEAN];
    in.rel_resid = sc[S_BB] > 0.0 ? std::sqrt(sc[S_RR] / sc[S_BB]) : 0.0;
    if (istatus[b] == MPP_EBREAKDOWN) in.status = MPP_EBREAKDOWN;
    if (!std::isfinite(sc[S_BB])) in.status = MPP_EINVAL;   // non-finite input
    else if (in.status == MPP_OK && !(in.rel_resid <= o.rtol)) in.status = MPP_ENOTCONVERGED;
    worst = worse(worst, in.status);
  }
  return worst;
}

// Validates the per-problem constants into a host array [B][3].
bool read_params(int B, const double* rho_neg, const double* rho_pos, const double* sigma,
                 std::vector<double>& host) {
  if (!rho_neg || !rho_pos || !sigma) return false;
  host.assign(3 * (size_t)B, 0.0);
  for (int b = 0; b < B; ++b) {
    const double rn = rho_neg[b], rp = rho_pos[b], sg = sigma[b];
    if (!(rn > 0.0) || !(rp > 0.0) || !std::isfinite(rn) || !std::isfinite(rp) ||
        !(sg >= 0.0) || !std::isfinite(sg))
      return false;
    host[3 * b + 0] = rn;
    host[3 * b + 1] = rp;
    host[3 * b + 2] = sg;
  }
  return true;
}

// Faces, curvature, jump term and the multigrid hierarchy for level set phi, in the
// operator's workspace.  Returns MPP_EINVAL for a non-finite phi.
int build_into(mpp_op_s* op, const double* phi, const std::vector<double>& host, hipStream_t s) {
  const int B = op->batch;
  op->defl_ready = false;   // built again at the next deflated solve
  op->h_defl_light.assign(B, -1);
  for (int b = 0; b < B; ++b) {   // the lighter phase's side bit (phi > 0: 1)
    const double rn = host[3 * b], rp = host[3 * b + 1];
    op->h_defl_light[b] = rn < rp ? 0 : (rp < rn ? 1 : -1);
  }
  ck(hipMemcpyAsync(op->rho, host.data(), sizeof(double) * 3 * B, hipMemcpyHostToDevice, s));
  // the outer status array doubles as the non-finite flag during the build
  ck(hipMemsetAsync(op->outer.status, 0, sizeof(int) * B, s));
  hipLaunchKernelGGL(k_params, dim3((B + 255) / 256), dim3(256), 0, s, op->rho, op->inv_rho64,
                     op->inv_rho32, B);
  ck_launch();
  Level& L0 = op->lev[0];
  const int n = op->n, cells = (int)L0.cells;
  const dim3 g = grid_of(L0, B);
  {
    const int ntx = (n + 63) / 64, nty = (n + 3) / 4, kz = 16, nkz = (n + kz - 1) / kz;
    const int ntiles = ntx * nty * nkz;
    hipLaunchKernelGGL(k_faces, dim3(8 * ((ntiles + 7) / 8), B), dim3(256), 0, s, phi, op->rho, n,
                       ntx, nty, kz, ntiles, L0.code, L0.f64[0], L0.f64[1], L0.f64[2], L0.f32[0],
                       L0.f32[1], L0.f32[2], op->outer.status);
  }
  ck_launch();
  hipLaunchKernelGGL(k_curvature, g, dim3(kBlock), 0, s, phi, L0.code, n, cells, op->kappa);
  ck_launch();
  hipLaunchKernelGGL(k_jump, g, dim3(kBlock), 0, s, phi, L0.code, op->kappa, op->rho, n, cells,
                     op->jterm);
  ck_launch();
  for (int l = 1; l < op->nlev; ++l) {
    Level& Lf = op->lev[l - 1];
    Level& Lc = op->lev[l];
    hipLaunchKernelGGL(k_coarsen_faces, grid_of(Lc, B), dim3(kBlock), 0, s, Lf.f64[0], Lf.f64[1],
                       Lf.f64[2], Lf.n, Lc.f64[0], Lc.f64[1], Lc.f64[2], Lc.f32[0], Lc.f32[1],
                       Lc.f32[2]);
    ck_launch();
  }
  factor_coarsest(op, s);
  ck(hipMemcpyAsync(op->h_status, op->outer.status, sizeof(int) * B, hipMemcpyDeviceToHost, s));
  ck(hipStreamSynchronize(s));
  for (int b = 0; b < B; ++b)
    if (op->h_status[b]) return MPP_EINVAL;
  return MPP_OK;
}

void free_op(mpp_op_s* op) {
  for (GraphEntry& g : op->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  if (op->cap_stream) (void)hipStreamDestroy(op->cap_stream);
  for (hipEvent_t e : op->prof.pool) (void)hipEventDestroy(e);
  for (void* h : {(void*)op->h_active, (void*)op->h_iters, (void*)op->h_status,
                  (void*)op->h_scal})
    if (h) (void)hipHostFree(h);
  delete op;
}

}  // namespace

extern "C" {

int mpp_build_operator(const mpp_desc* desc, const double* phi, const double* rho_neg,
                       const double* rho_pos, const double* sigma, void* workspace,
                       size_t workspace_bytes, void* stream, mpp_op* out) {
  if (out) *out = nullptr;
  if (!desc_ok(desc) || !phi || !workspace || !out) return MPP_EINVAL;
  const int B = desc->batch;
  std::vector<double> host;
  if (!read_params(B, rho_neg, rho_pos, sigma, host)) return MPP_EINVAL;
  mpp_op_s tmp;
  const size_t need = layout(&tmp, desc, nullptr);
  if (workspace_bytes < need) return MPP_ENOMEM;
  mpp_op_s* op = new (std::nothrow) mpp_op_s();
  if (!op) return MPP_ENOMEM;
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(workspace) + 255) & ~uintptr_t(255));
  layout(op, desc, base);
  op->flags = desc->flags;
  op->use_graphs = (desc->flags & MPP_FLAG_NO_GRAPHS) == 0;
  op->ws = workspace;
  op->ws_bytes = workspace_bytes;
  // pinned host arrays for the polls and the results (small copies without staging)
  if (hipHostMalloc((void**)&op->h_active, sizeof(int) * B, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&op->h_iters, sizeof(int) * B, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&op->h_status, sizeof(int) * B, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&op->h_scal, sizeof(double) * B * kSlots, hipHostMallocDefault) !=
          hipSuccess) {
    free_op(op);
    return MPP_ENOMEM;
  }
  int st;
  try {
    st = build_into(op, phi, host, reinterpret_cast<hipStream_t>(stream));
  } catch (HipError& e) {
    st = status_of(e.e);
  }
  if (st != MPP_OK) {
    free_op(op);
    return st;
  }
  *out = op;
  return MPP_OK;
}

int mpp_update_operator(mpp_op op, const double* phi, const double* rho_neg,
                        const double* rho_pos, const double* sigma, void* stream) {
  if (!op || !phi) return MPP_EINVAL;
  std::vector<double> host;
  if (!read_params(op->batch, rho_neg, rho_pos, sigma, host)) return MPP_EINVAL;
  op->guess_f = nullptr;   // the learned guess's right-hand side is no longer current
  try {
    return build_into(op, phi, host, reinterpret_cast<hipStream_t>(stream));
  } catch (HipError& e) {
    return status_of(e.e);
  }
}

int mpp_profile_start(mpp_op op) {
  if (!op) return MPP_EINVAL;
  Prof& P = op->prof;
  P.on = true;
  P.recs.clear();
  P.used = 0;
  for (int k = 0; k < kKernelIds; ++k) {
    P.ms[k] = 0.0;
    P.bytes[k] = 0.0;
    P.launches[k] = 0;
  }
  return MPP_OK;
}

int mpp_profile_stop(mpp_op op, mpp_kernel_stat* stats, int32_t max_stats, int32_t* n_stats) {
  if (!op || (max_stats > 0 && !stats)) return MPP_EINVAL;
  Prof& P = op->prof;
  try {
    for (const ProfRec& r : P.recs) ck(hipEventSynchronize(r.b));
    prof_collect(P);
  } catch (HipError& e) {
    P.on = false;
    return status_of(e.e);
  }
  P.on = false;
  int cnt = 0;
  for (int k = 0; k < kKernelIds; ++k) {
    if (P.launches[k] == 0) continue;
    if (cnt < max_stats) {
      mpp_kernel_stat& st = stats[cnt];
      std::memset(&st, 0, sizeof(st));
      std::snprintf(st.name, sizeof(st.name), "%s", kKernelNames[k]);
      st.launches = (int32_t)P.launches[k];
      st.total_ms = P.ms[k];
      st.bytes = P.bytes[k];
    }
    ++cnt;
  }
  if (n_stats) *n_stats = std::min(cnt, (int)std::max(max_stats, 0));
  return MPP_OK;
}

void mpp_destroy_operator(mpp_op op) {
  if (!op) return;
  free_op(op);
}

int mpp_deflation_info(mpp_op op, uint8_t* labels, int32_t* k, double* E, void* stream) {
  if (!op || !k) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  op->guess_f = nullptr;   // the learned guess's right-hand side is no longer current
  try {
    if (!op->defl_ready) build_deflation(op, s);
    const int B = op->batch;
    for (int b = 0; b < B; ++b) k[b] = op->h_defl_k[b];
    if (labels) {
      if (op->defl_any) {
        ck(hipMemcpyAsync(labels, op->defl.lab, op->cells * B, hipMemcpyDeviceToDevice, s));
      } else {
        hipLaunchKernelGGL(k_u8_fill, dim3(1024), dim3(256), 0, s, labels, op->cells * B);
        ck_launch();
      }
    }
    if (E) {
      const size_t bytes = sizeof(double) * B * kDefMax * kDefMax;
      if (op->defl_any) {
        ck(hipMemcpyAsync(E, op->defl_e, bytes, hipMemcpyDeviceToHost, s));
      } else {
        std::memset(E, 0, bytes);
      }
    }
    ck(hipStreamSynchronize(s));
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

int mpp_levels(mpp_op op, int32_t* nlevels, int32_t* sizes) {
  if (!op || !nlevels) return MPP_EINVAL;
  *nlevels = op->nlev;
  if (sizes)
    for (int l = 0; l < op->nlev; ++l) sizes[l] = op->lev[l].n;
  return MPP_OK;
}

int mpp_apply_stencil(mpp_op op, const double* x, double* y, void* stream) {
  if (!op || !x || !y || x == y) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  op->guess_f = nullptr;   // the learned guess's right-hand side is no longer current
  try {
    use_shift(op, 0.0, s);
    timed(op, K_APPLY, alg_bytes(op, K_APPLY, sizeof(double)), s, [&] {
      launch_apply<double>(op, faces_of<double>(op, 0), x, y, op->outer, 0, Sel{}, s);
    });
    ck_launch();
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

int mpp_rhs(mpp_op op, const double* f, double* b, double* mean_out, void* stream) {
  if (!op || !f || !b) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  op->guess_f = nullptr;   // the learned guess's right-hand side is no longer current
  try {
    make_rhs(op, op->inner, f, b, s, 0.0, false);
    if (mean_out) {
      ck(hipMemcpyAsync(op->h_scal, op->inner.scal, sizeof(double) * op->batch * kSlots,
                        hipMemcpyDeviceToHost, s));
      ck(hipStreamSynchronize(s));
      for (int q = 0; q < op->batch; ++q) mean_out[q] = op->h_scal[(size_t)q * kSlots + S_MEAN];
    }
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

int mpp_vcycle(mpp_op op, const double* r, double* z, int nu, void* stream) {
  if (!op || !r || !z || r == z || nu < 1) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  op->guess_f = nullptr;   // the learned guess's right-hand side is no longer current
  try {
    use_shift(op, 0.0, s);
    ensure_tuned<double>(op, s);
    op->nu_c = nu;
    vcycle<double>(op, 0, r, z, nu, Sel{}, s);
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

int mpp_operator_fields(mpp_op op, double* bx, double* by, double* bz, double* kappa,
                        double* jterm, void* stream) {
  if (!op) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t bytes = sizeof(double) * op->cells * op->batch;
  try {
    double* dst[5] = {bx, by, bz, kappa, jterm};
    const double* src[5] = {op->lev[0].f64[0], op->lev[0].f64[1], op->lev[0].f64[2], op->kappa,
                            op->jterm};
    for (int q = 0; q < 5; ++q)
      if (dst[q]) ck(hipMemcpyAsync(dst[q], src[q], bytes, hipMemcpyDeviceToDevice, s));
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

int mpp_solve(mpp_op op, const double* f, double* p, const mpp_solve_opts* opts,
              mpp_solve_info* info, void* stream) {
  if (!op || !f || !p || !opts || !info || f == p) return MPP_EINVAL;
  if (!opts_valid(*opts)) return MPP_EINVAL;
  const mpp_solve_opts& o = *opts;
  // the right-hand side of the learned guess just made for this f: b as it stands, the
  // mean and norm from the inner control block
  const bool reuse = o.reuse_rhs == 1 && op->guess_f == f;
  op->guess_f = nullptr;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int B = op->batch;
  std::vector<int> outer_count(B, 0);
  std::vector<int> istatus(B, MPP_OK);
  try {
    use_shift(op, 0.0, s);
    Ctl& oc = op->outer;
    reset_ctl(op, oc, o.max_iter, s);
    if (reuse) {
      hipLaunchKernelGGL(k_take_rhs, dim3((B + 255) / 256), dim3(256), 0, s, oc,
                         (const double*)op->inner.scal, B, o.rtol * o.rtol);
      ck_launch();
    } else {
      make_rhs(op, oc, f, op->b, s, o.rtol, true);
    }
    solve_core(op, o, p, outer_count, istatus, s);
    remove_mean(op, oc, op->x, s);
    finish_solve(op, o.mode == MPP_MODE_MIXED, p, s);
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return fill_info(op, o, outer_count, istatus, info);
}

int mpp_heat_solve(mpp_op op, const double* t_old, const double* src, double dt, double* t,
                   const mpp_solve_opts* opts, mpp_solve_info* info, void* stream) {
  if (!op || !t_old || !t || !opts || !info || src == t) return MPP_EINVAL;
  const mpp_solve_opts& o = *opts;
  if (!(dt >= 0.0) || !std::isfinite(dt)) return MPP_EINVAL;
  const bool jacobi = o.nu == 0;
  if (jacobi) {
    if (!(o.rtol > 0.0) || o.max_iter < 1 || o.check_every < 1 ||
        (o.guess != MPP_GUESS_ZERO && o.guess != MPP_GUESS_GIVEN))
      return MPP_EINVAL;
  } else if (!opts_valid(o)) {
    return MPP_EINVAL;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int B = op->batch;
  const Level& L0 = op->lev[0];
  const dim3 g = grid_of(L0, B);
  const int cells = (int)L0.cells;
  std::vector<int> outer_count(B, 0);
  std::vector<int> istatus(B, MPP_OK);
  // multigrid solves (A - I/dt) T = -(T_old + dt f) / dt; dt = 0 (T = T_old) goes to the
  // Jacobi form, which is exact there
  const bool mg = !jacobi && dt > 0.0;
  op->guess_f = nullptr;   // the learned guess's right-hand side is no longer current
  try {
    Ctl& oc = op->outer;
    reset_ctl(op, oc, o.max_iter, s);
    hipLaunchKernelGGL(k_heat_set_dt, dim3((B + 255) / 256), dim3(256), 0, s, oc.scal, B, dt);
    ck_launch();
    // the right-hand side first: t may be t_old
    hipLaunchKernelGGL(k_heat_rhs, g, dim3(kBlock), 0, s, t_old, src, mg ? 1.0 / dt : 1.0, op->b,
                       cells, oc);
    ck_launch();
    EpiArgs eb = epi(E_BB);
    eb.rtol2 = o.rtol * o.rtol;
    finish_sums(op, oc, eb, L0.bpp, s);
    if (mg) {
      use_shift(op, 1.0 / dt, s);
      solve_core(op, o, t, outer_count, istatus, s);
    } else {
      double* const x = op->x;
      if (o.guess == MPP_GUESS_ZERO) {
        hipLaunchKernelGGL(k_fill<double>, g, dim3(kBlock), 0, s, x, cells, 0.0);
        ck_launch();
      } else {
        ck(hipMemcpyAsync(x, t, sizeof(double) * op->cells * B, hipMemcpyDeviceToDevice, s));
      }
      for (int restart = 0; restart < 4; ++restart) {
        heat_pcg(op, oc, x, o.check_every, s);
        // true residual; re-arms the problems that are not there yet
        finish_sums(op, oc, epi(E_START), heat_residual(op, op->b, x, op->r, oc, s), s);
        for (int b = 0; b < B; ++b) outer_count[b] += 1;
        if (!any_active(op, oc, s)) break;
      }
    }
    finish_solve(op, mg && o.mode == MPP_MODE_MIXED, t, s);
  } catch (HipError& e) {
    return status_of(e.e);
  }
  const int st = fill_info(op, o, outer_count, istatus, info);
  for (int b = 0; b < B; ++b) info[b].removed_mean = 0.0;
  return st;
}

}  // extern "C"

// ------------------------------------------------------------------------------
// learned initial guess
// ------------------------------------------------------------------------------
namespace {

bool net_fits(const mpp_op_s* op, const mpp_net_s* net) {
  return net->n <= op->n && op->n % net->n == 0 && op->batch <= net->bmax;
}

// solver rhs into op->b (S_MEAN, S_BB in op->inner), then the coarse means and rms
void net_inputs(mpp_op_s* op, mpp_net_s* net, const double* f, const double* p, uint16_t* x,
                float* t, hipStream_t s) {
  const int B = op->batch, nc = net->n, r = op->n / net->n;
  const int cells_c = nc * nc * nc;
  reset_ctl(op, op->inner, 1, s);
  // (with an FP32 copy of b in r32 for the guess's sweeps)
  make_rhs(op, op->inner, f, op->b, s, 0.0, true, op->r32);
  const dim3 cgrid((unsigned)((cells_c + 255) / 256), B);
  const unsigned nb = (unsigned)(((size_t)cells_c * B + 255) / 256);
  // the per-workgroup partial sums of the rms go to the prediction buffer, which the
  // network only writes later (cgrid.x doubles per problem, far below its n^3 floats)
  double* part = reinterpret_cast<double*>(net->y);
  if (r == 4)
    hipLaunchKernelGGL(k_feat_coarsen<4>, cgrid, dim3(256), 0, s, op->lev[0].code, op->inv_rho64,
                       op->b, p, op->n, r, nc, net->coarse, part);
  else
    hipLaunchKernelGGL(k_feat_coarsen<0>, cgrid, dim3(256), 0, s, op->lev[0].code, op->inv_rho64,
                       op->b, p, op->n, r, nc, net->coarse, part);
  ck_launch();
  hipLaunchKernelGGL(k_feat_rms, dim3(B), dim3(1024), 0, s, part, (int)cgrid.x, cells_c,
                     net->rms64, net->rms32);
  ck_launch();
  hipLaunchKernelGGL(k_feat_write, dim3(nb), dim3(256), 0, s, net->coarse, net->rms64, nc, B, x,
                     t);
  ck_launch();
}

}  // namespace

extern "C" {

int mpp_net_features(mpp_net net, mpp_op op, const double* f, const double* p, uint16_t* x,
                     float* t, float* rms, void* stream) {
  if (!net || !op || !f || !x || (t && !p) || !net_fits(op, net)) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  op->guess_f = nullptr;   // the learned guess's right-hand side is no longer current
  try {
    net_inputs(op, net, f, t ? p : nullptr, x, t, s);
    if (rms)
      ck(hipMemcpyAsync(rms, net->rms32, sizeof(float) * op->batch, hipMemcpyDeviceToDevice, s));
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

int mpp_learned_guess(mpp_op op, mpp_net net, const double* f, double* p, int32_t sweeps,
                      int32_t judge, int32_t* fell_back, void* stream) {
  if (!op || !net || !f || !p || f == p || sweeps < 0 || sweeps > 8 || !net_fits(op, net) ||
      (judge != MPP_JUDGE_PLAIN && judge != MPP_JUDGE_DEFLATED))
    return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int B = op->batch, r = op->n / net->n;
  const Level& L0 = op->lev[0];
  op->guess_f = nullptr;   // the learned guess's right-hand side is no longer current
  try {
    use_shift(op, 0.0, s);
    ensure_tuned<double>(op, s);
    ensure_tuned<float>(op, s);
    // the deflated judge needs the regions (their build uses the scratch vectors below)
    const bool dj = judge == MPP_JUDGE_DEFLATED;
    if (dj && !op->defl_ready) build_deflation(op, s);
    net_inputs(op, net, f, nullptr, net->x4, nullptr, s);
    const int st = mppnet::forward(net, net->x4, net->y, B, s);
    if (st != MPP_OK) return st;
    // a block per row of the fine grid
    const int nf = op->n;
    const dim3 pgrid((unsigned)nf * (unsigned)nf, B);
    const dim3 pblk(nf >= 256 ? 256 : 64 * ((nf + 63) / 64));
    if (r == 4)
      hipLaunchKernelGGL(k_guess_prolong<4>, pgrid, pblk, 0, s, net->y, net->rms64, net->n, r, p);
    else
      hipLaunchKernelGGL(k_guess_prolong<0>, pgrid, pblk, 0, s, net->y, net->rms64, net->n, r, p);
    ck_launch();
    Ctl& ctl = op->inner;
    // the mean of p (removed by the energy scaling below) and p.b in one pass, then p.Ap
    // (no A p stored): alpha = (p.b) / (p.Ap) scales p to the energy-norm optimum
    const Faces<double> F = faces_of<double>(op, 0);
    const dim3 g = grid_of(L0, B);
    hipLaunchKernelGGL(k_sum_dot, g, dim3(kBlock), 0, s, (const double*)p, (const double*)op->b,
                       (int)L0.cells, ctl);
    ck_launch();
    EpiArgs em = epi(E_STORE_MEAN);
    em.slot = S_SUM;
    em.inv_cells = 1.0 / (double)L0.cells;
    finish_sums(op, ctl, em, L0.bpp, s);
    EpiArgs e1 = epi(E_STORE_MEAN);
    e1.slot = S_RZ;
    e1.inv_cells = 1.0;
    Ctl shifted = ctl;   // the p.b partials follow the sum's
    shifted.partials += L0.bpp;
    finish_sums(op, shifted, e1, L0.bpp, s);
    EpiArgs e2 = e1;
    e2.slot = S_PQ;
    finish_sums(op, ctl, e2, launch_apply<double>(op, F, p, (double*)nullptr, ctl, 1, Sel{}, s),
                s);
    ck_launch();
    hipLaunchKernelGGL(k_energy_scale, g, dim3(kBlock), 0, s, p, (int)L0.cells, ctl.scal,
                       (int)S_RZ, (int)S_PQ, (int)S_SUM, (int)kSlots, op->z32);
    ck_launch();
    // red-black sweeps on A p = b in FP32 (b in r32 from the right-hand side's assembly,
    // p in z32 from the scaling), alternating between z32 and q32, then p in FP64; pf: the
    // guess in FP32 (p holds exactly its values)
    float* pf = op->z32;
    if (sweeps > 0) {
      float* bufs[2] = {op->z32, op->q32};
      pf = bufs[sweeps & 1];
      for (int q = 0; q < sweeps; ++q) {
        launch_rb<float, 0, true>(op, 0, op->kz[1][0], faces_of<float>(op, 0),
                                  (const float*)op->r32, (const float*)bufs[q & 1],
                                  (const float*)nullptr, bufs[(q + 1) & 1], 0, ctl, 0, Sel{}, s);
        ck_launch();
      }
      hipLaunchKernelGGL(k_widen, g, dim3(kBlock), 0, s, (const float*)bufs[sweeps & 1], p,
                         (int)L0.cells);
      ck_launch();
    }
    // the judge's residual norms in FP32 arithmetic (FP64 sums) on the same values: r in
    // d32 from b in r32 and the guess in pf
    const Faces<float> F32 = faces_of<float>(op, 0);
    if (!dj) {
      // fallback check on ||b - A p|| against ||b||
      finish_sums(op, ctl, epi(E_START),
                  launch_residual<float>(op, F32, op->r32, pf, op->d32, ctl, 0, s), s);
      ck_launch();
    } else {
      // the deflated solve starts from P (b - A p) with the guess and from P b without it:
      // ||P (b - A p)||^2 into S_RR, ||P b||^2 into S_BB (norms before the band correction
      // plus its change; problems without regions compare the plain norms)
      const Defl& D = op->defl;
      const int cells = (int)L0.cells;
      EpiArgs es = epi(E_STORE_MEAN);
      es.inv_cells = 1.0;
      const int parts = launch_residual<float>(op, F32, op->r32, pf, op->d32, ctl, 0, s);
      hipLaunchKernelGGL(k_region_sums<double>, dim3(op->defl_rblk, B), dim3(kDefThreads), 0, s,
                         (const double*)op->b, D.lab, cells, D, (const int*)nullptr);
      hipLaunchKernelGGL(k_defl_zb, dim3(B), dim3(64), 0, s, D, op->defl_rblk, (const int*)nullptr);
      hipLaunchKernelGGL(k_band_sums<float>, dim3(kDefBandBlocks, B), dim3(kDefThreads), 0, s,
                         (const float*)pf, cells, D, Sel{});
      hipLaunchKernelGGL(k_defl_coef, dim3(B), dim3(64), 0, s, D, 1, (const int*)nullptr);
      // (norms only: the band corrections are not stored)
      hipLaunchKernelGGL(k_band_fix<float>, dim3(kDefBandBlocks, B), dim3(kDefThreads), 0, s,
                         op->d32, cells, D, ctl, -1, parts, Sel{}, 0);
      ck_launch();
      es.slot = S_RR;
      finish_sums(op, ctl, es, parts + kDefBandBlocks, s);
      // ||b||^2 is in S_BB from the right-hand side's assembly: only the band's change
      hipLaunchKernelGGL(k_defl_coef, dim3(B), dim3(64), 0, s, D, 0, (const int*)nullptr);
      hipLaunchKernelGGL(k_band_fix<double>, dim3(kDefBandBlocks, B), dim3(kDefThreads), 0, s,
                         op->b, cells, D, ctl, -1, 0, Sel{}, 0);
      ck_launch();
      EpiArgs ea = epi(E_STORE_MEAN);
      ea.slot = S_BAND;
      ea.inv_cells = 1.0;
      finish_sums(op, ctl, ea, kDefBandBlocks, s);
    }
    ck(hipMemcpyAsync(op->h_scal, ctl.scal, sizeof(double) * B * kSlots, hipMemcpyDeviceToHost, s));
    ck(hipStreamSynchronize(s));
    for (int q = 0; q < B; ++q) {
      const double* sc = op->h_scal + (size_t)q * kSlots;
      // ||P b||^2 = ||b||^2 + the band's change on the deflated system
      const double bb = dj ? sc[S_BB] + sc[S_BAND] : sc[S_BB];
      const bool bad = !(std::isfinite(sc[S_RR]) && sc[S_RR] < bb);
      if (bad) ck(hipMemsetAsync(p + (size_t)q * L0.cells, 0, sizeof(double) * L0.cells, s));
      if (fell_back) fell_back[q] = bad ? 1 : 0;
    }
    op->guess_f = f;   // b, S_MEAN and S_BB of the inner control block are f's
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------
// the projection around the solve
// ------------------------------------------------------------------------------
namespace {

bool reinit_args_ok(int n, int batch, const double* phi0, const double* phi, int iters,
                    double dtau) {
  return n >= 2 && n <= 1024 && batch >= 1 && batch <= 65535 && phi0 && phi && iters >= 0 &&
         phi0 != phi && dtau > 0.0 && std::isfinite(dtau);
}

// iters re-distancing steps ping-ponging between phi and work; the result ends in phi
int reinit_run(int n, int batch, const double* phi0, double* phi, double* work, int iters,
               double dtau, hipStream_t s) {
  const int cells = n * n * n;
  const dim3 grid((cells + kLsBlock - 1) / kLsBlock, batch);
  const LsTiles tl = ls_tiles(n);
  const dim3 zgrid(8 * ((tl.ntiles + 7) / 8), batch);
  try {
    double* src = phi;
    double* dst = work;
    for (int it = 0; it < iters; ++it) {
      hipLaunchKernelGGL(k_ls_reinit_z, zgrid, dim3(kLsTX * kLsTY), 0, s, phi0, src, n, tl, dtau,
                         dst);
      ck_launch();
      std::swap(src, dst);
    }
    if (src != phi) {
      hipLaunchKernelGGL(k_ls_copy, grid, dim3(kLsBlock), 0, s, src, cells, phi);
      ck_launch();
    }
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

// Scratch of the allocation-free re-distancing entry point: one field of up to
// kReinitScratchDoubles values, a copy per device, held until the process ends.  In host
// code `scratch` names a host-side stand-in, never a device address: kernels and copies
// only ever get the device address that hipGetSymbolAddress returns for the current
// device, looked up once per device and kept in reinit_scratch_ptr.
constexpr size_t kReinitScratchDoubles = size_t(1) << 24;   // 128 MiB: one 256^3 field
static __device__ __align__(256) double scratch[kReinitScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int reinit_scratch(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return MPP_EDEVICE;
  if (dev >= kMaxDevices) return MPP_EDEVICE;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return MPP_EDEVICE;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return MPP_OK;
}

}  // namespace

extern "C" {

int mpp_divergence(mpp_op op, const double* ux, const double* uy, const double* uz, double dt,
                   double* f, void* stream) {
  if (!op || !ux || !uy || !uz || !f || !(dt > 0.0) || !std::isfinite(dt)) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Level& L0 = op->lev[0];
  op->guess_f = nullptr;   // the learned guess's right-hand side is no longer current
  try {
    hipLaunchKernelGGL(k_divergence, grid_of(L0, op->batch), dim3(kBlock), 0, s, ux, uy, uz, op->n,
                       (int)L0.cells, dt, f);
    ck_launch();
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

int mpp_project(mpp_op op, const double* phi, const double* p, double dt, double* ux, double* uy,
                double* uz, void* stream) {
  if (!op || !phi || !p || !ux || !uy || !uz || !(dt > 0.0) || !std::isfinite(dt))
    return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Level& L0 = op->lev[0];
  op->guess_f = nullptr;   // the learned guess's right-hand side is no longer current
  try {
    hipLaunchKernelGGL(k_project, grid_of(L0, op->batch), dim3(kBlock), 0, s, phi, op->kappa, p,
                       op->rho, op->n, (int)L0.cells, dt, ux, uy, uz);
    ck_launch();
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

int mpp_ls_advect(int n, int batch, const double* phi, const double* ux, const double* uy,
                  const double* uz, double dt, double* phi_out, void* stream) {
  if (n < 2 || n > 1024 || batch < 1 || batch > 65535 || !phi || !ux || !uy || !uz ||
      !phi_out || phi_out == phi || !(dt > 0.0) || !std::isfinite(dt))
    return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const LsTiles tl = ls_tiles(n);
  const dim3 grid(8 * ((tl.ntiles + 7) / 8), batch);
  try {
    hipLaunchKernelGGL(k_ls_advect_z, grid, dim3(kLsTX * kLsTY), 0, s, phi, ux, uy, uz, n, tl, dt,
                       phi_out);
    ck_launch();
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

int mpp_ls_reinit(int n, int batch, const double* phi0, double* phi, double* work, int iters,
                  double dtau, void* stream) {
  if (!reinit_args_ok(n, batch, phi0, phi, iters, dtau) || !work || phi0 == work || phi == work)
    return MPP_EINVAL;
  return reinit_run(n, batch, phi0, phi, work, iters, dtau, reinterpret_cast<hipStream_t>(stream));
}

int mpp_ls_reinit_noalloc(int n, int batch, const double* phi0, double* phi, int iters,
                          double dtau, void* stream) {
  if (!reinit_args_ok(n, batch, phi0, phi, iters, dtau)) return MPP_EINVAL;
  if ((size_t)n * n * n * (size_t)batch > kReinitScratchDoubles) return MPP_ENOMEM;
  double* work = nullptr;
  const int st = reinit_scratch(&work);
  if (st != MPP_OK) return st;
  if (work == phi0 || work == phi) return MPP_EINVAL;
  return reinit_run(n, batch, phi0, phi, work, iters, dtau, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"

// ------------------------------------------------------------------------------
// block-structured layout
// ------------------------------------------------------------------------------
namespace {

bool blk_ok(int n, int batch, int nb, int g) {
  return n >= 2 && n <= 1024 && batch >= 1 && batch <= 65535 && nb >= 2 && n % nb == 0 &&
         g >= 0 && g <= nb;
}

int blk_launch_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MPP_OK : MPP_EDEVICE;
}

}  // namespace

extern "C" {

int mpp_blocks_scatter(int n, int batch, int nb, int g, const double* grid, double* blocks,
                       void* stream) {
  if (!blk_ok(n, batch, nb, g) || !grid || !blocks || (const void*)grid == (const void*)blocks)
    return MPP_EINVAL;
  const BlkShape S = blk_shape(n, nb, g);
#define L_(NB_, G_)                                                                       \
  hipLaunchKernelGGL((k_blk_copy<0, NB_, G_>), dim3((unsigned)S.nblk, batch), dim3(kBlkThreads), \
                     0, reinterpret_cast<hipStream_t>(stream), S, grid, blocks)
  MPP_BLK_DISPATCH(S, L_);
#undef L_
  return blk_launch_status();
}

int mpp_blocks_gather(int n, int batch, int nb, int g, const double* blocks, double* grid,
                      void* stream) {
  if (!blk_ok(n, batch, nb, g) || !grid || !blocks || (const void*)grid == (const void*)blocks)
    return MPP_EINVAL;
  const BlkShape S = blk_shape(n, nb, g);
#define L_(NB_, G_)                                                                       \
  hipLaunchKernelGGL((k_blk_copy<1, NB_, G_>), dim3((unsigned)S.nblk, batch), dim3(kBlkThreads), \
                     0, reinterpret_cast<hipStream_t>(stream), S, blocks, grid)
  MPP_BLK_DISPATCH(S, L_);
#undef L_
  return blk_launch_status();
}

int mpp_blocks_fill_guards(int n, int batch, int nb, int g, double* blocks, void* stream) {
  if (!blk_ok(n, batch, nb, g) || !blocks) return MPP_EINVAL;
  if (g == 0) return MPP_OK;
  const BlkShape S = blk_shape(n, nb, g);
#define L_(NB_, G_)                                                                   \
  hipLaunchKernelGGL((k_blk_fill<NB_, G_>), dim3((unsigned)S.nblk, batch), dim3(kBlkThreads), \
                     0, reinterpret_cast<hipStream_t>(stream), S, blocks)
  MPP_BLK_DISPATCH(S, L_);
#undef L_
  return blk_launch_status();
}

int mpp_blocks_apply(mpp_op op, int nb, int g, const double* x_blocks, double* y_blocks,
                     void* stream) {
  if (!op || !x_blocks || !y_blocks || (const void*)x_blocks == (const void*)y_blocks)
    return MPP_EINVAL;
  if (!blk_ok(op->n, op->batch, nb, g) || g < 1) return MPP_EINVAL;
  const BlkShape S = blk_shape(op->n, nb, g);
  if (S.P3 * sizeof(double) > 65536) return MPP_EINVAL;   // the padded block is staged in LDS
  const Level& L0 = op->lev[0];
#define L_(NB_, G_)                                                                          \
  hipLaunchKernelGGL((k_blk_apply<NB_, G_>), dim3((unsigned)S.nblk, op->batch), dim3(kBlkThreads), \
                     S.P3 * sizeof(double), reinterpret_cast<hipStream_t>(stream), S, L0.f64[0], \
                     L0.f64[1], L0.f64[2], x_blocks, y_blocks)
  MPP_BLK_DISPATCH(S, L_);
#undef L_
  return blk_launch_status();
}

}  // extern "C"

// ------------------------------------------------------------------------------
// two-level composite grid
// ------------------------------------------------------------------------------
struct mpp_amr_s {
  AmrShape A;
  uint8_t* refined0;   // device [nblk0]
  int* map1;           // device [nbx1^3]
  int* list1;          // device [nblk1]
  std::vector<int> h_list1;
};

namespace {

bool amr_shape_ok(int n0, int nb, int g) {
  return n0 >= 2 && n0 <= 512 && nb >= 2 && n0 % nb == 0 && g >= 1 && g <= nb &&
         (size_t)(nb + 2 * g) * (nb + 2 * g) * (nb + 2 * g) <= (1u << 20);
}

size_t amr_table_bytes(int n0, int nb) {
  const size_t nbx0 = (size_t)(n0 / nb), nblk0 = nbx0 * nbx0 * nbx0;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  return up(nblk0) + up(sizeof(int) * 8 * nblk0) + up(sizeof(int) * 8 * nblk0) + 256;
}

}  // namespace

extern "C" {

size_t mpp_amr_workspace_bytes(int n0, int nb) {
  if (!(n0 >= 2 && n0 <= 512 && nb >= 2 && n0 % nb == 0)) return 0;
  return amr_table_bytes(n0, nb);
}

int mpp_amr_create(int n0, int nb, int g, const uint8_t* refined0, void* workspace,
                   size_t workspace_bytes, void* stream, mpp_amr* out) {
  if (out) *out = nullptr;
  if (!amr_shape_ok(n0, nb, g) || !refined0 || !workspace || !out) return MPP_EINVAL;
  if (workspace_bytes < amr_table_bytes(n0, nb)) return MPP_ENOMEM;
  AmrShape A;
  A.n0 = n0;
  A.nb = nb;
  A.g = g;
  A.P = nb + 2 * g;
  A.P3 = (size_t)A.P * A.P * A.P;
  A.nbx0 = n0 / nb;
  A.nbx1 = 2 * A.nbx0;
  A.nblk0 = A.nbx0 * A.nbx0 * A.nbx0;
  // the face factors, each 1 / (centre distance * cell volume / face area)
  const double h0 = 1.0 / n0, h1 = 0.5 * h0;
  A.same0 = 1.0 / (h0 * h0);
  A.same1 = 1.0 / (h1 * h1);
  A.fine_side = 1.0 / (1.5 * h1 * h1);
  A.coarse_side = 1.0 / (12.0 * h1 * h1);
  std::vector<int> map1((size_t)A.nbx1 * A.nbx1 * A.nbx1, -1), list1;
  std::vector<uint8_t> ref(A.nblk0);
  for (int b = 0; b < A.nblk0; ++b) {
    ref[b] = refined0[b] ? 1 : 0;
    if (!ref[b]) continue;
    const int bi = b % A.nbx0, bj = (b / A.nbx0) % A.nbx0, bk = b / (A.nbx0 * A.nbx0);
    for (int ch = 0; ch < 8; ++ch) {
      const int pos = (2 * bi + (ch & 1)) + A.nbx1 * ((2 * bj + ((ch >> 1) & 1)) +
                                                      A.nbx1 * (2 * bk + (ch >> 2)));
      map1[pos] = (int)list1.size();
      list1.push_back(pos);
    }
  }
  A.nblk1 = (int)list1.size();
  mpp_amr_s* a = new (std::nothrow) mpp_amr_s();
  if (!a) return MPP_ENOMEM;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(workspace) + 255) & ~uintptr_t(255));
  a->A = A;
  a->refined0 = reinterpret_cast<uint8_t*>(base);
  a->map1 = reinterpret_cast<int*>(base + up(A.nblk0));
  a->list1 = reinterpret_cast<int*>(base + up(A.nblk0) + up(sizeof(int) * 8 * A.nblk0));
  a->h_list1 = list1;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(a->refined0, ref.data(), ref.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(a->map1, map1.data(), sizeof(int) * map1.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !list1.empty())
    e = hipMemcpyAsync(a->list1, list1.data(), sizeof(int) * list1.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host tables go out of scope
  if (e != hipSuccess) {
    delete a;
    return MPP_EDEVICE;
  }
  *out = a;
  return MPP_OK;
}

void mpp_amr_destroy(mpp_amr a) { delete a; }

int mpp_amr_level1_blocks(mpp_amr a, int32_t* nblk1, int32_t* list1) {
  if (!a || !nblk1) return MPP_EINVAL;
  *nblk1 = a->A.nblk1;
  if (list1) std::copy(a->h_list1.begin(), a->h_list1.end(), list1);
  return MPP_OK;
}

int mpp_amr_fill_guards(mpp_amr a, double* blocks0, double* blocks1, void* stream) {
  if (!a || !blocks0 || (a->A.nblk1 > 0 && !blocks1) || blocks0 == blocks1) return MPP_EINVAL;
  const AmrShape& A = a->A;
#define L_(NB_, G_)                                                                          \
  hipLaunchKernelGGL((k_amr_fill<NB_, G_>), dim3((unsigned)(A.nblk0 + A.nblk1)), dim3(kBlkThreads), \
                     0, reinterpret_cast<hipStream_t>(stream), A, a->refined0, a->map1, a->list1, \
                     blocks0, blocks1)
  MPP_BLK_DISPATCH(A, L_);
#undef L_
  return blk_launch_status();
}

int mpp_amr_apply(mpp_amr a, const double* phi0, const double* phi1, const double* x0,
                  const double* x1, double rho_neg, double rho_pos, double* y0, double* y1,
                  void* stream) {
  if (!a || !phi0 || !x0 || !y0) return MPP_EINVAL;
  const AmrShape& A = a->A;
  if (A.nblk1 > 0 && (!phi1 || !x1 || !y1)) return MPP_EINVAL;
  if (!(rho_neg > 0.0) || !(rho_pos > 0.0) || !std::isfinite(rho_neg) || !std::isfinite(rho_pos))
    return MPP_EINVAL;
  const void* ins[4] = {phi0, phi1, x0, x1};
  for (const void* in : ins)
    if (in && (in == (const void*)y0 || in == (const void*)y1)) return MPP_EINVAL;
  if (y1 && y0 == y1) return MPP_EINVAL;
#define L_(NB_, G_)                                                                          \
  hipLaunchKernelGGL((k_amr_apply<NB_, G_>), dim3((unsigned)(A.nblk0 + A.nblk1), (NB_ == 16 && G_ == 1) ? 2 : 1), dim3(kBlkThreads), \
                     0, reinterpret_cast<hipStream_t>(stream), A, a->refined0, a->map1, a->list1, \
                     phi0, phi1, x0, x1, rho_neg, rho_pos, y0, y1)
  MPP_BLK_DISPATCH(A, L_);
#undef L_
  return blk_launch_status();
}

}  // extern "C"

namespace {

struct AmrWork {
  double* v[6][2];   // r, z, p, q, negd, t; each level 0 then level 1
  double* rc;        // averaged residual on the level-0 grid
  double* zc;        // its coarse correction
  double* part;      // [2][nblocks]
  double* S;         // [AS_COUNT]
  size_t bytes;      // total
};

AmrWork amr_work_layout(const AmrShape& A, void* base) {
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t n0 = (size_t)A.nblk0 * A.P3, n1 = (size_t)A.nblk1 * A.P3;
  const size_t vec = up(sizeof(double) * (n0 + n1));
  const size_t nblocks = (size_t)A.nblk0 + A.nblk1;
  AmrWork W;
  char* b = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(base) + 255) & ~uintptr_t(255));
  for (int i = 0; i < 6; ++i) {
    W.v[i][0] = reinterpret_cast<double*>(b + i * vec);
    W.v[i][1] = W.v[i][0] + n0;
  }
  const size_t grid = up(sizeof(double) * (size_t)A.n0 * A.n0 * A.n0);
  W.rc = reinterpret_cast<double*>(b + 6 * vec);
  W.zc = reinterpret_cast<double*>(b + 6 * vec + grid);
  W.part = reinterpret_cast<double*>(b + 6 * vec + 2 * grid);
  W.S = reinterpret_cast<double*>(b + 6 * vec + 2 * grid + up(sizeof(double) * 2 * nblocks));
  W.bytes = 6 * vec + 2 * grid + up(sizeof(double) * 2 * nblocks) + up(sizeof(double) * AS_COUNT) +
            256;
  return W;
}

void amr_launch_fill(const mpp_amr_s* a, double* b0, double* b1, hipStream_t s) {
  const AmrShape& A = a->A;
#define L_(NB_, G_)                                                                           \
  hipLaunchKernelGGL((k_amr_fill<NB_, G_>), dim3((unsigned)(A.nblk0 + A.nblk1)), dim3(kBlkThreads), \
                     0, s, A, a->refined0, a->map1, a->list1, b0, b1)
  MPP_BLK_DISPATCH(A, L_);
#undef L_
}

void amr_launch_apply(const mpp_amr_s* a, const double* phi0, const double* phi1,
                      const double* x0, const double* x1, double rn, double rp, double* y0,
                      double* y1, hipStream_t s) {
  const AmrShape& A = a->A;
#define L_(NB_, G_)                                                                           \
  hipLaunchKernelGGL((k_amr_apply<NB_, G_>),                                                  \
                     dim3((unsigned)(A.nblk0 + A.nblk1), (NB_ == 16 && G_ == 1) ? 2 : 1),     \
                     dim3(kBlkThreads), 0, s, A, a->refined0, a->map1, a->list1, phi0, phi1, x0, \
                     x1, rn, rp, y0, y1)
  MPP_BLK_DISPATCH(A, L_);
#undef L_
}

template <int MODE>
void amr_launch_vec(const mpp_amr_s* a, const AmrVecs& V, const AmrWork& W, hipStream_t s) {
  const AmrShape& A = a->A;
#define L_(NB_, G_)                                                                           \
  hipLaunchKernelGGL((k_amr_vec<MODE, NB_, G_>), dim3((unsigned)(A.nblk0 + A.nblk1)),        \
                     dim3(kBlkThreads), 0, s, A, a->refined0, a->list1, V, W.S, W.part)
  MPP_BLK_DISPATCH(A, L_);
#undef L_
}

// Two-level multigrid preconditioner z ~= (-A)^{-1} r, symmetric in the weighted inner
// product: kAmrNu damped Jacobi sweeps on -A z = r (the first from z = 0), the coarse
// correction (the residual r + A z averaged over every level-0 cell, one FP64 V-cycle of
// the level-0 operator on it, its negative given to every leaf of the cell), kAmrNu more
// sweeps; then the partial sums of <r, z> and <r, r> (and p = z when FIRST).
constexpr int kAmrNu = 1;
constexpr double kAmrOmega = 0.8;

template <bool FIRST>
void amr_precondition(const mpp_amr_s* a, mpp_op coarse, const double* phi0, const double* phi1,
                      double rn, double rp, const AmrVecs& V, const AmrWork& W, hipStream_t s) {
  const AmrShape& A = a->A;
  auto az = [&]() {   // t = A z
    amr_launch_fill(a, V.z[0], V.z[1], s);
    amr_launch_apply(a, phi0, phi1, V.z[0], V.z[1], rn, rp, V.t[0], V.t[1], s);
  };
  amr_launch_vec<AV_JAC0>(a, V, W, s);
  for (int i = 1; i < kAmrNu; ++i) {
    az();
    amr_launch_vec<AV_JAC>(a, V, W, s);
  }
  az();
  const size_t cells = (size_t)A.n0 * A.n0 * A.n0;
  const unsigned grid = (unsigned)std::min<size_t>((cells + kBlkThreads - 1) / kBlkThreads, 8192);
#define L_(NB_, G_)                                                                           \
  hipLaunchKernelGGL((k_amr_restrict<NB_, G_>), dim3(grid), dim3(kBlkThreads), 0, s, A,      \
                     a->refined0, a->map1, V.r[0], V.r[1], V.t[0], V.t[1], W.rc)
  MPP_BLK_DISPATCH(A, L_);
#undef L_
  use_shift(coarse, 0.0, s);
  ensure_tuned<double>(coarse, s);
  coarse->nu_c = 2;
  vcycle<double>(coarse, 0, W.rc, W.zc, 2, Sel{}, s);
  amr_launch_vec<AV_CADD>(a, V, W, s);
  for (int i = 0; i < kAmrNu; ++i) {
    az();
    amr_launch_vec<AV_JAC>(a, V, W, s);
  }
  amr_launch_vec<FIRST ? AV_ZDOTP : AV_ZDOT>(a, V, W, s);
}

void amr_launch_finish(const mpp_amr_s* a, int mode, const AmrWork& W, hipStream_t s) {
  hipLaunchKernelGGL(k_amr_finish, dim3(1), dim3(kBlkThreads), 0, s, mode, W.part,
                     a->A.nblk0 + a->A.nblk1, W.S);
}

}  // namespace

extern "C" {

size_t mpp_amr_solve_work_bytes(mpp_amr a) {
  if (!a) return 0;
  return amr_work_layout(a->A, nullptr).bytes;
}

int mpp_amr_solve(mpp_amr a, mpp_op coarse, const double* phi0, const double* phi1,
                  double rho_neg, double rho_pos, const double* b0, const double* b1, double* x0,
                  double* x1, double rtol, int32_t max_iter, void* work, size_t work_bytes,
                  int32_t* iters, double* rel_resid, void* stream) {
  if (iters) *iters = 0;
  if (rel_resid) *rel_resid = 0.0;
  if (!a || !phi0 || !b0 || !x0 || !work) return MPP_EINVAL;
  const AmrShape& A = a->A;
  if (coarse && (coarse->n != A.n0 || coarse->batch != 1)) return MPP_EINVAL;
  if (A.nblk1 > 0 && (!phi1 || !b1 || !x1)) return MPP_EINVAL;
  if (!(rho_neg > 0.0) || !(rho_pos > 0.0) || !std::isfinite(rho_neg) || !std::isfinite(rho_pos))
    return MPP_EINVAL;
  if (!(rtol > 0.0) || max_iter < 0) return MPP_EINVAL;
  if ((const void*)x0 == (const void*)b0 || (const void*)x0 == (const void*)phi0 ||
      (x1 && ((const void*)x1 == (const void*)b1 || (const void*)x1 == (const void*)phi1)))
    return MPP_EINVAL;
  if (work_bytes < amr_work_layout(A, nullptr).bytes) return MPP_ENOMEM;
  const AmrWork W = amr_work_layout(A, work);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  AmrVecs V;
  for (int l = 0; l < 2; ++l) {
    V.x[l] = l ? x1 : x0;
    V.r[l] = W.v[0][l];
    V.z[l] = W.v[1][l];
    V.p[l] = W.v[2][l];
    V.q[l] = W.v[3][l];
    V.negd[l] = W.v[4][l];
    V.t[l] = W.v[5][l];
    V.b[l] = l ? b1 : b0;
  }
  V.zc = W.zc;
  V.omega = kAmrOmega;
  const char* base = reinterpret_cast<const char*>(W.v[0][0]);
  if (hipMemsetAsync(W.v[0][0], 0, (size_t)(reinterpret_cast<const char*>(W.S) - base) +
                                         sizeof(double) * AS_COUNT, s) != hipSuccess)
    return MPP_EDEVICE;
  {
    const AmrShape& AA = A;
#define L_(NB_, G_)                                                                           \
    hipLaunchKernelGGL((k_amr_negdiag<NB_, G_>), dim3((unsigned)(AA.nblk0 + AA.nblk1)),       \
                       dim3(kBlkThreads), 0, s, AA, a->refined0, a->map1, a->list1, phi0, phi1, \
                       rho_neg, rho_pos, W.v[4][0], W.v[4][1])
    MPP_BLK_DISPATCH(AA, L_);
#undef L_
  }
  // b' = b - <b, 1>, r = b' - A x, z = p = r / -diag
  amr_launch_vec<AV_MEAN>(a, V, W, s);
  amr_launch_finish(a, AF_MEAN, W, s);
  amr_launch_vec<AV_INIT>(a, V, W, s);
  amr_launch_finish(a, AF_BB, W, s);
  amr_launch_fill(a, x0, x1, s);
  amr_launch_apply(a, phi0, phi1, x0, x1, rho_neg, rho_pos, W.v[3][0], W.v[3][1], s);
  try {
    if (coarse) {
      amr_launch_vec<AV_R>(a, V, W, s);
      amr_precondition<true>(a, coarse, phi0, phi1, rho_neg, rho_pos, V, W, s);
    } else {
      amr_launch_vec<AV_RES>(a, V, W, s);
    }
  } catch (HipError& e) {
    return status_of(e.e);
  }
  amr_launch_finish(a, AF_RZ0, W, s);
  int st = MPP_ENOTCONVERGED, it = 0;
  const int check_every = 8;
  double h[AS_COUNT];
  for (;;) {
    if (it % check_every == 0 || it == max_iter) {
      if (hipMemcpyAsync(h, W.S, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return MPP_EDEVICE;
      if (!(h[AS_RR] > rtol * rtol * h[AS_BB])) {   // also b' = 0
        st = MPP_OK;
        break;
      }
      if (!std::isfinite(h[AS_RR]) || h[AS_FLAG] != 0.0) {
        st = MPP_EBREAKDOWN;
        break;
      }
      if (it == max_iter) break;
    }
    amr_launch_fill(a, W.v[2][0], W.v[2][1], s);
    amr_launch_apply(a, phi0, phi1, W.v[2][0], W.v[2][1], rho_neg, rho_pos, W.v[3][0], W.v[3][1], s);
    amr_launch_vec<AV_DOT>(a, V, W, s);
    amr_launch_finish(a, AF_ALPHA, W, s);
    if (coarse) {
      amr_launch_vec<AV_MOVE>(a, V, W, s);
      try {
        amr_precondition<false>(a, coarse, phi0, phi1, rho_neg, rho_pos, V, W, s);
      } catch (HipError& e) {
        return status_of(e.e);
      }
    } else {
      amr_launch_vec<AV_STEP>(a, V, W, s);
    }
    amr_launch_finish(a, AF_BETA, W, s);
    amr_launch_vec<AV_DIR>(a, V, W, s);
    ++it;
  }
  // x of zero weighted mean, then its true residual
  AmrVecs VX = V;
  VX.b[0] = x0;
  VX.b[1] = x1;
  amr_launch_vec<AV_MEAN>(a, VX, W, s);
  amr_launch_finish(a, AF_XMEAN, W, s);
  amr_launch_vec<AV_SHIFT>(a, V, W, s);
  amr_launch_vec<AV_INIT>(a, V, W, s);
  amr_launch_fill(a, x0, x1, s);
  amr_launch_apply(a, phi0, phi1, x0, x1, rho_neg, rho_pos, W.v[3][0], W.v[3][1], s);
  amr_launch_vec<AV_RES>(a, V, W, s);
  amr_launch_finish(a, AF_RR, W, s);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(h, W.S, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return MPP_EDEVICE;
  if (iters) *iters = it;
  if (rel_resid) *rel_resid = h[AS_BB] > 0.0 ? std::sqrt(h[AS_RR] / h[AS_BB]) : 0.0;
  return st;
}

}  // extern "C"

extern "C" {

int mpp_amr_coarse_operator(mpp_amr a, mpp_op op, const double* phi0, const double* phi1,
                            double rho_neg, double rho_pos, void* stream) {
  if (!a || !op || !phi0) return MPP_EINVAL;
  const AmrShape& A = a->A;
  if (op->n != A.n0 || op->batch != 1 || (A.nblk1 > 0 && !phi1)) return MPP_EINVAL;
  if (!(rho_neg > 0.0) || !(rho_pos > 0.0) || !std::isfinite(rho_neg) || !std::isfinite(rho_pos))
    return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Level& L0 = op->lev[0];
  const size_t cells = (size_t)A.n0 * A.n0 * A.n0;
  const unsigned grid = (unsigned)std::min<size_t>((cells + 255) / 256, 8192);
  try {
#define L_(NB_, G_)                                                                           \
    hipLaunchKernelGGL((k_amr_coarse_faces<NB_, G_>), dim3(grid), dim3(256), 0, s, A,         \
                       a->refined0, a->map1, phi0, phi1, rho_neg, rho_pos, L0.code, L0.f64[0],  \
                       L0.f64[1], L0.f64[2], L0.f32[0], L0.f32[1], L0.f32[2])
    MPP_BLK_DISPATCH(A, L_);
#undef L_
    ck_launch();
    // the coarser levels and the coarsest inverse from the new faces
    for (int l = 1; l < op->nlev; ++l) {
      Level& Lf = op->lev[l - 1];
      Level& Lc = op->lev[l];
      hipLaunchKernelGGL(k_coarsen_faces, grid_of(Lc, 1), dim3(kBlock), 0, s, Lf.f64[0], Lf.f64[1],
                         Lf.f64[2], Lf.n, Lc.f64[0], Lc.f64[1], Lc.f64[2], Lc.f32[0], Lc.f32[1],
                         Lc.f32[2]);
      ck_launch();
    }
    factor_coarsest(op, s);
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

}  // extern "C"
