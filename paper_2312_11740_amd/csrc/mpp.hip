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
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.h"

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
  if (!d || d->n < 2 || d->n > 1024 || d->batch < 1 || d->batch > 65535 || d->flags != 0)
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
      lv.b32 = cv.take<float>(cl);
      lv.x32 = cv.take<float>(cl);
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
  op->partials = cv.take<double>((size_t)B * op->pstride);
  op->counters = cv.take<unsigned>((size_t)B);
  for (Ctl* c : {&op->outer, &op->inner}) {
    c->scal = cv.take<double>((size_t)B * kSlots);
    c->active = cv.take<int>((size_t)B);
    c->iters = cv.take<int>((size_t)B);
    c->status = cv.take<int>((size_t)B);
    c->partials = op->partials;
    c->counters = op->counters;
    c->pstride = op->pstride;
  }
  return cv.off + 256;
}

template <typename T>
Faces<T> faces_of(const mpp_op_s* op, int l);

template <>
Faces<double> faces_of<double>(const mpp_op_s* op, int l) {
  const Level& lv = op->lev[l];
  return Faces<double>{l == 0 ? lv.code : nullptr, lv.f64[0], lv.f64[1], lv.f64[2], op->inv_rho64};
}
template <>
Faces<float> faces_of<float>(const mpp_op_s* op, int l) {
  const Level& lv = op->lev[l];
  return Faces<float>{l == 0 ? lv.code : nullptr, lv.f32[0], lv.f32[1], lv.f32[2], op->inv_rho32};
}

template <typename T> T* lvl_b(Level& L);
template <typename T> T* lvl_x(Level& L);
template <> double* lvl_b<double>(Level& L) { return L.b64; }
template <> double* lvl_x<double>(Level& L) { return L.x64; }
template <> float* lvl_b<float>(Level& L) { return L.b32; }
template <> float* lvl_x<float>(Level& L) { return L.x32; }

inline dim3 grid_of(const Level& lv, int B) { return dim3(lv.bpp, B); }

EpiArgs epi(int kind) {
  EpiArgs e{};
  e.kind = kind;
  return e;
}

// ------------------------------------------------------------------------------
// V-cycle: z ~= A^{-1} r, zero initial guess
// ------------------------------------------------------------------------------
template <typename T>
void vcycle(mpp_op_s* op, int l, const T* rhs, T* x, int nu, const int* active, hipStream_t s) {
  Level& L = op->lev[l];
  const int B = op->batch;
  if (l == op->nlev - 1) {
    hipLaunchKernelGGL(k_coarse_solve<T>, dim3(B), dim3(kBlock), 0, s, op->coarse_inv,
                       op->coarse_m, rhs, x, active);
    ck_launch();
    return;
  }
  const Faces<T> F = faces_of<T>(op, l);
  const dim3 g = grid_of(L, B);
  const int n = L.n, cells = (int)L.cells;
  auto smooth = [&](int colour, int from_zero) {
    hipLaunchKernelGGL(k_smooth<T>, g, dim3(kBlock), 0, s, F, n, cells, rhs, x, colour,
                       from_zero, active);
    ck_launch();
  };
  smooth(0, 1);
  smooth(1, 0);
  for (int q = 1; q < nu; ++q) {
    smooth(0, 0);
    smooth(1, 0);
  }
  Level& Lc = op->lev[l + 1];
  hipLaunchKernelGGL(k_resid_restrict<T>, grid_of(Lc, B), dim3(kBlock), 0, s, F, n, rhs, x,
                     lvl_b<T>(Lc), active);
  ck_launch();
  vcycle<T>(op, l + 1, lvl_b<T>(Lc), lvl_x<T>(Lc), nu, active, s);
  hipLaunchKernelGGL(k_prolong_add<T>, g, dim3(kBlock), 0, s, n, lvl_x<T>(Lc), x, active);
  ck_launch();
  for (int q = 0; q < nu; ++q) {
    smooth(1, 0);
    smooth(0, 0);
  }
}

bool any_active(mpp_op_s* op, const Ctl& ctl, hipStream_t s) {
  ck(hipMemcpyAsync(op->h_active, ctl.active, sizeof(int) * op->batch, hipMemcpyDeviceToHost, s));
  ck(hipStreamSynchronize(s));
  for (int b = 0; b < op->batch; ++b)
    if (op->h_active[b]) return true;
  return false;
}

// ------------------------------------------------------------------------------
// Preconditioned CG on -A for every problem whose ctl.active flag is set by the
// start epilogue.  Uses ctl.scal[S_TOL2] as the per-problem target on ||r||^2.
// ------------------------------------------------------------------------------
template <typename T>
void pcg(mpp_op_s* op, Ctl& ctl, const T* rhs, T* x, T* r, T* z, T* p, T* q, int nu,
         int check_every, int xzero, const EpiArgs& start, hipStream_t s) {
  Level& L0 = op->lev[0];
  const int B = op->batch;
  const dim3 g = grid_of(L0, B);
  const Faces<T> F = faces_of<T>(op, 0);
  const int n = L0.n, cells = (int)L0.cells;
  hipLaunchKernelGGL(k_residual<T>, g, dim3(kBlock), 0, s, F, n, cells, rhs, x, r, ctl, start,
                     xzero);
  ck_launch();
  if (!any_active(op, ctl, s)) return;
  EpiArgs erz = epi(E_RZ), epq = epi(E_PQ), err = epi(E_RR_ITER);
  erz.first = 1;
  vcycle<T>(op, 0, r, z, nu, ctl.active, s);
  hipLaunchKernelGGL(k_dot<T>, g, dim3(kBlock), 0, s, r, z, cells, ctl, erz, ctl.active);
  ck_launch();
  hipLaunchKernelGGL(k_update_p<T>, g, dim3(kBlock), 0, s, z, p, cells, ctl, 1);
  ck_launch();
  erz.first = 0;
  const int cap = ctl.max_iter + check_every + 1;
  for (int it = 0; it < cap; ++it) {
    hipLaunchKernelGGL((k_apply<T, true>), g, dim3(kBlock), 0, s, F, n, cells, p, q, ctl, epq,
                       ctl.active);
    ck_launch();
    hipLaunchKernelGGL(k_update_xr<T>, g, dim3(kBlock), 0, s, x, r, p, q, cells, ctl, err);
    ck_launch();
    if ((it + 1) % check_every == 0 && !any_active(op, ctl, s)) return;
    vcycle<T>(op, 0, r, z, nu, ctl.active, s);
    hipLaunchKernelGGL(k_dot<T>, g, dim3(kBlock), 0, s, r, z, cells, ctl, erz, ctl.active);
    ck_launch();
    hipLaunchKernelGGL(k_update_p<T>, g, dim3(kBlock), 0, s, z, p, cells, ctl, 0);
    ck_launch();
  }
  any_active(op, ctl, s);
}

void reset_ctl(mpp_op_s* op, Ctl& ctl, int max_iter, hipStream_t s) {
  const int B = op->batch;
  ck(hipMemsetAsync(ctl.active, 0, sizeof(int) * B, s));
  ck(hipMemsetAsync(ctl.iters, 0, sizeof(int) * B, s));
  ck(hipMemsetAsync(ctl.status, 0, sizeof(int) * B, s));
  ck(hipMemsetAsync(ctl.scal, 0, sizeof(double) * B * kSlots, s));
  ctl.max_iter = max_iter;
}

// b = f + jterm - mean, into `out`; S_MEAN of ctl
void make_rhs(mpp_op_s* op, Ctl& ctl, const double* f, double* out, hipStream_t s,
              double rtol, bool want_bb) {
  const Level& L0 = op->lev[0];
  const dim3 g = grid_of(L0, op->batch);
  const int cells = (int)L0.cells;
  EpiArgs em = epi(E_MEAN);
  em.inv_cells = 1.0 / (double)L0.cells;
  hipLaunchKernelGGL(k_rhs_sum, g, dim3(kBlock), 0, s, f, op->jterm, out, cells, ctl, em);
  ck_launch();
  EpiArgs eb = epi(E_BB);
  eb.rtol2 = rtol * rtol;
  hipLaunchKernelGGL(k_sub_mean_sq, g, dim3(kBlock), 0, s, out, cells, ctl, eb, (int)S_MEAN,
                     want_bb ? 1 : 0);
  ck_launch();
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
  hipLaunchKernelGGL(k_sub_mean_sq, g, dim3(kBlock), 0, s, x, cells, ctl, e, (int)S_SUM, 0);
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
  o->check_every = 2;
  o->inner_rtol = 1e-5;
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

int mpp_build_operator(const mpp_desc* desc, const double* phi, const double* rho_neg,
                       const double* rho_pos, const double* sigma, void* workspace,
                       size_t workspace_bytes, void* stream, mpp_op* out) {
  if (out) *out = nullptr;
  if (!desc_ok(desc) || !phi || !rho_neg || !rho_pos || !sigma || !workspace || !out)
    return MPP_EINVAL;
  const int B = desc->batch;
  std::vector<double> host(3 * (size_t)B);
  for (int b = 0; b < B; ++b) {
    const double rn = rho_neg[b], rp = rho_pos[b], sg = sigma[b];
    if (!(rn > 0.0) || !(rp > 0.0) || !std::isfinite(rn) || !std::isfinite(rp) ||
        !(sg >= 0.0) || !std::isfinite(sg))
      return MPP_EINVAL;
    host[3 * b + 0] = rn;
    host[3 * b + 1] = rp;
    host[3 * b + 2] = sg;
  }
  mpp_op_s* op = new (std::nothrow) mpp_op_s();
  if (!op) return MPP_ENOMEM;
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(workspace) + 255) & ~uintptr_t(255));
  const size_t need = layout(op, desc, nullptr);
  if (workspace_bytes < need) {
    delete op;
    return MPP_ENOMEM;
  }
  layout(op, desc, base);
  op->ws = workspace;
  op->ws_bytes = workspace_bytes;
  op->h_active = new int[B];
  op->h_iters = new int[B];
  op->h_status = new int[B];
  op->h_scal = new double[(size_t)B * kSlots];
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  try {
    ck(hipMemcpyAsync(op->rho, host.data(), sizeof(double) * 3 * B, hipMemcpyHostToDevice, s));
    ck(hipMemsetAsync(op->counters, 0, sizeof(unsigned) * B, s));
    // a scratch int for the non-finite flag: reuse the outer status array
    ck(hipMemsetAsync(op->outer.status, 0, sizeof(int) * B, s));
    hipLaunchKernelGGL(k_params, dim3((B + 255) / 256), dim3(256), 0, s, op->rho, op->inv_rho64,
                       op->inv_rho32, B);
    ck_launch();
    Level& L0 = op->lev[0];
    const int n = op->n, cells = (int)L0.cells;
    const dim3 g = grid_of(L0, B);
    hipLaunchKernelGGL(k_faces, g, dim3(kBlock), 0, s, phi, op->rho, n, cells, L0.code,
                       L0.f64[0], L0.f64[1], L0.f64[2], L0.f32[0], L0.f32[1], L0.f32[2],
                       op->outer.status);
    ck_launch();
    hipLaunchKernelGGL(k_curvature, g, dim3(kBlock), 0, s, phi, L0.code, n, cells, op->kappa);
    ck_launch();
    hipLaunchKernelGGL(k_jump, g, dim3(kBlock), 0, s, phi, L0.code, op->kappa, op->rho, n, cells,
                       op->jterm);
    ck_launch();
    for (int l = 1; l < op->nlev; ++l) {
      Level& Lf = op->lev[l - 1];
      Level& Lc = op->lev[l];
      hipLaunchKernelGGL(k_coarsen_faces, grid_of(Lc, B), dim3(kBlock), 0, s, Lf.f64[0],
                         Lf.f64[1], Lf.f64[2], Lf.n, Lc.f64[0], Lc.f64[1], Lc.f64[2], Lc.f32[0],
                         Lc.f32[1], Lc.f32[2]);
      ck_launch();
    }
    const Level& Lc = op->lev[op->nlev - 1];
    hipLaunchKernelGGL(k_coarse_factor, dim3(B), dim3(kBlock), 0, s, Lc.f64[0], Lc.f64[1],
                       Lc.f64[2], Lc.n, op->coarse_work, op->coarse_inv);
    ck_launch();
    ck(hipMemcpyAsync(op->h_status, op->outer.status, sizeof(int) * B, hipMemcpyDeviceToHost, s));
    ck(hipStreamSynchronize(s));
  } catch (HipError& e) {
    delete[] op->h_active; delete[] op->h_iters; delete[] op->h_status; delete[] op->h_scal;
    delete op;
    return status_of(e.e);
  }
  for (int b = 0; b < B; ++b)
    if (op->h_status[b]) {
      delete[] op->h_active; delete[] op->h_iters; delete[] op->h_status; delete[] op->h_scal;
      delete op;
      return MPP_EINVAL;  // non-finite phi
    }
  *out = op;
  return MPP_OK;
}

void mpp_destroy_operator(mpp_op op) {
  if (!op) return;
  delete[] op->h_active;
  delete[] op->h_iters;
  delete[] op->h_status;
  delete[] op->h_scal;
  delete op;
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
  try {
    const Level& L0 = op->lev[0];
    hipLaunchKernelGGL((k_apply<double, false>), grid_of(L0, op->batch), dim3(kBlock), 0, s,
                       faces_of<double>(op, 0), L0.n, (int)L0.cells, x, y, op->outer, epi(0),
                       (const int*)nullptr);
    ck_launch();
  } catch (HipError& e) {
    return status_of(e.e);
  }
  return MPP_OK;
}

int mpp_rhs(mpp_op op, const double* f, double* b, double* mean_out, void* stream) {
  if (!op || !f || !b) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
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
  try {
    vcycle<double>(op, 0, r, z, nu, nullptr, s);
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
  const mpp_solve_opts& o = *opts;
  if (!(o.rtol > 0.0) || o.max_iter < 1 || o.nu < 1 || o.check_every < 1 ||
      (o.mode != MPP_MODE_FP64 && o.mode != MPP_MODE_MIXED) ||
      (o.guess != MPP_GUESS_ZERO && o.guess != MPP_GUESS_GIVEN))
    return MPP_EINVAL;
  if (o.mode == MPP_MODE_MIXED && !(o.inner_rtol > 0.0 && o.inner_rtol < 1.0)) return MPP_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int B = op->batch;
  const Level& L0 = op->lev[0];
  const dim3 g = grid_of(L0, B);
  const int cells = (int)L0.cells;
  std::vector<int> outer_count(B, 0);
  std::vector<int> istatus(B, MPP_OK);
  try {
    Ctl& oc = op->outer;
    reset_ctl(op, oc, o.max_iter, s);
    make_rhs(op, oc, f, op->b, s, o.rtol, true);
    if (o.guess == MPP_GUESS_ZERO) {
      hipLaunchKernelGGL(k_fill<double>, g, dim3(kBlock), 0, s, p, cells, 0.0);
      ck_launch();
    }
    EpiArgs start = epi(E_START);
    if (o.mode == MPP_MODE_FP64) {
      for (int restart = 0; restart < 4; ++restart) {
        pcg<double>(op, oc, op->b, p, op->r, op->z, op->p, op->q, o.nu, o.check_every, 0, start, s);
        // true residual; re-arms the problems that are not there yet
        hipLaunchKernelGGL(k_residual<double>, g, dim3(kBlock), 0, s, faces_of<double>(op, 0),
                           L0.n, cells, op->b, p, op->r, oc, start, 0);
        ck_launch();
        for (int b = 0; b < B; ++b) outer_count[b] += 1;
        if (!any_active(op, oc, s)) break;
      }
    } else {
      Ctl& ic = op->inner;
      reset_ctl(op, ic, o.max_iter, s);
      EpiArgs istart = epi(E_START_REL);
      istart.rtol2 = o.inner_rtol * o.inner_rtol;
      istart.gate = oc.active;
      bool settled = false;
      for (int outer = 0; outer < 40 && !settled; ++outer) {
        hipLaunchKernelGGL(k_residual<double>, g, dim3(kBlock), 0, s, faces_of<double>(op, 0),
                           L0.n, cells, op->b, p, op->r, oc, start, 0);
        ck_launch();
        if (!any_active(op, oc, s)) {
          settled = true;
          break;
        }
        for (int b = 0; b < B; ++b) outer_count[b] += op->h_active[b];
        hipLaunchKernelGGL(k_scale_down, g, dim3(kBlock), 0, s, op->r, op->r32, cells, oc.scal,
                           oc.active);
        ck_launch();
        hipLaunchKernelGGL(k_fill<float>, g, dim3(kBlock), 0, s, op->d32, cells, 0.0f);
        ck_launch();
        pcg<float>(op, ic, op->r32, op->d32, op->r32, op->z32, op->p32, op->q32, o.nu,
                   o.check_every, 1, istart, s);
        hipLaunchKernelGGL(k_correct, g, dim3(kBlock), 0, s, p, op->d32, cells, oc.scal, oc.active);
        ck_launch();
        // an inner breakdown or an exhausted iteration budget ends the refinement
        ck(hipMemcpyAsync(op->h_status, ic.status, sizeof(int) * B, hipMemcpyDeviceToHost, s));
        ck(hipStreamSynchronize(s));
        for (int b = 0; b < B; ++b)
          if (op->h_status[b] != MPP_OK) settled = true;
      }
      // final true residual of the returned iterate
      hipLaunchKernelGGL(k_residual<double>, g, dim3(kBlock), 0, s, faces_of<double>(op, 0),
                         L0.n, cells, op->b, p, op->r, oc, start, 0);
      ck_launch();
    }
    remove_mean(op, oc, p, s);
    ck(hipMemcpyAsync(op->h_scal, oc.scal, sizeof(double) * B * kSlots, hipMemcpyDeviceToHost, s));
    ck(hipMemcpyAsync(op->h_status, oc.status, sizeof(int) * B, hipMemcpyDeviceToHost, s));
    ck(hipMemcpyAsync(op->h_iters, (o.mode == MPP_MODE_FP64 ? oc.iters : op->inner.iters),
                      sizeof(int) * B, hipMemcpyDeviceToHost, s));
    ck(hipMemcpyAsync(op->h_active, oc.active, sizeof(int) * B, hipMemcpyDeviceToHost, s));
    if (o.mode == MPP_MODE_MIXED)
      ck(hipMemcpyAsync(istatus.data(), op->inner.status, sizeof(int) * B, hipMemcpyDeviceToHost, s));
    ck(hipStreamSynchronize(s));
  } catch (HipError& e) {
    return status_of(e.e);
  }
  int worst = MPP_OK;
  for (int b = 0; b < B; ++b) {
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
    if (!std::isfinite(sc[S_BB])) in.status = MPP_EINVAL;   // non-finite f
    else if (in.status == MPP_OK && !(in.rel_resid <= o.rtol)) in.status = MPP_ENOTCONVERGED;
    worst = worse(worst, in.status);
  }
  return worst;
}

}  // extern "C"
