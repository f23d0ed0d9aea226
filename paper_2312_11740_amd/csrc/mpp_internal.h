// Internal declarations of the gfx950 pressure-projection library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "mpp.h"

namespace mpp {

constexpr int kMaxLevels = 16;
constexpr int kBlock = 256;           // threads per block of the cell kernels
constexpr int kMaxCoarse = 1000;      // cells of the coarsest level (direct solve)

// per-problem scalar slots of a solve (doubles)
enum Slot {
  S_MEAN = 0,   // mean projected out of f + jterm
  S_BB,         // ||b||^2
  S_TOL2,       // rtol^2 * ||b||^2: convergence threshold on ||r||^2
  S_RR,         // ||r||^2 of the recurrence (or of the true residual after a restart)
  S_RZ,         // r.z of the current iteration
  S_BETA,       // rz_new / rz_old
  S_PQ,         // p.q
  S_ALPHA,      // rz / pq
  S_SCALE,      // mixed mode: ||r|| of the outer residual that scaled the inner rhs
  S_SUM,        // scratch sum (means)
  S_DT,         // heat diffusion: the time step (read by the kernels, so captured
                //   iteration graphs stay valid for any dt)
  S_BAND,       // learned guess: the band's change of ||b||^2 on the deflated system
  kSlots = 16
};

// Convergence bookkeeping shared by the kernels of one PCG run (device pointers).
struct Ctl {
  double* scal;         // [B][kSlots]
  int* active;          // [B] 1 while the problem iterates
  int* iters;           // [B] iterations done
  int* status;          // [B] MPP_OK / MPP_ENOTCONVERGED / MPP_EBREAKDOWN
  double* partials;     // [B][pstride] block partial sums
  unsigned* counters;   // [B] arrival counters of the last-block reductions (kept 0)
  int pstride;
  int max_iter;
  const int* list;      // while CG iterates: the problems its launches serve (Sel), else nullptr
};

// The problems a launch serves.  Block row y (blockIdx.y; blockIdx.x for the kernels with
// one block per problem) serves problem y, or with a list problem list[1 + y] while
// y < list[0] and nothing on the rows past that; a problem whose active flag is 0 is
// skipped.  A listed launch has as many rows as the live count of the last poll rounded
// up to a power of two (never fewer than the list holds), so the late iterations of a
// batch, with few live problems, launch few rows.
struct Sel {
  const int* active = nullptr;   // [B] flags; nullptr: no problem skipped
  const int* list = nullptr;     // [1 + B] count, then problem indices in ascending order
};

__host__ __device__ inline Sel sel_of(const Ctl& c) { return Sel{c.active, c.list}; }

__device__ inline int row_problem(const int* list, int row) {
  return list ? (row < list[0] ? list[1 + row] : -1) : row;
}

// the problem of block row `row`, -1: the row has nothing to do
__device__ inline int sel_problem(const Sel& s, int row) {
  const int b = row_problem(s.list, row);
  return (b < 0 || (s.active && !s.active[b])) ? -1 : b;
}

// Face coefficients of one level, in precision T.  On the finest level `code`
// holds per cell: bits 0..5 set when the -x,+x,-y,+y,-z,+z face is crossed by the
// interface (its coefficient is read from bx/by/bz), bit 6 set on the "+" side; all
// other faces take 1/rho of the cell's side from inv_rho[2*b + side].  Coarse levels
// have code == nullptr and read every face from the arrays.
template <typename T>
struct Faces {
  const uint8_t* code;
  const T* bx;
  const T* by;
  const T* bz;
  const T* inv_rho;     // [B][2]
  T sig;                // diagonal shift of this level: the operator is A - sig I (0 for the
                        // pressure; 1/dt halved per coarser level for implicit diffusion)
};

struct Level {
  int n = 0;
  size_t cells = 0;         // n^3 per problem
  uint8_t* code = nullptr;  // level 0 only
  double* f64[3] = {nullptr, nullptr, nullptr};
  float* f32[3] = {nullptr, nullptr, nullptr};
  // V-cycle right-hand side and correction of this level (levels >= 1)
  double* b64 = nullptr;
  double* x64 = nullptr;
  double* t64 = nullptr;    // scratch for the out-of-place sweeps
  float* b32 = nullptr;
  float* x32 = nullptr;
  float* t32 = nullptr;
  int bpp = 1;              // blocks per problem of the cell kernels on this level
};

// Deflation of the light-phase regions (the kernels and the method: deflate.h).
constexpr int kDefMax = 32;          // regions per problem
constexpr int kDefPairs = 4;         // (region, value) pairs per band cell: own + 3 others
constexpr int kCclBatch = 8;         // labelling rounds launched between host checks
constexpr int kDefBandBlocks = 32;   // blocks over a problem's band list
constexpr int kDefRegionBlocks = 256;  // at most this many blocks over a problem's light cells

// Per-problem deflation state in device memory.
struct Defl {
  uint8_t* lab;      // [B][cells] region (1..k) of each cell, 0 outside every region
  int* bcell;        // [B][cap] band cells (cell index in the problem), in cell order
  uint32_t* blab;    // [B][cap] regions of the pairs, a byte each (byte 0: the cell's own)
  double* bval;      // [B][cap][kDefPairs] (A z_j) at the cell
  int* bcount;       // [B] band cells (0: the problem is not deflated)
  int* k;            // [B] regions (0: not deflated)
  double* einv;      // [B][kDefMax][kDefMax] E^{-1}
  double* zb;        // [B][kDefMax] Z^T b of the right-hand side of the current CG
  double* coef;      // [B][kDefMax] a = E^{-1} s (per iteration) / the start and end terms
  double* part;      // [B][pcap][kDefMax] per-block sums over regions
  int* light;        // [B][lcap] cells of the lighter phase, in cell order
  int* lcount;       // [B] their number (0: the problem is not deflated)
  int cap;           // band cells a problem can hold
  int lcap;          // light-phase cells a problem can hold
  int pcap;          // blocks of part per problem
};

// Kernel classes timed by the profiler.
enum KernelId {
  K_APPLY_DOT = 0,   // q = A p and p.q
  K_RESIDUAL,        // r = b - A x and ||r||^2
  K_SMOOTH,          // one colour of red-black Gauss-Seidel, in place
  K_RESID_RESTRICT,  // coarse rhs = mean over children of b - A x
  K_PROLONG,         // x += parent value
  K_DOT,             // r.z
  K_UPDATE_P,        // p = z + beta p
  K_UPDATE_XR,       // x += alpha p, r -= alpha q, ||r||^2
  K_COARSE_VCYCLE,   // all levels below the finest, one record per V-cycle
  K_APPLY,           // y = A x
  K_RB_ZERO,         // fused red-black sweep from a zero iterate (finest level)
  K_RB,              // fused red-black sweep
  K_RB_PROLONG,      // fused red-black sweep after adding the coarse correction
  K_HEAT_APPLY,      // q = (dt A - I) p and p.q
  K_HEAT_RESIDUAL,   // r = b - (dt A - I) x and ||r||^2
  K_HEAT_JACOBI,     // z = r / diag and r.z
  K_DEFL,            // deflation: band sums, the corrected p.q, the band correction of r
  kKernelIds
};

struct ProfRec {
  int kid;
  hipEvent_t a, b;
  double bytes;
};

struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<ProfRec> recs;
  double ms[kKernelIds] = {};
  double bytes[kKernelIds] = {};
  long launches[kKernelIds] = {};
};

// A captured block of CG iterations and what it was captured for.
struct GraphKey {
  int tsize, nu, nu_c, iters, max_iter;
  int defl, tail, rows, first;
  const void* ptr[6];
  double shift = 0.0;   // the operator's diagonal shift (a kernel argument in the graph)
  bool operator==(const GraphKey& o) const {
    if (tsize != o.tsize || nu != o.nu || nu_c != o.nu_c || iters != o.iters ||
        max_iter != o.max_iter || defl != o.defl || tail != o.tail || rows != o.rows ||
        first != o.first || shift != o.shift)
      return false;
    for (int q = 0; q < 6; ++q)
      if (ptr[q] != o.ptr[q]) return false;
    return true;
  }
};

struct GraphEntry {
  GraphKey key;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

}  // namespace mpp

struct mpp_op_s {
  mpp::Prof prof;
  bool use_graphs = true;
  std::vector<mpp::GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;
  double* x = nullptr;              // FP64 iterate (the caller's p is copied in and out)
  int kz[2][mpp::kMaxLevels] = {};  // tuned z-chunk of the fused sweeps [fp32?][level], 0 = default
  // the sweep kernels tuned for a batch of which one problem is left (the tail of a
  // batched solve: few live problems want more, smaller tiles each)
  int kz_tail[2][mpp::kMaxLevels] = {};
  bool tail = false;                // the CG block being run uses kz_tail
  int* tail_mask = nullptr;         // [B] device: problem 0 active (tuning the tail)
  int* live = nullptr;              // [1 + B] device: the list of the CG iterations (Sel)
  int rows = 0;                     // block rows of the listed launches
  bool tuned[2] = {false, false};
  int nu_c = 2;                     // sweeps per level below the finest
  int n = 0, batch = 0, nlev = 0;
  uint32_t flags = 0;
  mpp::Level lev[mpp::kMaxLevels];
  size_t cells = 0;
  int coarse_m = 0;
  double* coarse_inv = nullptr;   // [B][m][m] inverse of (-A_c + 11^T/m), or of (-A_c + sig_c I)
  double shift = 0.0;             // diagonal shift of the finest level in use (0: pressure)
  double coarse_shift = 0.0;      // the coarsest level's shift coarse_inv was built for
  double* coarse_work = nullptr;  // [B][m][m] factorisation scratch
  double* rho = nullptr;          // [B][3]: rho_neg, rho_pos, sigma
  double* inv_rho64 = nullptr;    // [B][2]
  float* inv_rho32 = nullptr;     // [B][2]
  double* kappa = nullptr;        // [B][cells]
  double* jterm = nullptr;        // [B][cells]
  // FP64 PCG vectors
  double *b = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  // FP32 inner vectors (mixed mode)
  float *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr;
  // control
  mpp::Ctl outer{}, inner{};
  double* partials = nullptr;
  unsigned* counters = nullptr;
  int pstride = 0;
  // deflation (built at the first deflated solve after a build or update)
  mpp::Defl defl{};
  double* defl_e = nullptr;       // [B][kDefMax][kDefMax] E = Z^T A Z
  int* defl_light = nullptr;      // [B] side bit of the lighter phase, -1: none
  int* defl_flag = nullptr;       // [kCclBatch][B] changed flags of a batch of labelling rounds
  int* defl_total = nullptr;      // [B] totals of the compactions
  int* defl_over = nullptr;       // [B] problems whose deflation does not fit
  int defl_rblk = 1;              // blocks per problem of the region sums
  bool defl_ready = false;        // built for the current operator
  bool defl_use = false;          // the CG being run is deflated
  std::vector<int> h_defl_light;  // host: side bit of the lighter phase per problem, -1 none
  bool defl_any = false;          // some problem is deflated
  std::vector<int> h_defl_k;      // host copy of defl.k
  // host mirrors for polling
  int* h_active = nullptr;
  int* h_iters = nullptr;
  int* h_status = nullptr;
  double* h_scal = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // f of the last call on the operator when that was a learned guess (its right-hand side
  // is then in b, its mean and norm in the inner control block), else nullptr
  const double* guess_f = nullptr;
};
