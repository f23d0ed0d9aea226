/*
 * mpp.h -- C ABI of the MI355X (gfx950) multiphase pressure-projection solver.
 *
 * The library solves the variable-density pressure Poisson equation of a
 * fractional-step projection method,
 *
 *        div( (1/rho) grad p ) = f        on [0,1]^3, homogeneous Neumann walls,
 *
 * on a cell-centred n^3 grid.  Flash-X (arXiv 2312.11740) frames this step: Sec. 2
 * (staggered stencil: pressure, density and the level set at cell centres, vectors
 * on faces; signed level set phi > 0 in air and < 0 in liquid), Sec. 3 (IncompNS
 * varDens with density set from the level set by the Multiphase unit, and the
 * multigrid Poisson solver behind Grid_solvePoisson).  The discrete operator is
 *
 *        (A p)_c = sum over the 6 faces f of c of beta_f (p_nb - p_c) / h^2,  h = 1/n,
 *
 * with beta_f = 1/rho of the phase when both cells lie on the same side of the
 * interface, beta_f = 1/(theta rho_a + (1-theta) rho_b) on a face crossed by it
 * (ghost-fluid coefficient of Liu, Fedkiw & Kang, theta = |phi_a|/(|phi_a|+|phi_b|)),
 * and 0 through walls.  A cell with phi > 0 is on the "+" side (density rho_pos), a
 * cell with phi <= 0 on the "-" side (rho_neg).
 *
 * The surface-tension jump [p] = p(+) - p(-) = sigma*kappa, kappa = -div(grad phi /
 * |grad phi|) from central differences of phi, enters the right-hand side
 * (ghost-fluid method of Kang, Fedkiw & Liu): b = f + jterm, then b -= mean(b).
 * The solver returns the unique zero-mean p with A p = b to a relative residual
 * ||b - A p||_2 <= rtol ||b||_2, by conjugate gradients on -A preconditioned with a
 * geometric multigrid V-cycle.
 *
 * Around the solve (sections below): the projection that produces f from the face
 * velocities and corrects them with p; the level-set step that moves phi with the
 * corrected velocity and keeps it a distance; an implicit heat-diffusion step on the
 * same operator and multigrid (a diagonal shift per level); a block-structured layout
 * with guard cells; and a learned initial guess for the solve.
 *
 * Memory and layout.  Every array argument is DEVICE memory on the current HIP
 * device unless marked "host".  A grid field is n^3 doubles, x fastest: cell (i,j,k)
 * at offset i + n*(j + n*k).  Batched calls take [batch][n^3] contiguous fields.
 * The caller owns every array and the workspace; the library never allocates
 * device memory.  All work is enqueued on `stream` (a hipStream_t, NULL = default
 * stream); calls return after the results are complete on the stream, except where
 * stated.  One operator may be used by one call at a time: concurrent calls on the
 * same operator race on its workspace.
 *
 * Errors.  Every call returns MPP_OK or a negative status; no exception crosses the
 * ABI.  Invalid sizes, null pointers and non-positive or non-finite densities give
 * MPP_EINVAL before any device work; HIP failures give MPP_EDEVICE.
 */
#ifndef MPP_H
#define MPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPP_OK 0
#define MPP_EINVAL (-1)         /* invalid argument (size, pointer, density, sigma) */
#define MPP_ENOMEM (-2)         /* workspace too small */
#define MPP_EDEVICE (-3)        /* a HIP runtime call failed */
#define MPP_ENOTCONVERGED (-4)  /* max_iter reached; p holds the last iterate */
#define MPP_EBREAKDOWN (-5)     /* CG breakdown (non-positive curvature or NaN) */

/* solve modes */
#define MPP_MODE_FP64 0   /* FP64 throughout */
#define MPP_MODE_MIXED 1  /* FP64 residual refinement around an FP32 MG-PCG */

/* initial guess */
#define MPP_GUESS_ZERO 0
#define MPP_GUESS_GIVEN 1 /* p holds the initial guess on entry */

typedef struct mpp_op_s *mpp_op;

/* Problem shape.  n: cells per side, 2 <= n <= 1024, with n = m * 2^k for some
 * m <= 10 (the multigrid coarsens while the size is even and above 4; the coarsest
 * level, at most 10^3 cells, is solved directly).  batch: independent problems of
 * the same n solved together (>= 1). */
typedef struct {
    int32_t n;
    int32_t batch;
    uint32_t flags; /* 0 or MPP_FLAG_NO_GRAPHS */
} mpp_desc;

/* desc.flags: launch every kernel directly instead of replaying captured HIP graphs
 * of the CG iterations (same results; for debugging and profiling). */
#define MPP_FLAG_NO_GRAPHS 1u

typedef struct {
    double rtol;          /* relative residual target, e.g. 1e-10 */
    int32_t max_iter;     /* CG iterations (all inner iterations in mixed mode) */
    int32_t mode;         /* MPP_MODE_FP64 or MPP_MODE_MIXED */
    int32_t guess;        /* MPP_GUESS_ZERO or MPP_GUESS_GIVEN */
    int32_t nu;           /* pre- and post-smoothing red-black sweeps per level, >= 1 */
    int32_t check_every;  /* iterations between host polls of convergence, >= 1 */
    int32_t nu_coarse;    /* sweeps on the levels below the finest (0: nu) */
    double inner_rtol;    /* mixed mode: tightest inner FP32 target (e.g. 1e-5); each
                           * refinement step asks only for the reduction it still
                           * needs, between inner_rtol and 1/2 */
    int32_t deflate;      /* 1: deflate the regions of the lighter phase (below), 0: plain
                           * MG-PCG */
    int32_t reuse_rhs;    /* 1: when the previous call on this operator was
                           * mpp_learned_guess with the same f (whose contents the caller
                           * has not changed since), take the right-hand side that call
                           * assembled instead of assembling it again; otherwise, or 0,
                           * assemble it from f */
} mpp_solve_opts;

/* Deflation (opts->deflate = 1).  Every connected region of the lighter phase (a bubble,
 * through cell faces) adds a slow mode to the multigrid-preconditioned operator at a high
 * density ratio.  Up to 32 regions per problem (the first 32 by their smallest cell index)
 * are deflated: with Z the indicator fields of the regions and E = Z^T A Z, CG runs on
 * P A x = P b, P = I - A Z E^{-1} Z^T, and the solution takes x + Z E^{-1} Z^T (b - A x)
 * at the end (Nicolaides 1987; Tang & Vuik 2007).  The regions and the cells next to
 * their boundaries are found once per operator build, at the first deflated solve.  The
 * solution is the same (to the tolerance); only the iteration count changes.  Problems
 * with equal densities, no region or regions whose band exceeds an eighth of the cells
 * are solved without deflation.  Pressure solves only (mpp_heat_solve ignores it). */

typedef struct {
    int32_t status;       /* MPP_OK, MPP_ENOTCONVERGED or MPP_EBREAKDOWN */
    int32_t iters;        /* CG iterations (sum of inner iterations in mixed mode) */
    int32_t outer_iters;  /* FP64 refinement steps (mixed mode), else restarts + 1 */
    int32_t reserved;
    double rel_resid;     /* final true ||b - A p|| / ||b|| in FP64 */
    double removed_mean;  /* mean of f + jterm projected out of the right-hand side */
    double bnorm;         /* ||b||_2 after the projection */
} mpp_solve_info;

/* Default options: rtol 1e-10, max_iter 500, FP64, zero guess, nu 2, check_every 2,
 * nu_coarse 0 (as nu), inner_rtol 1e-5, deflate 1. */
void mpp_default_opts(mpp_solve_opts *opts);

/* Bytes of device workspace an operator of this shape needs (0 if desc is invalid). */
size_t mpp_workspace_bytes(const mpp_desc *desc);

/* Build the operator for level set phi (device, [batch][n^3]) and per-problem
 * densities and surface tension (host arrays of `batch` doubles: rho_neg > 0 for
 * phi <= 0, rho_pos > 0 for phi > 0, sigma >= 0; all finite).  Computes the face
 * coefficients, the interface curvature, the jump term and the multigrid hierarchy
 * (coarse coefficients as means of the fine ones, a dense factor of the coarsest
 * level) inside `workspace` (device, mpp_workspace_bytes(desc) bytes, 256-byte
 * aligned, owned by the caller and kept alive until mpp_destroy_operator).  On
 * success *out receives a handle (host memory owned by the library).  phi is read
 * during the call only.  The operator is immutable afterwards. */
int mpp_build_operator(const mpp_desc *desc, const double *phi, const double *rho_neg,
                       const double *rho_pos, const double *sigma, void *workspace,
                       size_t workspace_bytes, void *stream, mpp_op *out);

/* Rebuilds an operator in place for a new level set and new constants (same shape,
 * same workspace), e.g. once per time step of a projection method.  Arguments as
 * for mpp_build_operator.  Keeps the operator's captured launch graphs valid. */
int mpp_update_operator(mpp_op op, const double *phi, const double *rho_neg,
                        const double *rho_pos, const double *sigma, void *stream);

/* y = A x for every problem (device, [batch][n^3]); no jump term.  x and y must not
 * overlap.  Asynchronous: returns once the work is enqueued on the stream. */
int mpp_apply_stencil(mpp_op op, const double *x, double *y, void *stream);

/* Solve A p = f + jterm (mean-projected) for every problem.  f, p: device
 * [batch][n^3]; p is the initial guess on entry when opts->guess == MPP_GUESS_GIVEN
 * and the zero-mean solution on exit.  info: host array of `batch` records, filled
 * on every return that got past argument checks (also MPP_ENOTCONVERGED, where p
 * holds the last iterate).  Returns the worst status over the batch. */
int mpp_solve(mpp_op op, const double *f, double *p, const mpp_solve_opts *opts,
              mpp_solve_info *info, void *stream);

/* The right-hand side the solver uses: b = f + jterm, minus its mean (device
 * [batch][n^3]).  mean_out: host [batch], may be NULL (then asynchronous). */
int mpp_rhs(mpp_op op, const double *f, double *b, double *mean_out, void *stream);

/* One multigrid V-cycle as a preconditioner: z ~= A^{-1} r with zero initial guess,
 * nu red-black sweeps before and black-red sweeps after the coarse correction on
 * every level; FP64.  r, z: device [batch][n^3].  Asynchronous. */
int mpp_vcycle(mpp_op op, const double *r, double *z, int nu, void *stream);

/* Copies of the operator's data for inspection (device destinations, [batch][n^3]
 * each; any pointer may be NULL): face coefficients of the finest level (low face of
 * each cell, 0 on walls), curvature (0 away from the interface) and jump term. */
int mpp_operator_fields(mpp_op op, double *beta_x, double *beta_y, double *beta_z,
                        double *kappa, double *jterm, void *stream);

/* The deflation data of the operator (built now if a solve has not built it yet): the
 * region of every cell (labels: device [batch][n^3] bytes, 0 outside every region, or
 * NULL), the number of regions per problem (k: host [batch]; 0 when the problem is not
 * deflated) and E = Z^T A Z (host [batch][32][32], the first k rows and columns used, or
 * NULL).  Synchronous. */
int mpp_deflation_info(mpp_op op, uint8_t *labels, int32_t *k, double *E, void *stream);

/* Number of multigrid levels and the size of each (host array of up to 16). */
int mpp_levels(mpp_op op, int32_t *nlevels, int32_t *sizes);

/* Kernel timing.  Between mpp_profile_start and mpp_profile_stop every launch on the
 * finest level made by calls on this operator is bracketed by HIP events on the
 * call's stream (the levels below the finest are timed as one record per V-cycle).
 * stop waits for the events and returns, per kernel, the launch count, the summed
 * event time and the summed algorithmic bytes (each array the kernel must read or
 * write counted once; see the kernel descriptions in the library).  stats: host
 * array of max_stats records; *n_stats receives the number filled. */
typedef struct {
    char name[32];
    int32_t launches;
    int32_t reserved;
    double total_ms;
    double bytes;
} mpp_kernel_stat;

int mpp_profile_start(mpp_op op);
int mpp_profile_stop(mpp_op op, mpp_kernel_stat *stats, int32_t max_stats, int32_t *n_stats);

/* Releases the handle (not the caller's workspace). */
void mpp_destroy_operator(mpp_op op);


/* ------------------------------------------------------------------------------
 * The projection around the solve (the fractional step of the paper's Sec. 2 on the
 * staggered grid).  Face velocities are device [batch][n^3] arrays in the low-face
 * layout of the coefficients: ux[i,j,k] on the face between cells (i-1,j,k) and
 * (i,j,k); ux[0,j,k] is the wall face (read as 0; written as 0 by mpp_project); high
 * wall faces are implicit zeros.
 * ------------------------------------------------------------------------------ */

/* f = div(u)/dt at the cell centres: (sum over the axes of (u on the high face - u on
 * the low face) / h) / dt, h = 1/n.  f: device [batch][n^3].  dt > 0 and finite.
 * Asynchronous. */
int mpp_divergence(mpp_op op, const double *ux, const double *uy, const double *uz, double dt,
                   double *f, void *stream);

/* u = u - dt beta^ grad p on every interior face, with the gradient corrected by the
 * surface-tension jump: (p_b - p_a - d J) / h between the lower cell a and the upper
 * cell b, J = sigma ((1-theta) kappa_a + theta kappa_b) the jump at the face's crossing
 * and d = +1 when a is on the phi <= 0 side and b on the phi > 0 side, -1 for the
 * opposite crossing, 0 on faces the interface does not cross; beta^ the operator's
 * face coefficient.  This is the flux whose jump part the operator moved into its
 * right-hand side, so with p the solution for f = div(u*)/dt the result is discretely
 * divergence-free.  phi: the device level set the operator was built from; p: device
 * [batch][n^3]; ux, uy, uz updated in place.  Asynchronous. */
int mpp_project(mpp_op op, const double *phi, const double *p, double dt, double *ux,
                double *uy, double *uz, void *stream);

/* ------------------------------------------------------------------------------
 * Level set (Sec. 3: the Multiphase unit moves phi with the flow and, through
 * StencilsLevelSet, keeps it a signed distance).  The paper gives no scheme; this
 * library uses first-order upwind advection and smoothed-sign Godunov re-distancing,
 * FP64.  Cell fields are device [batch][n^3] arrays (x fastest); face velocities use
 * the low-face layout above.  Differences across a wall are 0.  These calls need no
 * operator.
 * ------------------------------------------------------------------------------ */

/* One forward-Euler step of phi_t + u . grad phi = 0: phi_out = phi - dt (a_x + a_y +
 * a_z), a_d = u_d D_d phi with u_d = (u on the low face + u on the high face) / 2 at the
 * cell centre and D_d the backward difference (phi_c - phi_{c-1}) / h when u_d > 0, the
 * forward difference (phi_{c+1} - phi_c) / h otherwise.  2 <= n <= 1024, 1 <= batch <=
 * 65535, dt > 0 and finite, phi_out distinct from phi.  Asynchronous. */
int mpp_ls_advect(int n, int batch, const double *phi, const double *ux, const double *uy,
                  const double *uz, double dt, double *phi_out, void *stream);

/* iters pseudo-time steps of size dtau of phi_tau + S (|grad phi| - 1) = 0, each from
 * the previous iterate: phi <- phi - dtau S (G - 1), S = phi0 / sqrt(phi0^2 + h^2), G =
 * sqrt(sum over the axes of max(t1^2, t2^2)) with (t1, t2) = (max(back, 0), min(fwd, 0))
 * where S > 0 and (min(back, 0), max(fwd, 0)) otherwise (Godunov upwinding).  phi0
 * (fixed signs, usually phi before the first step) is read only; phi is updated in
 * place; work is a caller-owned device scratch array of the same size.  The three
 * arrays must be distinct; iters >= 0, dtau > 0 (stable up to h/2 ~ 0.5/n).
 * Asynchronous. */
int mpp_ls_reinit(int n, int batch, const double *phi0, double *phi, double *work, int iters,
                  double dtau, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): mpp_ls_reinit without the work array.
 * The pseudo-time ping-pong uses a scratch field that the library holds for each GPU it
 * runs on until the process ends (2^24 doubles, 128 MiB: one 256^3 field); the call
 * allocates nothing.  n^3 * batch above 2^24 gives MPP_ENOMEM, other arguments as for
 * mpp_ls_reinit (MPP_EINVAL), all before any device work.  Results equal mpp_ls_reinit's
 * bit for bit.  Every call on one GPU shares that GPU's scratch field: calls that overlap
 * on one GPU (other streams, other threads) race and must be serialised by the caller.
 * Asynchronous. */
int mpp_ls_reinit_noalloc(int n, int batch, const double *phi0, double *phi, int iters,
                          double dtau, void *stream);

/* ------------------------------------------------------------------------------
 * Implicit heat diffusion (the diffusion term of the transport equation of Sec. 2
 * with a coefficient that changes with the phase: the varDiffusion configuration of
 * HeatAD, Sec. 3).  One backward-Euler step
 *        (I - dt div(K grad)) T = T_old + dt f,   insulated walls,
 * on an operator whose face coefficients are read as conductivities: build it with
 * rho_neg = 1/K_neg and rho_pos = 1/K_pos (K_neg where phi <= 0); crossed faces then
 * hold the two conductivities in series, split where the interface crosses the face.
 * Nothing else of the operator (curvature, jump term, multigrid levels) is used.
 * ------------------------------------------------------------------------------ */

/* t_old, t: device [batch][n^3]; src: device [batch][n^3] or NULL (no source).  t
 * holds the initial guess when opts->guess is MPP_GUESS_GIVEN (ignored with
 * MPP_GUESS_ZERO) and receives T; t may be t_old, src may not be t.  dt >= 0 and
 * finite.  Solved to ||b - H T|| <= opts->rtol ||b|| in FP64 (H = I - dt div(K grad),
 * b = T_old + dt f), with the true residual checked at the end.  opts->nu selects the
 * preconditioner:
 *   nu >= 1: the pressure solve's MG-PCG (opts->mode FP64 or MIXED, nu sweeps, the
 *            other options as for mpp_solve) on (A - I/dt) T = -(T_old + dt f)/dt,
 *            every level carrying its diagonal shift (1/dt, halved per coarser level);
 *   nu == 0: CG on (dt A - I) T = -(T_old + dt f) with the inverse diagonal (FP64;
 *            rtol, max_iter, check_every and guess are used); its iterations grow as
 *            the square root of 1 + 12 dt K_max / h^2.
 * dt == 0 gives T = T_old exactly (one iteration of the diagonal form).  info[batch] as
 * for mpp_solve (removed_mean 0).  Solves on the same operator may alternate with
 * pressure solves: the shift and the coarsest inverse follow the call.  Synchronous with
 * respect to the host.  Returns the worst status of the batch. */
int mpp_heat_solve(mpp_op op, const double *t_old, const double *src, double dt, double *t,
                   const mpp_solve_opts *opts, mpp_solve_info *info, void *stream);

/* ------------------------------------------------------------------------------
 * Block-structured layout (Sec. 2: the grid is a set of blocks of cells; the setup
 * command of Sec. 4 builds 16^3 blocks; Sec. 4's driver fills guard cells, exchanging
 * halos between blocks and applying the physical boundary condition, before the
 * physics works block by block).  A problem of n^3 cells is cut into (n/nb)^3 blocks
 * of nb^3 cells; block (bi, bj, bk) has index bi + (n/nb) (bj + (n/nb) bk) and is stored
 * as P^3 doubles, P = nb + 2 g (g guard layers on every side, x fastest, the interior at
 * offsets g .. g + nb - 1); problems follow each other: [batch][blocks][P^3].  Guard
 * cells hold the value of the cell at their position in the neighbouring block (faces,
 * edges and corners); outside the domain the field mirrored about the wall (even
 * reflection: the zero-gradient condition of the no-flux walls).
 * Common requirements: 2 <= n <= 1024, 1 <= batch <= 65535, 2 <= nb, n % nb == 0,
 * 0 <= g <= nb; device pointers; asynchronous on `stream`; MPP_EINVAL on a violated
 * requirement, MPP_EDEVICE if a launch fails.
 * ------------------------------------------------------------------------------ */

/* grid [batch][n^3] -> the block interiors (guards are not written); grid != blocks. */
int mpp_blocks_scatter(int n, int batch, int nb, int g, const double *grid, double *blocks,
                       void *stream);

/* the block interiors -> grid [batch][n^3]; grid != blocks. */
int mpp_blocks_gather(int n, int batch, int nb, int g, const double *blocks, double *grid,
                      void *stream);

/* Writes every guard cell from the block interiors, in place (interiors are read only).
 * g == 0: nothing to do. */
int mpp_blocks_fill_guards(int n, int batch, int nb, int g, double *blocks, void *stream);

/* y = A x block by block for the operator's problems (n and batch from op): each
 * interior cell reads its six neighbours from its own block, so x's guards must have
 * been filled; faces are the operator's grid-layout coefficients (no jump term).  y's
 * guards are set to 0.  g >= 1, P^3 <= 8192 (the padded block is staged in LDS, e.g. nb
 * 16 with g <= 2); x != y. */
int mpp_blocks_apply(mpp_op op, int nb, int g, const double *x_blocks, double *y_blocks,
                     void *stream);

/* ------------------------------------------------------------------------------
 * Two-level composite grid (Sec. 2 and Fig. 2: blocks at two resolutions, the finer
 * one where the interface is).  Level 0 is n0^3 cells (spacing 1/n0) in (n0/nb)^3
 * blocks of nb^3 cells, all stored; refined0[b] != 0 marks the level-0 blocks covered by
 * level 1 (spacing 1/(2 n0)).  Level 1 is stored sparsely: the 8 children of each
 * refined block, each nb^3 level-1 cells, in the order of their parents and, within a
 * parent, child a + 2b + 4c for its offsets a, b, c in x, y, z.  Blocks of both levels
 * are P^3 doubles with g guard layers as in the uniform block layout (P = nb + 2g, x
 * fastest): level 0 as [(n0/nb)^3][P^3], level 1 as [nblk1][P^3].
 * The leaf cells are those of the unrefined level-0 blocks and of every level-1 block.
 * The operator is the conservative finite-volume Laplacian on the leaves,
 *     (A x)_c = (1/V_c) sum_faces area * beta * (x_other - x_c) / distance,
 * with no flux through the walls; across a coarse-fine face the fine cell sees the
 * coarse cell itself (centres 1.5 fine spacings apart) and the coarse cell the four
 * fine cells across its face, so every flux leaves one leaf and enters another.  beta is
 * the ghost-fluid coefficient of the two cells' level-set values (lower coordinate
 * first; 1/rho on each side, the series value on a crossed face).
 * Requirements: 2 <= n0 <= 512, 2 <= nb, n0 % nb == 0, 1 <= g <= nb; device pointers
 * unless stated; asynchronous on `stream` unless stated; MPP_EINVAL on a violated
 * requirement, MPP_EDEVICE if a HIP call fails.  One problem per call.
 * ------------------------------------------------------------------------------ */
typedef struct mpp_amr_s *mpp_amr;

/* Device workspace the tables of a grid of n0^3 level-0 cells in blocks of nb^3 need
 * (0 if the shape is invalid). */
size_t mpp_amr_workspace_bytes(int n0, int nb);

/* Builds the block tables of the refinement refined0 (HOST, (n0/nb)^3 bytes, block
 * (bi, bj, bk) at bi + (n0/nb)(bj + (n0/nb) bk)) in `workspace` (device, owned by the
 * caller, kept alive until mpp_amr_destroy); synchronous.  *out receives the handle. */
int mpp_amr_create(int n0, int nb, int g, const uint8_t *refined0, void *workspace,
                   size_t workspace_bytes, void *stream, mpp_amr *out);
void mpp_amr_destroy(mpp_amr a);

/* Number of stored level-1 blocks and (list1: HOST, may be NULL, nblk1 entries) the
 * position of each, bi + (2 n0/nb)(bj + (2 n0/nb) bk) in level-1 block coordinates. */
int mpp_amr_level1_blocks(mpp_amr a, int32_t *nblk1, int32_t *list1);

/* Guard-cell fill of every stored block of both levels, in place (interiors are only
 * read).  A guard position outside the domain is mirrored about the wall on its own
 * level.  Inside, a level-0 guard takes the level-0 cell where that block is not refined
 * and the mean of the 8 level-1 cells it covers where it is; a level-1 guard takes the
 * level-1 cell where that block is stored and the level-0 cell containing it where it
 * is not (guards hold the volume average of the leaf field over the guard cell).
 * blocks1 may be NULL when nothing is refined. */
int mpp_amr_fill_guards(mpp_amr a, double *blocks0, double *blocks1, void *stream);

/* y = A x on the leaves.  phi (level set) and x in the block layout of both levels with
 * their guards filled (mpp_amr_fill_guards).  y is written on every stored block: A x in
 * the interiors of leaf blocks, 0 in guards and in refined level-0 blocks.  rho_neg and
 * rho_pos (> 0) are the densities where phi <= 0 and phi > 0.  y0 and y1 distinct from
 * each other and from the inputs; the level-1 pointers may be NULL when nothing is
 * refined. */
int mpp_amr_apply(mpp_amr a, const double *phi0, const double *phi1, const double *x0,
                  const double *x1, double rho_neg, double rho_pos, double *y0, double *y1,
                  void *stream);

/* Device workspace mpp_amr_solve needs for this grid (0 if a is NULL): five vectors in
 * the block layout of both levels plus per-block partial sums. */
size_t mpp_amr_solve_work_bytes(mpp_amr a);

/* Solves A x = b on the leaves by preconditioned conjugate gradients in the volume-
 * weighted inner product sum_leaves V_c u_c v_c (A is symmetric in it, -A positive
 * semi-definite with the constants as null space: the Neumann walls).  coarse == NULL:
 * the preconditioner is the inverse diagonal.  Otherwise a two-level multigrid cycle:
 * a damped Jacobi sweep (weight 0.8) on the leaves, the residual averaged over every
 * level-0 cell and corrected by one FP64 V-cycle of `coarse` (two sweeps per level), the
 * correction given to every leaf of the cell, one more Jacobi sweep.  `coarse` is an
 * operator of batch 1 on the n0^3 level-0 grid, built (mpp_build_operator) from the
 * level-0 level set in grid layout and the same densities, best with its faces next to
 * refined blocks taken from the fine level (mpp_amr_coarse_operator).
 * The weighted mean of b is removed first (the domain's volume is 1); x is returned with
 * zero weighted mean.  Stops when the weighted norm of the residual b' - A x is at most
 * rtol times that of b', polled every 8 iterations, or after max_iter iterations.
 * phi: level set with filled guards; b: interiors of the leaf blocks; x: in, the initial
 * guess on the leaves; out, the solution on the leaves with its guards filled (values of
 * refined level-0 blocks are left as they are).  work: device, >=
 * mpp_amr_solve_work_bytes(a), owned by the caller.  *iters: iterations done; *rel_resid:
 * the weighted relative residual of the returned x, recomputed from it (both HOST, may be
 * NULL).  Synchronous.  MPP_OK, MPP_ENOTCONVERGED (x holds the last iterate),
 * MPP_EBREAKDOWN, MPP_EINVAL (x aliasing b or phi, rtol <= 0, max_iter < 0, ...),
 * MPP_ENOMEM (work too small). */
int mpp_amr_solve(mpp_amr a, mpp_op coarse, const double *phi0, const double *phi1,
                  double rho_neg, double rho_pos, const double *b0, const double *b1, double *x0,
                  double *x1, double rtol, int32_t max_iter, void *work, size_t work_bytes,
                  int32_t *iters, double *rel_resid, void *stream);

/* Makes `op` (batch 1, built on the n0^3 level-0 grid from the level-0 level set phi0,
 * device grid layout) the level-0 operator of mpp_amr_solve's two-level cycle for this
 * grid: every level-0 face touching a refined block takes the mean of the four
 * fine-level coefficients across it (between two refined blocks the four pairs of
 * level-1 cells, across a coarse-fine face the four level-1 cells and the level-0 cell;
 * phi1: level-1 level set in the block layout), marked as crossed in the cell codes;
 * then the coarser levels and the coarsest inverse are rebuilt from the new faces.  The
 * operator's pressure-solve terms (curvature, jump) are left as they were. */
int mpp_amr_coarse_operator(mpp_amr a, mpp_op op, const double *phi0, const double *phi1,
                            double rho_neg, double rho_pos, void *stream);

/* ------------------------------------------------------------------------------
 * Learned initial guess.  Not part of the paper's method (whose solver starts from
 * the previous pressure or from zero): a small 3D U-Net maps the density field and
 * the right-hand side of a problem to an approximate solution that seeds the PCG.
 *
 * Network at resolution n (n % 16 == 0, 16 <= n <= 256), fields channels-last
 * ([batch][z][y][x][channel], x fastest among the cells):
 *   input 4 channels: log10(1/rho)/3, b/rms(b), 0, 0
 *   e1 = conv(4->16), conv(16->16)                  at n
 *   e2 = pool, conv(16->32), conv(32->32)           at n/2
 *   bt = pool, conv(32->64), conv(64->64)           at n/4
 *   d2 = up(bt) ++ e2, conv(96->32), conv(32->32)   at n/2
 *   d1 = up(d2) ++ e1, conv(48->16), conv(16->16)   at n
 *   y  = 1x1x1 conv(16->1) of d1                    at n
 * every 3x3x3 convolution with zero padding, bias and ReLU; pool is the mean of
 * 2x2x2 children, up repeats a value into its 8 children, ++ concatenates channels.
 * Parameters are FP32 ("master") in one flat vector, layer by layer, each
 * convolution as W[tap][c_out][c_in] with tap = 9(dz+1) + 3(dy+1) + (dx+1), then its
 * bias[c_out]; the head as w[16] then bias.  Products run on the matrix cores with
 * BF16 operands (weights and activations rounded to nearest even) and FP32
 * accumulation; activations are stored in BF16.
 * ------------------------------------------------------------------------------ */
typedef struct mpp_net_s *mpp_net;

/* Length of the flat parameter vector (354577). */
int32_t mpp_net_param_count(void);

/* Device workspace a network of resolution n, able to run batches of up to
 * batch_max samples forward and backward, needs (0 if the shape is invalid). */
size_t mpp_net_workspace_bytes(int32_t n, int32_t batch_max);

/* Creates a network in `workspace` (device, 256-byte aligned, owned by the caller and
 * kept alive until mpp_net_destroy) with parameters drawn from `seed` (He-normal
 * convolution weights, zero biases, a zero head) and zeroed optimiser state.  *out
 * receives the handle. */
int mpp_net_create(int32_t n, int32_t batch_max, uint64_t seed, void *workspace,
                   size_t workspace_bytes, void *stream, mpp_net *out);
void mpp_net_destroy(mpp_net net);

/* Host copies of the FP32 parameters (mpp_net_param_count() floats).  set also
 * resets the optimiser state.  Both synchronous. */
int mpp_net_set_params(mpp_net net, const float *params, void *stream);
int mpp_net_get_params(mpp_net net, float *params, void *stream);

/* y = net(x) for `batch` samples.  x: device BF16 bit patterns [batch][n^3][4];
 * y: device FP32 [batch][n^3].  Keeps the activations for mpp_net_backward. */
int mpp_net_forward(mpp_net net, const uint16_t *x, float *y, int32_t batch, void *stream);

/* Training loss of `batch` predictions y against targets t (device FP32
 * [batch][n^3], each target of zero mean): per sample the squared error of the
 * zero-mean prediction relative to the target's squared norm,
 *   L_s = sum (y - mean y - t)^2 / sum t^2,
 * and dy = d(mean_s L_s)/dy (device FP32 [batch][n^3]).  loss: device FP32
 * [batch] per-sample values. */
int mpp_net_loss(mpp_net net, const float *y, const float *t, float *dy, float *loss,
                 int32_t batch, void *stream);

/* Gradient of sum(dy * y) over the parameters, for the inputs of the last
 * mpp_net_forward (same batch), into the network's FP32 gradient vector (replaced,
 * not accumulated). */
int mpp_net_backward(mpp_net net, const float *dy, int32_t batch, void *stream);

/* Host copy of the gradient vector (mpp_net_param_count() floats); synchronous. */
int mpp_net_get_grads(mpp_net net, float *grads, void *stream);

/* One Adam step on the FP32 parameters with the current gradient: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), with
 * t the count of steps since creation or the last set_params. */
int mpp_net_adam(mpp_net net, float lr, float beta1, float beta2, float eps, void *stream);

/* Training on samples the solver generated (mpp_net_features of solved problems: the
 * density field and right-hand side as inputs, the solution as target).  Runs `steps`
 * training steps, each: draw `batch` of the `count` samples, forward pass, the loss of
 * mpp_net_loss, backward pass, one Adam step (as mpp_net_adam).  Step number g =
 * first_step + s (s = 0 .. steps-1; first_step lets a long run be split into calls) uses
 * the samples idx(q), q = g * batch + j, j = 0 .. batch-1: q mod count when seed == 0
 * (in order), otherwise output number q of the SplitMix64 stream started at seed, mod
 * count (a counter-based draw: any step's batch follows from seed and g alone).  Its
 * learning rate is lr0 * (lr1 / lr0)^(g / (total_steps - 1)), geometric from lr0 at step 0
 * to lr1 at step total_steps - 1 (lr0 throughout when total_steps <= 1).
 * x: device BF16 bits [count][n^3][4]; t: device FP32 [count][n^3] (zero-mean targets);
 * losses: device FP32 [steps][batch] per-sample losses before each step's update (may be
 * NULL).  Requires 1 <= batch <= the network's batch_max, count >= 1, steps >= 0,
 * first_step >= 0, lr0, lr1, eps > 0 and finite, 0 <= beta1, beta2 < 1; else MPP_EINVAL
 * before any device work.  Asynchronous. */
typedef struct {
    int32_t batch;        /* samples per step */
    int32_t steps;        /* steps in this call */
    int64_t first_step;   /* global number of the first step (schedule and draw) */
    int64_t total_steps;  /* length of the whole schedule */
    float lr0, lr1;       /* learning rate at step 0 and at step total_steps - 1 */
    float beta1, beta2, eps;  /* Adam constants, e.g. 0.9, 0.999, 1e-8 */
    int32_t reserved;
    uint64_t seed;        /* 0: samples in order; else the SplitMix64 seed of the draw */
} mpp_net_train_opts;

int mpp_net_train(mpp_net net, const uint16_t *x, const float *t, int64_t count,
                  const mpp_net_train_opts *opts, float *losses, void *stream);

/* Network inputs (and optionally targets) of the problems of an operator whose size
 * is r * n for an integer r >= 1 (op batch <= net batch_max).  b is the solver's
 * right-hand side (f + jterm, mean-projected); coarse values are means over r^3
 * blocks of cells: x[...,0] = log10(mean 1/rho)/3, x[...,1] = b_c / rms(b_c),
 * x[...,2..3] = 0.  f: device [batch][(r n)^3].  x: device BF16 bits
 * [batch][n^3][4].  p (device, may be NULL): solutions, whose block means scaled by
 * n^2 / rms(b_c) (p is of the order of h^2 b, h = 1/n) go to t (device FP32
 * [batch][n^3]).  rms: device FP32 [batch] (may be NULL). */
int mpp_net_features(mpp_net net, mpp_op op, const double *f, const double *p, uint16_t *x,
                     float *t, float *rms, void *stream);

/* Learned initial guess for mpp_solve with MPP_GUESS_GIVEN: features as in
 * mpp_net_features, the network, the prediction times rms(b_c) / n^2 prolonged to the
 * operator's grid by trilinear interpolation of the cell values (clamped at the
 * walls), its mean removed, scaled by (p.b) / (p.Ap) (the multiple of the prediction
 * closest to the solution in the energy norm, so never farther than zero), then
 * `sweeps` (0..8) red-black Gauss-Seidel sweeps on A p = b in FP32 (p then holds FP32
 * values).  The solver judges the guess against a zero start as the solve will see
 * them: judge MPP_JUDGE_PLAIN compares ||b - A p|| with ||b|| (for a solve without
 * deflation), MPP_JUDGE_DEFLATED compares ||P (b - A p)|| with ||P b|| (for a deflated
 * solve; P as in the deflation note above); the residual is taken in FP32 arithmetic.
 * A problem whose guess is not finite or does not start below the zero start gets p = 0
 * instead and fell_back[b] = 1 (host int32 [batch], may be NULL).  p: device FP64
 * [batch][(r n)^3].  The right-hand side assembled here can serve the next mpp_solve
 * on the same f (mpp_solve_opts.reuse_rhs). */
#define MPP_JUDGE_PLAIN 0
#define MPP_JUDGE_DEFLATED 1
int mpp_learned_guess(mpp_op op, mpp_net net, const double *f, double *p, int32_t sweeps,
                      int32_t judge, int32_t *fell_back, void *stream);

const char *mpp_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* MPP_H */
