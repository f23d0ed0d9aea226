/*
 * mpp_oracle.c -- plain, slow FP64 CPU oracle for the variable-density
 * pressure-projection solve
 *
 *        div( (1/rho) grad p ) = f         on [0,1]^3, homogeneous Neumann walls,
 *
 * with a sharp ghost-fluid treatment of the density jump at a level-set interface
 * and the surface-tension pressure jump [p] = sigma*kappa folded into the right-hand
 * side.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker of the GPU path and nothing
 * else: only the test-suite, the package's smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or helper with the GPU
 * library, and the GPU library never links, loads or calls it.
 *
 * What the paper fixes (Flash-X, arXiv 2312.11740):
 *   - Sec. 2 and the caption of Fig. 2: a staggered stencil with scalars (pressure,
 *     density, the level set) at cell centres and vector quantities on faces; the
 *     interface is the zero set of a signed distance phi, positive in air and
 *     negative in liquid.
 *   - Sec. 3 (IncompNS varDens, Multiphase, StencilsLevelSet, Grid_solvePoisson):
 *     a fractional-step projection whose pressure equation has the variable
 *     coefficient 1/rho set from the level set, solved by multigrid.
 *   - Sec. 4, Fig. 13 (TOML parameters): unit domain, gas/liquid density ratio 1e-3.
 * Everything else is a stated reading (not in the paper):
 *   - face coefficient on a face crossed by the interface: the series-resistance
 *     ghost-fluid coefficient of Liu, Fedkiw & Kang (J. Comput. Phys. 160, 2000);
 *   - jump [p] = p(phi>0) - p(phi<=0) = sigma*kappa with kappa = -div(grad phi/|grad phi|),
 *     as in the ghost-fluid multiphase method of Kang, Fedkiw & Liu (J. Sci. Comput. 15,
 *     2000); this gives Young-Laplace p_in - p_out = 2 sigma / R for a sphere under
 *     either orientation of phi;
 *   - a cell with phi == 0 belongs to the phi <= 0 side.
 * Around the solve (each section below states its reading):
 *   - the projection: f = div(u*)/dt on the staggered faces, u = u* - dt beta grad p
 *     with the jump-corrected gradient (Sec. 2);
 *   - the level set: first-order upwind advection by the face velocities and
 *     smoothed-sign Godunov re-distancing (Sec. 3, Multiphase / StencilsLevelSet);
 *   - heat diffusion: one backward-Euler step with the conductivity of each phase, the
 *     two in series on crossed faces (Sec. 2 transport equation, Sec. 3 HeatAD);
 *   - the block-structured layout: blocks with guard cells filled from their
 *     neighbours, mirrored at the walls (Sec. 2 blocks, Sec. 4 guard-cell fill);
 *   - two levels of refinement (Sec. 2, Fig. 2: blocks at two resolutions): the
 *     conservative finite-volume operator on the leaf cells, each coarse-fine flux
 *     taken once from the fine face and shared by both sides; guard cells as the
 *     volume average of the leaf field over the guard cell; the solve on it by CG with
 *     the inverse diagonal in the volume-weighted inner product.
 *
 * Conventions (shared with the GPU library only through this description):
 *   n^3 cells, h = 1/n, cell (i,j,k) centre ((i+1/2)h, (j+1/2)h, (k+1/2)h),
 *   linear index i + n*(j + n*k) (x fastest).  Face arrays hold the LOW face of each
 *   cell: bx[i,j,k] is the coefficient between (i-1,j,k) and (i,j,k); bx[0,j,k] = 0
 *   (wall).  High wall faces are implicit zeros.
 *   (A x)_c = sum over the six faces of beta_f (x_nb - x_c) / h^2.
 *
 * Every routine here is a direct statement of its definition: no blocking, fusion or
 * reordering beyond an OpenMP split over independent cells.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOTCONVERGED (-4)
#define ORC_EBREAKDOWN (-5)

static size_t ix(int n, int i, int j, int k)
{
    return (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k);
}

/* ------------------------------------------------------------------------ */
/* Level set, sides and the ghost-fluid face coefficient                     */
/* ------------------------------------------------------------------------ */

/* side "+" (gas in the paper's orientation) iff phi > 0; phi == 0 goes to "-". */
static int is_plus(double phi) { return phi > 0.0; }

/* Fraction of the segment from cell a to cell b that lies on a's side of the
 * interface, from linear interpolation of phi between the two centres. */
static double crossing_theta(double phi_a, double phi_b)
{
    return fabs(phi_a) / (fabs(phi_a) + fabs(phi_b));
}

/* Coefficient 1/rho of the face between centres a and b.  Same side: the phase
 * value.  Crossing: resistances rho*length in series over the two pieces of the
 * segment (Liu-Fedkiw-Kang), 1 / (theta*rho_a + (1-theta)*rho_b). */
static double face_beta(double phi_a, double phi_b, double rho_neg, double rho_pos)
{
    double rho_a = is_plus(phi_a) ? rho_pos : rho_neg;
    double rho_b = is_plus(phi_b) ? rho_pos : rho_neg;
    if (is_plus(phi_a) == is_plus(phi_b))
        return 1.0 / rho_a;
    double theta = crossing_theta(phi_a, phi_b);
    return 1.0 / (theta * rho_a + (1.0 - theta) * rho_b);
}

int orc_faces(int n, const double *phi, double rho_neg, double rho_pos, double *bx,
              double *by, double *bz)
{
    if (n < 1 || !phi || !bx || !by || !bz)
        return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t c = ix(n, i, j, k);
                bx[c] = (i == 0) ? 0.0 : face_beta(phi[ix(n, i - 1, j, k)], phi[c], rho_neg, rho_pos);
                by[c] = (j == 0) ? 0.0 : face_beta(phi[ix(n, i, j - 1, k)], phi[c], rho_neg, rho_pos);
                bz[c] = (k == 0) ? 0.0 : face_beta(phi[ix(n, i, j, k - 1)], phi[c], rho_neg, rho_pos);
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Curvature kappa = -div(grad phi / |grad phi|)                             */
/* ------------------------------------------------------------------------ */

/* phi with linear extrapolation beyond the walls: phi(-1) = 2 phi(0) - phi(1),
 * phi(n) = 2 phi(n-1) - phi(n-2), applied axis by axis. */
static double phi_ext(int n, const double *phi, int i, int j, int k)
{
    if (i < 0)
        return 2.0 * phi_ext(n, phi, 0, j, k) - phi_ext(n, phi, 1, j, k);
    if (i > n - 1)
        return 2.0 * phi_ext(n, phi, n - 1, j, k) - phi_ext(n, phi, n - 2, j, k);
    if (j < 0)
        return 2.0 * phi_ext(n, phi, i, 0, k) - phi_ext(n, phi, i, 1, k);
    if (j > n - 1)
        return 2.0 * phi_ext(n, phi, i, n - 1, k) - phi_ext(n, phi, i, n - 2, k);
    if (k < 0)
        return 2.0 * phi_ext(n, phi, i, j, 0) - phi_ext(n, phi, i, j, 1);
    if (k > n - 1)
        return 2.0 * phi_ext(n, phi, i, j, n - 1) - phi_ext(n, phi, i, j, n - 2);
    return phi[ix(n, i, j, k)];
}

/* Mean curvature of the level sets of phi at the centre of cell (i,j,k):
 * second-order central differences for the gradient and the Hessian, then
 *   kappa = -[ (pyy+pzz) px^2 + (pxx+pzz) py^2 + (pxx+pyy) pz^2
 *              - 2 px py pxy - 2 px pz pxz - 2 py pz pyz ] / |grad phi|^3,
 * and 0 where |grad phi| < 1e-12. */
static double curvature_at(int n, const double *phi, int i, int j, int k)
{
    double h = 1.0 / n;
#define P(a, b, c) phi_ext(n, phi, i + (a), j + (b), k + (c))
    double p0 = P(0, 0, 0);
    double px = (P(1, 0, 0) - P(-1, 0, 0)) / (2.0 * h);
    double py = (P(0, 1, 0) - P(0, -1, 0)) / (2.0 * h);
    double pz = (P(0, 0, 1) - P(0, 0, -1)) / (2.0 * h);
    double pxx = (P(1, 0, 0) - 2.0 * p0 + P(-1, 0, 0)) / (h * h);
    double pyy = (P(0, 1, 0) - 2.0 * p0 + P(0, -1, 0)) / (h * h);
    double pzz = (P(0, 0, 1) - 2.0 * p0 + P(0, 0, -1)) / (h * h);
    double pxy = (P(1, 1, 0) - P(1, -1, 0) - P(-1, 1, 0) + P(-1, -1, 0)) / (4.0 * h * h);
    double pxz = (P(1, 0, 1) - P(1, 0, -1) - P(-1, 0, 1) + P(-1, 0, -1)) / (4.0 * h * h);
    double pyz = (P(0, 1, 1) - P(0, 1, -1) - P(0, -1, 1) + P(0, -1, -1)) / (4.0 * h * h);
#undef P
    double g2 = px * px + py * py + pz * pz;
    double g = sqrt(g2);
    if (g < 1e-12)
        return 0.0;
    double num = (pyy + pzz) * px * px + (pxx + pzz) * py * py + (pxx + pyy) * pz * pz
               - 2.0 * px * py * pxy - 2.0 * px * pz * pxz - 2.0 * py * pz * pyz;
    return -num / (g2 * g);
}

/* A cell is interface-adjacent when one of its in-domain neighbours is on the
 * other side. */
static int interface_adjacent(int n, const double *phi, int i, int j, int k)
{
    int s = is_plus(phi[ix(n, i, j, k)]);
    if (i > 0 && is_plus(phi[ix(n, i - 1, j, k)]) != s) return 1;
    if (i < n - 1 && is_plus(phi[ix(n, i + 1, j, k)]) != s) return 1;
    if (j > 0 && is_plus(phi[ix(n, i, j - 1, k)]) != s) return 1;
    if (j < n - 1 && is_plus(phi[ix(n, i, j + 1, k)]) != s) return 1;
    if (k > 0 && is_plus(phi[ix(n, i, j, k - 1)]) != s) return 1;
    if (k < n - 1 && is_plus(phi[ix(n, i, j, k + 1)]) != s) return 1;
    return 0;
}

/* kappa at every interface-adjacent cell, 0 elsewhere. */
int orc_curvature(int n, const double *phi, double *kappa)
{
    if (n < 2 || !phi || !kappa)
        return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                kappa[ix(n, i, j, k)] =
                    interface_adjacent(n, phi, i, j, k) ? curvature_at(n, phi, i, j, k) : 0.0;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Jump term of the right-hand side                                          */
/* ------------------------------------------------------------------------ */

/* For every face crossed by the interface, between a (low) and b (high):
 *   theta  = |phi_a| / (|phi_a| + |phi_b|)     (interface position measured from a)
 *   J      = sigma * ((1-theta) kappa_a + theta kappa_b)   (kappa interpolated to it)
 *   beta^  = the ghost-fluid face coefficient,
 * and the face adds s * beta^ * J / h^2 to each of its two cells, s = +1 for the
 * cell on the "-" side and -1 for the cell on the "+" side.  This moves the jump of
 * [p] = p+ - p- = J out of the stencil: A p = f + jterm.
 * kappa: per-cell curvature (orc_curvature's output, or any override field). */
int orc_jump(int n, const double *phi, const double *kappa, double rho_neg, double rho_pos,
             double sigma, double *jterm)
{
    if (n < 1 || !phi || !kappa || !jterm)
        return ORC_EINVAL;
    double inv_h2 = (double)n * (double)n;
    memset(jterm, 0, sizeof(double) * (size_t)n * n * n);
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int ia = i - (d == 0), ja = j - (d == 1), ka = k - (d == 2);
                    if (ia < 0 || ja < 0 || ka < 0)
                        continue;
                    size_t a = ix(n, ia, ja, ka), b = ix(n, i, j, k);
                    if (is_plus(phi[a]) == is_plus(phi[b]))
                        continue;
                    double theta = crossing_theta(phi[a], phi[b]);
                    double J = sigma * ((1.0 - theta) * kappa[a] + theta * kappa[b]);
                    double bh = face_beta(phi[a], phi[b], rho_neg, rho_pos);
                    double s_a = is_plus(phi[a]) ? -1.0 : 1.0;
                    jterm[a] += s_a * bh * J * inv_h2;
                    jterm[b] -= s_a * bh * J * inv_h2;
                }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side b = f + jterm, projected to zero mean                     */
/* ------------------------------------------------------------------------ */

/* Neumaier-compensated sum. */
static double csum(const double *v, size_t m)
{
    double s = 0.0, c = 0.0;
    for (size_t q = 0; q < m; ++q) {
        double t = s + v[q];
        if (fabs(s) >= fabs(v[q]))
            c += (s - t) + v[q];
        else
            c += (v[q] - t) + s;
        s = t;
    }
    return s + c;
}

/* b = f + jterm (jterm may be NULL), then b -= mean(b).  Returns the removed mean
 * through *mean_out (the compatibility defect of the Neumann problem). */
int orc_rhs(int n, const double *f, const double *jterm, double *b, double *mean_out)
{
    if (n < 1 || !f || !b)
        return ORC_EINVAL;
    size_t m = (size_t)n * n * n;
    for (size_t q = 0; q < m; ++q)
        b[q] = f[q] + (jterm ? jterm[q] : 0.0);
    double mean = csum(b, m) / (double)m;
    for (size_t q = 0; q < m; ++q)
        b[q] -= mean;
    if (mean_out)
        *mean_out = mean;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The operator                                                              */
/* ------------------------------------------------------------------------ */

/* y = A x,  (A x)_c = sum_faces beta_f (x_nb - x_c) / h^2, no flux through walls. */
void orc_apply(int n, const double *bx, const double *by, const double *bz,
               const double *x, double *y)
{
    double inv_h2 = (double)n * (double)n;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t c = ix(n, i, j, k);
                double s = 0.0;
                if (i > 0) s += bx[c] * (x[ix(n, i - 1, j, k)] - x[c]);
                if (i < n - 1) s += bx[ix(n, i + 1, j, k)] * (x[ix(n, i + 1, j, k)] - x[c]);
                if (j > 0) s += by[c] * (x[ix(n, i, j - 1, k)] - x[c]);
                if (j < n - 1) s += by[ix(n, i, j + 1, k)] * (x[ix(n, i, j + 1, k)] - x[c]);
                if (k > 0) s += bz[c] * (x[ix(n, i, j, k - 1)] - x[c]);
                if (k < n - 1) s += bz[ix(n, i, j, k + 1)] * (x[ix(n, i, j, k + 1)] - x[c]);
                y[c] = s * inv_h2;
            }
}

static double dot(const double *a, const double *b, size_t m)
{
    long double s = 0.0L;
    for (size_t q = 0; q < m; ++q)
        s += (long double)a[q] * (long double)b[q];
    return (double)s;
}

static double nrm2(const double *a, size_t m) { return sqrt(dot(a, a, m)); }

static void remove_mean(double *v, size_t m)
{
    double mean = csum(v, m) / (double)m;
    for (size_t q = 0; q < m; ++q)
        v[q] -= mean;
}

/* ||b - A x||_2 / ||b||_2 (0 if b == 0). */
double orc_rel_residual(int n, const double *bx, const double *by, const double *bz,
                        const double *b, const double *x)
{
    size_t m = (size_t)n * n * n;
    double *r = (double *)malloc(sizeof(double) * m);
    if (!r)
        return NAN;
    orc_apply(n, bx, by, bz, x, r);
    for (size_t q = 0; q < m; ++q)
        r[q] = b[q] - r[q];
    double bn = nrm2(b, m);
    double rn = nrm2(r, m);
    free(r);
    return bn > 0.0 ? rn / bn : rn;
}

/* ------------------------------------------------------------------------ */
/* Direct solve on small grids: Cholesky of (-A + 11^T/m)                    */
/* ------------------------------------------------------------------------ */

/* Dense (-A + J/m) in row-major order, J the all-ones matrix; SPD because the
 * constants (A's null space) get eigenvalue 1 and everything else is -A's. */
static void dense_regularised(int n, const double *bx, const double *by, const double *bz,
                              double *M)
{
    size_t m = (size_t)n * n * n;
    double *e = (double *)calloc(m, sizeof(double));
    double *col = (double *)malloc(sizeof(double) * m);
    for (size_t c = 0; c < m; ++c) {
        e[c] = 1.0;
        orc_apply(n, bx, by, bz, e, col);
        e[c] = 0.0;
        for (size_t r = 0; r < m; ++r)
            M[r * m + c] = -col[r] + 1.0 / (double)m;
    }
    free(e);
    free(col);
}

/* In-place Cholesky M = L L^T (lower triangle).  Returns 0 or the failing pivot+1. */
static size_t cholesky(double *M, size_t m)
{
    for (size_t j = 0; j < m; ++j) {
        double d = M[j * m + j];
        for (size_t q = 0; q < j; ++q)
            d -= M[j * m + q] * M[j * m + q];
        if (!(d > 0.0))
            return j + 1;
        double l = sqrt(d);
        M[j * m + j] = l;
        for (size_t r = j + 1; r < m; ++r) {
            double s = M[r * m + j];
            for (size_t q = 0; q < j; ++q)
                s -= M[r * m + q] * M[j * m + q];
            M[r * m + j] = s / l;
        }
    }
    return 0;
}

static void cholesky_solve(const double *L, size_t m, double *v)
{
    for (size_t r = 0; r < m; ++r) {
        double s = v[r];
        for (size_t q = 0; q < r; ++q)
            s -= L[r * m + q] * v[q];
        v[r] = s / L[r * m + r];
    }
    for (size_t r = m; r-- > 0;) {
        double s = v[r];
        for (size_t q = r + 1; q < m; ++q)
            s -= L[q * m + r] * v[q];
        v[r] = s / L[r * m + r];
    }
}

/* Unique zero-mean p with A p = b, for zero-mean b; n^3 <= 4096. */
int orc_solve_dense(int n, const double *bx, const double *by, const double *bz,
                    const double *b, double *p)
{
    if (n < 1 || n > 16)
        return ORC_EINVAL;
    size_t m = (size_t)n * n * n;
    double *M = (double *)malloc(sizeof(double) * m * m);
    if (!M)
        return ORC_ENOMEM;
    dense_regularised(n, bx, by, bz, M);
    if (cholesky(M, m)) {
        free(M);
        return ORC_EBREAKDOWN;
    }
    for (size_t q = 0; q < m; ++q)
        p[q] = -b[q];
    cholesky_solve(M, m, p);
    free(M);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Geometric multigrid V-cycle (the preconditioner's reference definition)   */
/* ------------------------------------------------------------------------ */
/*
 * Levels: n_0 = n; while n_l is even and n_l > 4, n_{l+1} = n_l / 2.  Level l has
 * h_l = 1/n_l and face coefficients averaged from level l-1: a coarse face is the
 * union of 2x2 fine faces on the same plane, and its coefficient is their mean.
 * Restriction: mean of the 8 children.  Prolongation: each child gets its parent's
 * value (piecewise constant).  Smoother: red-black Gauss-Seidel, red = (i+j+k) even,
 *   x_c <- (sum_f beta_f x_nb - h^2 b_c) / sum_f beta_f.
 * V(l, b): x = 0; nu times (red, black); r = b - A x; x += P V(l+1, R r);
 *          nu times (black, red); return x.
 * Coarsest level: x = (-A + 11^T/m)^{-1} (-b).
 */

typedef struct {
    int n;
    double *bx, *by, *bz;
} orc_level;

typedef struct {
    int nlev, nu;
    orc_level lev[16];
    double *Lc; /* Cholesky factor of the coarsest regularised operator */
    double *work[16][3];
} orc_mg;

static int level_count(int n)
{
    int L = 1;
    while (n % 2 == 0 && n > 4 && L < 16) {
        n /= 2;
        ++L;
    }
    return L;
}

/* Coarse face coefficients from fine ones (mean of the 4 fine faces on the plane). */
void orc_coarsen_faces(int nf, const double *fx, const double *fy, const double *fz,
                       double *cx, double *cy, double *cz)
{
    int nc = nf / 2;
    for (int K = 0; K < nc; ++K)
        for (int J = 0; J < nc; ++J)
            for (int I = 0; I < nc; ++I) {
                size_t C = ix(nc, I, J, K);
                double sx = 0.0, sy = 0.0, sz = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        sx += fx[ix(nf, 2 * I, 2 * J + a, 2 * K + b)];
                        sy += fy[ix(nf, 2 * I + a, 2 * J, 2 * K + b)];
                        sz += fz[ix(nf, 2 * I + a, 2 * J + b, 2 * K)];
                    }
                cx[C] = 0.25 * sx;
                cy[C] = 0.25 * sy;
                cz[C] = 0.25 * sz;
            }
}

/* Update all cells of one colour (colour = (i+j+k) mod 2) in place. */
void orc_gs_colour(int n, const double *bx, const double *by, const double *bz,
                   const double *b, double *x, int colour)
{
    double h2 = 1.0 / ((double)n * (double)n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                if (((i + j + k) & 1) != colour)
                    continue;
                size_t c = ix(n, i, j, k);
                double num = 0.0, den = 0.0;
                if (i > 0) { num += bx[c] * x[ix(n, i - 1, j, k)]; den += bx[c]; }
                if (i < n - 1) { double w = bx[ix(n, i + 1, j, k)]; num += w * x[ix(n, i + 1, j, k)]; den += w; }
                if (j > 0) { num += by[c] * x[ix(n, i, j - 1, k)]; den += by[c]; }
                if (j < n - 1) { double w = by[ix(n, i, j + 1, k)]; num += w * x[ix(n, i, j + 1, k)]; den += w; }
                if (k > 0) { num += bz[c] * x[ix(n, i, j, k - 1)]; den += bz[c]; }
                if (k < n - 1) { double w = bz[ix(n, i, j, k + 1)]; num += w * x[ix(n, i, j, k + 1)]; den += w; }
                x[c] = (num - h2 * b[c]) / den;
            }
}

void orc_restrict(int nf, const double *rf, double *bc)
{
    int nc = nf / 2;
    for (int K = 0; K < nc; ++K)
        for (int J = 0; J < nc; ++J)
            for (int I = 0; I < nc; ++I) {
                double s = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a)
                            s += rf[ix(nf, 2 * I + a, 2 * J + b, 2 * K + c)];
                bc[ix(nc, I, J, K)] = 0.125 * s;
            }
}

void orc_prolong_add(int nf, const double *ec, double *xf)
{
    int nc = nf / 2;
    for (int k = 0; k < nf; ++k)
        for (int j = 0; j < nf; ++j)
            for (int i = 0; i < nf; ++i)
                xf[ix(nf, i, j, k)] += ec[ix(nc, i / 2, j / 2, k / 2)];
}

void orc_mg_destroy(orc_mg *mg)
{
    if (!mg)
        return;
    for (int l = 1; l < mg->nlev; ++l) {
        free(mg->lev[l].bx);
        free(mg->lev[l].by);
        free(mg->lev[l].bz);
    }
    for (int l = 0; l < mg->nlev; ++l)
        for (int q = 0; q < 3; ++q)
            free(mg->work[l][q]);
    free(mg->Lc);
    free(mg);
}

/* Builds the hierarchy.  Level 0 borrows the caller's face arrays. */
orc_mg *orc_mg_create(int n, const double *bx, const double *by, const double *bz, int nu)
{
    if (n < 2 || nu < 1)
        return NULL;
    orc_mg *mg = (orc_mg *)calloc(1, sizeof(orc_mg));
    mg->nlev = level_count(n);
    mg->nu = nu;
    mg->lev[0].n = n;
    mg->lev[0].bx = (double *)bx;
    mg->lev[0].by = (double *)by;
    mg->lev[0].bz = (double *)bz;
    for (int l = 1; l < mg->nlev; ++l) {
        int nc = mg->lev[l - 1].n / 2;
        size_t mc = (size_t)nc * nc * nc;
        mg->lev[l].n = nc;
        mg->lev[l].bx = (double *)malloc(sizeof(double) * mc);
        mg->lev[l].by = (double *)malloc(sizeof(double) * mc);
        mg->lev[l].bz = (double *)malloc(sizeof(double) * mc);
        orc_coarsen_faces(mg->lev[l - 1].n, mg->lev[l - 1].bx, mg->lev[l - 1].by,
                          mg->lev[l - 1].bz, mg->lev[l].bx, mg->lev[l].by, mg->lev[l].bz);
    }
    for (int l = 0; l < mg->nlev; ++l) {
        size_t m = (size_t)mg->lev[l].n * mg->lev[l].n * mg->lev[l].n;
        for (int q = 0; q < 3; ++q)
            mg->work[l][q] = (double *)calloc(m, sizeof(double));
    }
    orc_level *c = &mg->lev[mg->nlev - 1];
    size_t mc = (size_t)c->n * c->n * c->n;
    if (mc > 4096) {
        orc_mg_destroy(mg);
        return NULL;
    }
    mg->Lc = (double *)malloc(sizeof(double) * mc * mc);
    dense_regularised(c->n, c->bx, c->by, c->bz, mg->Lc);
    if (cholesky(mg->Lc, mc)) {
        orc_mg_destroy(mg);
        return NULL;
    }
    return mg;
}

int orc_mg_levels(const orc_mg *mg) { return mg->nlev; }

/* x = V(l, b) (x is overwritten). */
static void vcycle(orc_mg *mg, int l, const double *b, double *x)
{
    orc_level *L = &mg->lev[l];
    size_t m = (size_t)L->n * L->n * L->n;
    if (l == mg->nlev - 1) {
        for (size_t q = 0; q < m; ++q)
            x[q] = -b[q];
        cholesky_solve(mg->Lc, m, x);
        return;
    }
    double *r = mg->work[l][0];
    double *bc = mg->work[l + 1][1];
    double *xc = mg->work[l + 1][2];
    memset(x, 0, sizeof(double) * m);
    for (int s = 0; s < mg->nu; ++s) {
        orc_gs_colour(L->n, L->bx, L->by, L->bz, b, x, 0);
        orc_gs_colour(L->n, L->bx, L->by, L->bz, b, x, 1);
    }
    orc_apply(L->n, L->bx, L->by, L->bz, x, r);
    for (size_t q = 0; q < m; ++q)
        r[q] = b[q] - r[q];
    orc_restrict(L->n, r, bc);
    vcycle(mg, l + 1, bc, xc);
    orc_prolong_add(L->n, xc, x);
    for (int s = 0; s < mg->nu; ++s) {
        orc_gs_colour(L->n, L->bx, L->by, L->bz, b, x, 1);
        orc_gs_colour(L->n, L->bx, L->by, L->bz, b, x, 0);
    }
}

/* z = V(0, r): one V-cycle applied to a level-0 residual. */
void orc_mg_vcycle(orc_mg *mg, const double *r, double *z) { vcycle(mg, 0, r, z); }

/* ------------------------------------------------------------------------ */
/* Preconditioned conjugate gradients on -A                                   */
/* ------------------------------------------------------------------------ */
/*
 * CG for the SPD (on zero-mean vectors) system (-A) x = -b; written with r = b - A x
 * and q = A p the signs cancel: alpha = (r.z)/(p.q), r -= alpha q.  z is projected
 * to zero mean.  Stops when ||r||_2 <= tol ||b||_2 for the recurrence residual, then
 * recomputes the true residual and continues from it if that one is not below tol.
 * x holds the initial guess on entry and the zero-mean solution on exit.
 */
typedef void (*precond_fn)(void *ctx, const double *r, double *z);

typedef struct {
    size_t m;
    const double *diag;
} jac_ctx;

static void jac_apply(void *ctx, const double *r, double *z)
{
    jac_ctx *J = (jac_ctx *)ctx;
    for (size_t q = 0; q < J->m; ++q)
        z[q] = r[q] / J->diag[q];
}

static void mg_apply(void *ctx, const double *r, double *z) { orc_mg_vcycle((orc_mg *)ctx, r, z); }

static int pcg(int n, const double *bx, const double *by, const double *bz, const double *b,
               double *x, double tol, int max_iter, precond_fn M, void *ctx, int *iters_out,
               double *relres_out)
{
    size_t m = (size_t)n * n * n;
    double *r = (double *)malloc(sizeof(double) * m);
    double *z = (double *)malloc(sizeof(double) * m);
    double *p = (double *)malloc(sizeof(double) * m);
    double *q = (double *)malloc(sizeof(double) * m);
    if (!r || !z || !p || !q) {
        free(r); free(z); free(p); free(q);
        return ORC_ENOMEM;
    }
    double bn = nrm2(b, m);
    int it = 0, status = ORC_ENOTCONVERGED;
    double rel = 0.0, best = INFINITY;
    int stall = 0;
    if (bn == 0.0) {
        memset(x, 0, sizeof(double) * m);
        status = ORC_OK;
        goto done;
    }
    for (;;) { /* restart loop: true residual */
        orc_apply(n, bx, by, bz, x, r);
        for (size_t c = 0; c < m; ++c)
            r[c] = b[c] - r[c];
        rel = nrm2(r, m) / bn;
        if (rel <= tol) {
            status = ORC_OK;
            break;
        }
        if (it >= max_iter)
            break;
        if (rel < 0.5 * best) {
            best = rel;
            stall = 0;
        } else if (++stall >= 3) { /* FP64 stagnation: report the level reached */
            status = ORC_ENOTCONVERGED;
            break;
        }
        M(ctx, r, z);
        remove_mean(z, m);
        memcpy(p, z, sizeof(double) * m);
        double rz = dot(r, z, m);
        while (it < max_iter) {
            orc_apply(n, bx, by, bz, p, q);
            double pq = dot(p, q, m);
            if (!(pq < 0.0) || !(rz < 0.0)) { /* -A and M must stay positive */
                status = ORC_EBREAKDOWN;
                goto done;
            }
            double alpha = rz / pq;
            for (size_t c = 0; c < m; ++c) {
                x[c] += alpha * p[c];
                r[c] -= alpha * q[c];
            }
            ++it;
            if (nrm2(r, m) <= tol * bn)
                break;
            M(ctx, r, z);
            remove_mean(z, m);
            double rz_new = dot(r, z, m);
            double beta = rz_new / rz;
            rz = rz_new;
            for (size_t c = 0; c < m; ++c)
                p[c] = z[c] + beta * p[c];
        }
    }
done:
    remove_mean(x, m);
    if (status != ORC_EBREAKDOWN)
        rel = orc_rel_residual(n, bx, by, bz, b, x);
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = rel;
    free(r); free(z); free(p); free(q);
    return status;
}

int orc_solve_jacobi_pcg(int n, const double *bx, const double *by, const double *bz,
                         const double *b, double *x, double tol, int max_iter, int *iters,
                         double *relres)
{
    size_t m = (size_t)n * n * n;
    double *diag = (double *)malloc(sizeof(double) * m);
    double inv_h2 = (double)n * (double)n;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t c = ix(n, i, j, k);
                double s = 0.0;
                if (i > 0) s += bx[c];
                if (i < n - 1) s += bx[ix(n, i + 1, j, k)];
                if (j > 0) s += by[c];
                if (j < n - 1) s += by[ix(n, i, j + 1, k)];
                if (k > 0) s += bz[c];
                if (k < n - 1) s += bz[ix(n, i, j, k + 1)];
                diag[c] = -s * inv_h2;
            }
    jac_ctx J = {m, diag};
    int st = pcg(n, bx, by, bz, b, x, tol, max_iter, jac_apply, &J, iters, relres);
    free(diag);
    return st;
}

int orc_solve_mg_pcg(int n, const double *bx, const double *by, const double *bz,
                     const double *b, double *x, double tol, int max_iter, int nu, int *iters,
                     double *relres)
{
    orc_mg *mg = orc_mg_create(n, bx, by, bz, nu);
    if (!mg)
        return ORC_EINVAL;
    int st = pcg(n, bx, by, bz, b, x, tol, max_iter, mg_apply, mg, iters, relres);
    orc_mg_destroy(mg);
    return st;
}

/* ------------------------------------------------------------------------ */
/* The projection around the solve (Sec. 2, fractional step on the staggered  */
/* grid): f = div(u*)/dt on the cell centres, then u = u* - dt beta grad p on  */
/* the faces, with the same jump-corrected gradient the right-hand side uses   */
/* ------------------------------------------------------------------------ */

/* Face velocities use the low-face layout of the coefficients: ux[i,j,k] is the
 * x-velocity on the face between (i-1,j,k) and (i,j,k); ux[0,j,k] is the wall (and
 * is read as 0, whatever it holds); high wall faces are implicit zeros.
 * f[c] = (sum over the three axes of (u on the high face - u on the low face) / h) / dt. */
int orc_divergence(int n, const double *ux, const double *uy, const double *uz, double dt,
                   double *f)
{
    if (n < 1 || !ux || !uy || !uz || !f || !(dt > 0.0))
        return ORC_EINVAL;
    double inv_h = (double)n;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t c = ix(n, i, j, k);
                double xl = i > 0 ? ux[c] : 0.0, xh = i < n - 1 ? ux[ix(n, i + 1, j, k)] : 0.0;
                double yl = j > 0 ? uy[c] : 0.0, yh = j < n - 1 ? uy[ix(n, i, j + 1, k)] : 0.0;
                double zl = k > 0 ? uz[c] : 0.0, zh = k < n - 1 ? uz[ix(n, i, j, k + 1)] : 0.0;
                f[c] = (((xh - xl) + (yh - yl)) + (zh - zl)) * inv_h / dt;
            }
    return ORC_OK;
}

/* u_f -= dt * beta^_f * (p_b - p_a - d_f J_f) / h on every interior face between a
 * (low) and b (high): J_f = sigma ((1-theta) kappa_a + theta kappa_b) and d_f = +1
 * when a is on the "-" side and b on the "+" side, -1 for the opposite crossing, 0
 * on same-side faces.  That is the gradient of p with b's value carried across the
 * interface to a's side (p+ - p- = J), the same flux whose jump part the jump term
 * moves to the right-hand side, so div(u) = div(u*) - dt (A p - jterm).  Wall faces
 * are set to 0. */
int orc_project(int n, const double *phi, const double *kappa, const double *p, double rho_neg,
                double rho_pos, double sigma, double dt, double *ux, double *uy, double *uz)
{
    if (n < 1 || !phi || !kappa || !p || !ux || !uy || !uz || !(dt > 0.0))
        return ORC_EINVAL;
    double inv_h = (double)n;
    double *u[3] = {ux, uy, uz};
    for (int d = 0; d < 3; ++d)
#pragma omp parallel for schedule(static)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    size_t b = ix(n, i, j, k);
                    int ia = i - (d == 0), ja = j - (d == 1), ka = k - (d == 2);
                    if (ia < 0 || ja < 0 || ka < 0) {
                        u[d][b] = 0.0;
                        continue;
                    }
                    size_t a = ix(n, ia, ja, ka);
                    double beta = face_beta(phi[a], phi[b], rho_neg, rho_pos);
                    double jump = 0.0;
                    if (is_plus(phi[a]) != is_plus(phi[b])) {
                        double theta = crossing_theta(phi[a], phi[b]);
                        double J = sigma * ((1.0 - theta) * kappa[a] + theta * kappa[b]);
                        jump = is_plus(phi[a]) ? -J : J;
                    }
                    u[d][b] -= dt * beta * ((p[b] - p[a]) - jump) * inv_h;
                }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Level set: advection by the face velocities and re-distancing             */
/* ------------------------------------------------------------------------ */
/* The level-set unit (Sec. 3, Multiphase / StencilsLevelSet) moves phi with the flow
 * and keeps it a signed distance; the paper names the operations but gives no scheme.
 * Readings (stated, not the paper's):
 *   - advection: phi_t + u . grad phi = 0, one forward-Euler step, first-order upwind
 *     differences, the cell-centre velocity the mean of the cell's two faces along each
 *     axis (wall faces 0), one-sided differences across a wall taken as 0 (phi
 *     extended by its boundary value);
 *   - re-distancing: pseudo-time steps of phi_tau + S(phi0) (|grad phi| - 1) = 0 with
 *     S(phi0) = phi0 / sqrt(phi0^2 + h^2) (Sussman, Smereka & Osher, J. Comput. Phys.
 *     114, 1994) and the first-order Godunov upwind |grad phi| (Rouy & Tourin), forward
 *     Euler, the same wall rule. */

/* out = phi - dt * (ax + ay + az), a_d = u_d * (backward difference if u_d > 0, else
 * forward difference) along axis d, u_d the cell-centre velocity. */
int orc_ls_advect(int n, const double *phi, const double *ux, const double *uy,
                  const double *uz, double dt, double *out)
{
    if (n < 2 || !phi || !ux || !uy || !uz || !out || !(dt > 0.0))
        return ORC_EINVAL;
    double inv_h = (double)n;
    const double *u[3] = {ux, uy, uz};
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int ijk3[3] = {i, j, k};
                size_t c = ix(n, i, j, k);
                double a[3];
                for (int d = 0; d < 3; ++d) {
                    int q = ijk3[d];
                    size_t step = d == 0 ? 1 : (d == 1 ? (size_t)n : (size_t)n * n);
                    double ulo = q > 0 ? u[d][c] : 0.0;
                    double uhi = q < n - 1 ? u[d][c + step] : 0.0;
                    double uc = 0.5 * (ulo + uhi);
                    double back = q > 0 ? (phi[c] - phi[c - step]) * inv_h : 0.0;
                    double fwd = q < n - 1 ? (phi[c + step] - phi[c]) * inv_h : 0.0;
                    a[d] = uc > 0.0 ? uc * back : uc * fwd;
                }
                out[c] = phi[c] - dt * ((a[0] + a[1]) + a[2]);
            }
    return ORC_OK;
}

/* Godunov |grad phi| at cell c for the sign s of phi0 (s > 0: max over the axes of
 * max(back+^2, fwd-^2); s < 0: max(back-^2, fwd+^2)), summed over the axes. */
static double godunov_grad(int n, const double *phi, int i, int j, int k, double s)
{
    double inv_h = (double)n;
    size_t c = ix(n, i, j, k);
    int ijk3[3] = {i, j, k};
    double g2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        int q = ijk3[d];
        size_t step = d == 0 ? 1 : (d == 1 ? (size_t)n : (size_t)n * n);
        double back = q > 0 ? (phi[c] - phi[c - step]) * inv_h : 0.0;
        double fwd = q < n - 1 ? (phi[c + step] - phi[c]) * inv_h : 0.0;
        double t1, t2;
        if (s > 0.0) {
            t1 = back > 0.0 ? back : 0.0;
            t2 = fwd < 0.0 ? fwd : 0.0;
        } else {
            t1 = back < 0.0 ? back : 0.0;
            t2 = fwd > 0.0 ? fwd : 0.0;
        }
        double a = t1 * t1, b = t2 * t2;
        g2 += a > b ? a : b;
    }
    return sqrt(g2);
}

/* iters pseudo-time steps of size dtau from phi (phi0 fixes the smoothed sign);
 * every step reads the previous iterate only.  out may alias phi. */
int orc_ls_reinit(int n, const double *phi0, const double *phi, int iters, double dtau,
                  double *out)
{
    if (n < 2 || !phi0 || !phi || !out || iters < 0 || !(dtau > 0.0))
        return ORC_EINVAL;
    size_t m = (size_t)n * n * n;
    double h = 1.0 / (double)n;
    double *cur = malloc(m * sizeof(double)), *nxt = malloc(m * sizeof(double));
    if (!cur || !nxt) {
        free(cur);
        free(nxt);
        return ORC_ENOMEM;
    }
    memcpy(cur, phi, m * sizeof(double));
    for (int it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    size_t c = ix(n, i, j, k);
                    double s = phi0[c] / sqrt(phi0[c] * phi0[c] + h * h);
                    double g = godunov_grad(n, cur, i, j, k, s);
                    nxt[c] = cur[c] - dtau * s * (g - 1.0);
                }
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    memcpy(out, cur, m * sizeof(double));
    free(cur);
    free(nxt);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Implicit heat diffusion: the diffusion term of the transport equation of   */
/* Sec. 2 with a coefficient that changes with the phase (the varDiffusion    */
/* configuration of HeatAD, Sec. 3), one backward-Euler step                  */
/*        (I - dt div(K grad)) T_new = T_old + dt f                           */
/* with insulated walls.  The face arrays carry K on every face; built by the */
/* face rule above from rho = 1/K of each phase they hold the two             */
/* conductivities in series, split where the interface crosses the face.      */
/* ------------------------------------------------------------------------ */

/* y = x - dt (A x) */
void orc_heat_apply(int n, const double *bx, const double *by, const double *bz, double dt,
                    const double *x, double *y)
{
    size_t m = (size_t)n * n * n;
    orc_apply(n, bx, by, bz, x, y);
    for (size_t c = 0; c < m; ++c)
        y[c] = x[c] - dt * y[c];
}

static double heat_rel_residual(int n, const double *bx, const double *by, const double *bz,
                                double dt, const double *rhs, const double *x, double *r)
{
    size_t m = (size_t)n * n * n;
    orc_heat_apply(n, bx, by, bz, dt, x, r);
    for (size_t c = 0; c < m; ++c)
        r[c] = rhs[c] - r[c];
    double bn = nrm2(rhs, m);
    double rn = nrm2(r, m);
    return bn > 0.0 ? rn / bn : rn;
}

/* Conjugate gradients (no preconditioner) on the symmetric positive definite heat
 * matrix.  x holds the start on entry and the solution on exit; stops once the true
 * residual satisfies ||rhs - H x|| <= tol ||rhs||. */
int orc_heat_solve(int n, const double *bx, const double *by, const double *bz, double dt,
                   const double *rhs, double *x, double tol, int max_iter, int *iters_out,
                   double *relres_out)
{
    if (n < 1 || !bx || !by || !bz || !rhs || !x || !(dt >= 0.0) || !(dt < INFINITY) ||
        !(tol > 0.0) || max_iter < 1)
        return ORC_EINVAL;
    size_t m = (size_t)n * n * n;
    double *r = (double *)malloc(sizeof(double) * m);
    double *p = (double *)malloc(sizeof(double) * m);
    double *q = (double *)malloc(sizeof(double) * m);
    if (!r || !p || !q) {
        free(r); free(p); free(q);
        return ORC_ENOMEM;
    }
    double bn = nrm2(rhs, m);
    int it = 0, status = ORC_ENOTCONVERGED;
    double rel = heat_rel_residual(n, bx, by, bz, dt, rhs, x, r);
    while (it < max_iter && rel > tol) {   /* restarts from the true residual */
        memcpy(p, r, sizeof(double) * m);
        double rr = dot(r, r, m);
        while (it < max_iter) {
            orc_heat_apply(n, bx, by, bz, dt, p, q);
            double pq = dot(p, q, m);
            if (!(pq > 0.0)) {
                status = ORC_EBREAKDOWN;
                goto done;
            }
            double alpha = rr / pq;
            for (size_t c = 0; c < m; ++c) {
                x[c] += alpha * p[c];
                r[c] -= alpha * q[c];
            }
            ++it;
            double rr_new = dot(r, r, m);
            if (sqrt(rr_new) <= tol * bn)
                break;
            double beta = rr_new / rr;
            rr = rr_new;
            for (size_t c = 0; c < m; ++c)
                p[c] = r[c] + beta * p[c];
        }
        rel = heat_rel_residual(n, bx, by, bz, dt, rhs, x, r);
    }
    if (rel <= tol)
        status = ORC_OK;
done:
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = rel;
    free(r); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Block-structured layout (Sec. 2: the grid is a set of blocks of cells; the  */
/* setup command of Sec. 4 uses 16^3 blocks; Sec. 4 also has the guard-cell   */
/* fill, which exchanges halos between blocks and applies the physical        */
/* boundary condition).  A problem of n^3 cells is cut into (n/nb)^3 blocks   */
/* of nb^3 cells, block (bi,bj,bk) at index bi + nbx (bj + nbx bk); each      */
/* block is stored with g guard layers on every side as (nb+2g)^3 values, x   */
/* fastest.  Guard cells hold the value of the cell at the same position in  */
/* the neighbouring block; outside the domain they mirror the field about    */
/* the wall (even reflection, the zero-gradient condition of the insulated   */
/* and no-flux walls used throughout).                                        */
/* ------------------------------------------------------------------------ */

static size_t blk_at(int nb, int g, size_t blk, int li, int lj, int lk)
{
    size_t P = (size_t)nb + 2 * (size_t)g;
    return blk * P * P * P + (size_t)(li + g) + P * ((size_t)(lj + g) + P * (size_t)(lk + g));
}

static int blk_args_ok(int n, int nb, int g)
{
    return n >= 1 && nb >= 1 && n % nb == 0 && g >= 0 && g <= nb;
}

/* grid -> block interiors (guards left as they are) */
int orc_blocks_scatter(int n, int nb, int g, const double *grid, double *blocks)
{
    if (!blk_args_ok(n, nb, g) || !grid || !blocks)
        return ORC_EINVAL;
    int nbx = n / nb;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t blk = (size_t)(i / nb) + nbx * ((size_t)(j / nb) + nbx * (size_t)(k / nb));
                blocks[blk_at(nb, g, blk, i % nb, j % nb, k % nb)] = grid[ix(n, i, j, k)];
            }
    return ORC_OK;
}

/* block interiors -> grid */
int orc_blocks_gather(int n, int nb, int g, const double *blocks, double *grid)
{
    if (!blk_args_ok(n, nb, g) || !grid || !blocks)
        return ORC_EINVAL;
    int nbx = n / nb;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t blk = (size_t)(i / nb) + nbx * ((size_t)(j / nb) + nbx * (size_t)(k / nb));
                grid[ix(n, i, j, k)] = blocks[blk_at(nb, g, blk, i % nb, j % nb, k % nb)];
            }
    return ORC_OK;
}

/* mirror a global coordinate about the walls into [0, n) */
static int mirror(int a, int n)
{
    if (a < 0)
        return -1 - a;
    if (a >= n)
        return 2 * n - 1 - a;
    return a;
}

/* every guard cell (faces, edges and corners) from the interior of the block that owns
 * its (mirrored) position */
int orc_blocks_fill_guards(int n, int nb, int g, double *blocks)
{
    if (!blk_args_ok(n, nb, g) || !blocks)
        return ORC_EINVAL;
    int nbx = n / nb;
    size_t nblk = (size_t)nbx * nbx * nbx;
    for (size_t blk = 0; blk < nblk; ++blk) {
        int bi = (int)(blk % nbx), bj = (int)((blk / nbx) % nbx), bk = (int)(blk / ((size_t)nbx * nbx));
        for (int lk = -g; lk < nb + g; ++lk)
            for (int lj = -g; lj < nb + g; ++lj)
                for (int li = -g; li < nb + g; ++li) {
                    if (li >= 0 && li < nb && lj >= 0 && lj < nb && lk >= 0 && lk < nb)
                        continue;
                    int I = mirror(bi * nb + li, n), J = mirror(bj * nb + lj, n), K = mirror(bk * nb + lk, n);
                    size_t src = (size_t)(I / nb) + nbx * ((size_t)(J / nb) + nbx * (size_t)(K / nb));
                    blocks[blk_at(nb, g, blk, li, lj, lk)] = blocks[blk_at(nb, g, src, I % nb, J % nb, K % nb)];
                }
    }
    return ORC_OK;
}

/* y = A x block by block: each interior cell reads its six neighbours from its own block
 * (guards included) and its face coefficients from the grid-layout arrays; the guards
 * of y are set to 0.  Walls carry a zero coefficient, so the mirrored guards there do
 * not enter. */
int orc_blocks_apply(int n, int nb, int g, const double *bx, const double *by, const double *bz,
                     const double *xblk, double *yblk)
{
    if (!blk_args_ok(n, nb, g) || g < 1 || !bx || !by || !bz || !xblk || !yblk)
        return ORC_EINVAL;
    int nbx = n / nb;
    size_t nblk = (size_t)nbx * nbx * nbx;
    size_t P = (size_t)nb + 2 * (size_t)g;
    double inv_h2 = (double)n * (double)n;
    memset(yblk, 0, sizeof(double) * nblk * P * P * P);
    for (size_t blk = 0; blk < nblk; ++blk) {
        int bi = (int)(blk % nbx), bj = (int)((blk / nbx) % nbx), bk = (int)(blk / ((size_t)nbx * nbx));
        for (int lk = 0; lk < nb; ++lk)
            for (int lj = 0; lj < nb; ++lj)
                for (int li = 0; li < nb; ++li) {
                    int i = bi * nb + li, j = bj * nb + lj, k = bk * nb + lk;
                    size_t c = ix(n, i, j, k);
                    double xc = xblk[blk_at(nb, g, blk, li, lj, lk)];
                    double w[6] = {bx[c], i < n - 1 ? bx[ix(n, i + 1, j, k)] : 0.0,
                                   by[c], j < n - 1 ? by[ix(n, i, j + 1, k)] : 0.0,
                                   bz[c], k < n - 1 ? bz[ix(n, i, j, k + 1)] : 0.0};
                    double xn[6] = {xblk[blk_at(nb, g, blk, li - 1, lj, lk)], xblk[blk_at(nb, g, blk, li + 1, lj, lk)],
                                    xblk[blk_at(nb, g, blk, li, lj - 1, lk)], xblk[blk_at(nb, g, blk, li, lj + 1, lk)],
                                    xblk[blk_at(nb, g, blk, li, lj, lk - 1)], xblk[blk_at(nb, g, blk, li, lj, lk + 1)]};
                    double s = 0.0;
                    for (int f = 0; f < 6; ++f)
                        s += w[f] * (xn[f] - xc);
                    yblk[blk_at(nb, g, blk, li, lj, lk)] = s * inv_h2;
                }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Two-level composite grid (Sec. 2: blocks at two resolutions, the finer one */
/* around the interface; Fig. 2 shows a block refined to half the spacing).   */
/* Level 0 has n0^3 cells (h0 = 1/n0) in blocks of nb^3; refined0[b] marks the */
/* level-0 blocks covered by level 1, whose (2 n0)^3 cells (h1 = h0 / 2) are   */
/* meaningful only inside refined blocks.  The leaf cells are the level-0     */
/* cells of unrefined blocks and the level-1 cells of refined ones.  The      */
/* operator is the conservative finite-volume form                             */
/*    (A x)_c = (1/V_c) sum_f a_f beta_f (x_nb - x_c) / d_f,                   */
/* a_f the face area, d_f the distance between the two cell centres; across a */
/* coarse-fine face the fine cell sees the coarse cell itself (d = 1.5 h1,    */
/* area h1^2) and the coarse cell the sum of the four fine fluxes, so every   */
/* flux leaves one cell and enters the other.  beta_f is the ghost-fluid      */
/* coefficient of the two cells, lower coordinate first.  Walls: no flux.     */
/* ------------------------------------------------------------------------ */

static int amr_refined(int n0, int nb, const uint8_t *refined0, int I, int J, int K)
{
    int nbx = n0 / nb;
    return refined0[(size_t)(I / nb) + nbx * ((size_t)(J / nb) + nbx * (size_t)(K / nb))] != 0;
}

/* diag != 0: the operator's diagonal instead (x read as 1 at the cell, 0 elsewhere) */
static int amr_op(int n0, int nb, const uint8_t *refined0, const double *phi0, const double *phi1,
                  const double *x0, const double *x1, double rho_neg, double rho_pos, double *y0,
                  double *y1, int diag);

int orc_amr_apply(int n0, int nb, const uint8_t *refined0, const double *phi0, const double *phi1,
                  const double *x0, const double *x1, double rho_neg, double rho_pos, double *y0,
                  double *y1)
{
    return amr_op(n0, nb, refined0, phi0, phi1, x0, x1, rho_neg, rho_pos, y0, y1, 0);
}

static int amr_op(int n0, int nb, const uint8_t *refined0, const double *phi0, const double *phi1,
                  const double *x0, const double *x1, double rho_neg, double rho_pos, double *y0,
                  double *y1, int diag)
{
    if (n0 < 1 || nb < 1 || n0 % nb || !refined0 || !phi0 || !phi1 || (!diag && (!x0 || !x1)) || !y0 || !y1 ||
        !(rho_neg > 0.0) || !(rho_pos > 0.0))
        return ORC_EINVAL;
    int n1 = 2 * n0;
    double h0 = 1.0 / n0, h1 = 0.5 * h0;
    double same0 = 1.0 / (h0 * h0), same1 = 1.0 / (h1 * h1);
    double fine_side = 1.0 / (1.5 * h1 * h1), coarse_side = 1.0 / (12.0 * h1 * h1);
    memset(y0, 0, sizeof(double) * (size_t)n0 * n0 * n0);
    memset(y1, 0, sizeof(double) * (size_t)n1 * n1 * n1);
#pragma omp parallel for schedule(static)
    for (int K = 0; K < n0; ++K)
        for (int J = 0; J < n0; ++J)
            for (int I = 0; I < n0; ++I) {
                if (amr_refined(n0, nb, refined0, I, J, K))
                    continue;
                size_t c = ix(n0, I, J, K);
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    for (int dir = -1; dir <= 1; dir += 2) {
                        int P[3] = {I, J, K};
                        P[d] += dir;
                        if (P[d] < 0 || P[d] >= n0)
                            continue;
                        if (!amr_refined(n0, nb, refined0, P[0], P[1], P[2])) {
                            size_t q = ix(n0, P[0], P[1], P[2]);
                            double beta = dir > 0 ? face_beta(phi0[c], phi0[q], rho_neg, rho_pos)
                                                  : face_beta(phi0[q], phi0[c], rho_neg, rho_pos);
                            s += beta * ((diag ? 0.0 : x0[q]) - (diag ? 1.0 : x0[c])) * same0;
                        } else {
                            /* the four fine cells across the face */
                            int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
                            for (int a = 0; a < 2; ++a)
                                for (int b = 0; b < 2; ++b) {
                                    int F[3];
                                    F[d] = dir > 0 ? 2 * P[d] : 2 * P[d] + 1;
                                    F[e1] = 2 * (e1 == 0 ? I : (e1 == 1 ? J : K)) + a;
                                    F[e2] = 2 * (e2 == 0 ? I : (e2 == 1 ? J : K)) + b;
                                    size_t q = ix(n1, F[0], F[1], F[2]);
                                    double beta = dir > 0 ? face_beta(phi0[c], phi1[q], rho_neg, rho_pos)
                                                          : face_beta(phi1[q], phi0[c], rho_neg, rho_pos);
                                    s += beta * ((diag ? 0.0 : x1[q]) - (diag ? 1.0 : x0[c])) * coarse_side;
                                }
                        }
                    }
                y0[c] = s;
            }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                if (!amr_refined(n0, nb, refined0, i / 2, j / 2, k / 2))
                    continue;
                size_t c = ix(n1, i, j, k);
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    for (int dir = -1; dir <= 1; dir += 2) {
                        int P[3] = {i, j, k};
                        P[d] += dir;
                        if (P[d] < 0 || P[d] >= n1)
                            continue;
                        if (amr_refined(n0, nb, refined0, P[0] / 2, P[1] / 2, P[2] / 2)) {
                            size_t q = ix(n1, P[0], P[1], P[2]);
                            double beta = dir > 0 ? face_beta(phi1[c], phi1[q], rho_neg, rho_pos)
                                                  : face_beta(phi1[q], phi1[c], rho_neg, rho_pos);
                            s += beta * ((diag ? 0.0 : x1[q]) - (diag ? 1.0 : x1[c])) * same1;
                        } else {
                            size_t q = ix(n0, P[0] / 2, P[1] / 2, P[2] / 2);
                            double beta = dir > 0 ? face_beta(phi1[c], phi0[q], rho_neg, rho_pos)
                                                  : face_beta(phi0[q], phi1[c], rho_neg, rho_pos);
                            s += beta * ((diag ? 0.0 : x0[q]) - (diag ? 1.0 : x1[c])) * fine_side;
                        }
                    }
                y1[c] = s;
            }
    return ORC_OK;
}

/* Guard cells of the composite grid, written into padded copies of every block of both
 * levels ([nbx0^3][P^3] and [(2 nbx0)^3][P^3], P = nb + 2g; blocks of level 1 outside
 * the refined region and refined blocks of level 0 are filled too, as if they were
 * leaves).  A guard position outside the domain is mirrored about the wall on its own
 * level.  Inside, a level-0 guard takes the level-0 value where that block is not
 * refined and the mean of the 8 level-1 cells it covers where it is; a level-1 guard
 * takes the level-1 value inside the refined region and the value of the level-0 cell
 * containing it outside. */
static double amr_value0(int n0, int nb, const uint8_t *refined0, const double *v0,
                         const double *v1, int I, int J, int K)
{
    if (!amr_refined(n0, nb, refined0, I, J, K))
        return v0[ix(n0, I, J, K)];
    /* pairwise: x pairs, then y, then z (8 equal values give that value exactly) */
    int n1 = 2 * n0;
    double q[4];
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            q[b + 2 * c] = v1[ix(n1, 2 * I, 2 * J + b, 2 * K + c)] + v1[ix(n1, 2 * I + 1, 2 * J + b, 2 * K + c)];
    return 0.125 * ((q[0] + q[1]) + (q[2] + q[3]));
}

static double amr_value1(int n0, int nb, const uint8_t *refined0, const double *v0,
                         const double *v1, int i, int j, int k)
{
    if (amr_refined(n0, nb, refined0, i / 2, j / 2, k / 2))
        return v1[ix(2 * n0, i, j, k)];
    return v0[ix(n0, i / 2, j / 2, k / 2)];
}

int orc_amr_fill(int n0, int nb, int g, const uint8_t *refined0, const double *v0, const double *v1,
                 double *blocks0, double *blocks1)
{
    if (n0 < 1 || nb < 1 || n0 % nb || g < 0 || g > nb || !refined0 || !v0 || !v1 || !blocks0 ||
        !blocks1)
        return ORC_EINVAL;
    int n1 = 2 * n0;
    for (int lev = 0; lev < 2; ++lev) {
        int n = lev ? n1 : n0, nbx = n / nb;
        double *blocks = lev ? blocks1 : blocks0;
        size_t nblk = (size_t)nbx * nbx * nbx;
        for (size_t blk = 0; blk < nblk; ++blk) {
            int bi = (int)(blk % nbx), bj = (int)((blk / nbx) % nbx), bk = (int)(blk / ((size_t)nbx * nbx));
            for (int lk = -g; lk < nb + g; ++lk)
                for (int lj = -g; lj < nb + g; ++lj)
                    for (int li = -g; li < nb + g; ++li) {
                        int I = mirror(bi * nb + li, n), J = mirror(bj * nb + lj, n), K = mirror(bk * nb + lk, n);
                        int inside = li >= 0 && li < nb && lj >= 0 && lj < nb && lk >= 0 && lk < nb;
                        double v;
                        if (inside)
                            v = lev ? v1[ix(n1, I, J, K)] : v0[ix(n0, I, J, K)];
                        else
                            v = lev ? amr_value1(n0, nb, refined0, v0, v1, I, J, K)
                                    : amr_value0(n0, nb, refined0, v0, v1, I, J, K);
                        blocks[blk_at(nb, g, blk, li, lj, lk)] = v;
                    }
        }
    }
    return ORC_OK;
}

/* Solve A x = b on the leaves of the composite grid by conjugate gradients preconditioned
 * with the inverse diagonal, in the volume-weighted inner product <u, v> = sum_leaves
 * V_c u_c v_c, in which A is symmetric and -A positive semi-definite (constants are its
 * null space, the Neumann walls).  b's weighted mean is removed first (the total volume
 * is 1); x (in: the initial guess, out: the solution) is returned with zero weighted
 * mean.  Stops when ||b' - A x|| <= rtol ||b'|| in the weighted norm (b' = b - mean).
 * Values off the leaves are ignored on input and zero on output. */
typedef struct {
    int n0, nb;
    const uint8_t *refined0;
    size_t m0, m1;
    double v0, v1;   /* cell volumes */
} amr_ctx;

static int amr_leaf(const amr_ctx *C, int lev, size_t c)
{
    int n = lev ? 2 * C->n0 : C->n0;
    int i = (int)(c % n), j = (int)((c / n) % n), k = (int)(c / ((size_t)n * n));
    if (lev)
        return amr_refined(C->n0, C->nb, C->refined0, i / 2, j / 2, k / 2);
    return !amr_refined(C->n0, C->nb, C->refined0, i, j, k);
}

static double amr_dot(const amr_ctx *C, const double *a0, const double *a1, const double *b0,
                      const double *b1)
{
    double s0 = 0.0, s1 = 0.0;
    for (size_t c = 0; c < C->m0; ++c)
        if (amr_leaf(C, 0, c))
            s0 += a0[c] * (b0 ? b0[c] : 1.0);
    for (size_t c = 0; c < C->m1; ++c)
        if (amr_leaf(C, 1, c))
            s1 += a1[c] * (b1 ? b1[c] : 1.0);
    return C->v0 * s0 + C->v1 * s1;
}

int orc_amr_solve(int n0, int nb, const uint8_t *refined0, const double *phi0, const double *phi1,
                  double rho_neg, double rho_pos, const double *b0, const double *b1, double *x0,
                  double *x1, double rtol, int max_iter, int *iters_out, double *relres_out)
{
    if (n0 < 1 || nb < 1 || n0 % nb || !refined0 || !phi0 || !phi1 || !b0 || !b1 || !x0 ||
        !x1 || !(rtol > 0.0) || max_iter < 0 || !(rho_neg > 0.0) || !(rho_pos > 0.0))
        return ORC_EINVAL;
    amr_ctx C = {n0, nb, refined0, (size_t)n0 * n0 * n0, (size_t)8 * n0 * n0 * n0,
                 1.0 / ((double)n0 * n0 * n0), 1.0 / (8.0 * n0 * n0 * n0)};
    size_t m0 = C.m0, m1 = C.m1;
    double *buf = (double *)calloc(7 * (m0 + m1), sizeof(double));
    if (!buf)
        return ORC_ENOMEM;
    double *r0 = buf, *r1 = r0 + m0, *z0 = r1 + m1, *z1 = z0 + m0, *p0 = z1 + m1, *p1 = p0 + m0;
    double *q0 = p1 + m1, *q1 = q0 + m0, *d0 = q1 + m1, *d1 = d0 + m0, *bb0 = d1 + m1,
           *bb1 = bb0 + m0, *t0 = bb1 + m1, *t1 = t0 + m0;
    /* diagonal (negated: positive) */
    amr_op(n0, nb, refined0, phi0, phi1, NULL, NULL, rho_neg, rho_pos, d0, d1, 1);
    double mean = amr_dot(&C, b0, b1, NULL, NULL);
    for (size_t c = 0; c < m0; ++c) {
        bb0[c] = amr_leaf(&C, 0, c) ? b0[c] - mean : 0.0;
        if (!amr_leaf(&C, 0, c)) x0[c] = 0.0;
    }
    for (size_t c = 0; c < m1; ++c) {
        bb1[c] = amr_leaf(&C, 1, c) ? b1[c] - mean : 0.0;
        if (!amr_leaf(&C, 1, c)) x1[c] = 0.0;
    }
    double bnorm = sqrt(amr_dot(&C, bb0, bb1, bb0, bb1));
    orc_amr_apply(n0, nb, refined0, phi0, phi1, x0, x1, rho_neg, rho_pos, q0, q1);
    for (size_t c = 0; c < m0; ++c) r0[c] = bb0[c] - q0[c];
    for (size_t c = 0; c < m1; ++c) r1[c] = bb1[c] - q1[c];
    int status = ORC_ENOTCONVERGED, it = 0;
    if (bnorm == 0.0) {
        status = ORC_OK;
    } else {
        for (size_t c = 0; c < m0; ++c) z0[c] = d0[c] != 0.0 ? r0[c] / -d0[c] : 0.0;
        for (size_t c = 0; c < m1; ++c) z1[c] = d1[c] != 0.0 ? r1[c] / -d1[c] : 0.0;
        memcpy(p0, z0, sizeof(double) * m0);
        memcpy(p1, z1, sizeof(double) * m1);
        double rz = amr_dot(&C, r0, r1, z0, z1);
        for (it = 0; it < max_iter;) {
            if (sqrt(amr_dot(&C, r0, r1, r0, r1)) <= rtol * bnorm) {
                status = ORC_OK;
                break;
            }
            orc_amr_apply(n0, nb, refined0, phi0, phi1, p0, p1, rho_neg, rho_pos, q0, q1);
            double pq = amr_dot(&C, p0, p1, q0, q1);   /* <p, A p> < 0 */
            if (!(pq < 0.0)) {
                status = ORC_EBREAKDOWN;
                break;
            }
            /* with M = -A: the step along p of CG on M x = -b' (p, z built from r = b' - A x
             * are the negatives of those CG builds from its residual -r) */
            double alpha = -rz / pq;
            for (size_t c = 0; c < m0; ++c) {
                x0[c] -= alpha * p0[c];
                r0[c] += alpha * q0[c];
                z0[c] = d0[c] != 0.0 ? r0[c] / -d0[c] : 0.0;
            }
            for (size_t c = 0; c < m1; ++c) {
                x1[c] -= alpha * p1[c];
                r1[c] += alpha * q1[c];
                z1[c] = d1[c] != 0.0 ? r1[c] / -d1[c] : 0.0;
            }
            ++it;
            double rz_new = amr_dot(&C, r0, r1, z0, z1);
            double beta = rz_new / rz;
            rz = rz_new;
            for (size_t c = 0; c < m0; ++c) p0[c] = z0[c] + beta * p0[c];
            for (size_t c = 0; c < m1; ++c) p1[c] = z1[c] + beta * p1[c];
        }
    }
    double xm = amr_dot(&C, x0, x1, NULL, NULL);
    for (size_t c = 0; c < m0; ++c) x0[c] = amr_leaf(&C, 0, c) ? x0[c] - xm : 0.0;
    for (size_t c = 0; c < m1; ++c) x1[c] = amr_leaf(&C, 1, c) ? x1[c] - xm : 0.0;
    /* the true residual of the returned x */
    orc_amr_apply(n0, nb, refined0, phi0, phi1, x0, x1, rho_neg, rho_pos, t0, t1);
    for (size_t c = 0; c < m0; ++c) t0[c] = amr_leaf(&C, 0, c) ? bb0[c] - t0[c] : 0.0;
    for (size_t c = 0; c < m1; ++c) t1[c] = amr_leaf(&C, 1, c) ? bb1[c] - t1[c] : 0.0;
    double rel = bnorm > 0.0 ? sqrt(amr_dot(&C, t0, t1, t0, t1)) / bnorm : 0.0;
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = rel;
    free(buf);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Whole pipeline: phi, f -> faces, kappa, jterm, b, p                       */
/* ------------------------------------------------------------------------ */
/* kappa_override: NULL to compute kappa from phi, else a per-cell field used as is. */
int orc_pipeline(int n, const double *phi, const double *f, double rho_neg, double rho_pos,
                 double sigma, const double *kappa_override, double *bx, double *by,
                 double *bz, double *kappa, double *jterm, double *b, double *mean_out)
{
    if (n < 2 || !(rho_neg > 0.0) || !(rho_pos > 0.0) || !(sigma >= 0.0) || !isfinite(rho_neg)
        || !isfinite(rho_pos) || !isfinite(sigma))
        return ORC_EINVAL;
    int st = orc_faces(n, phi, rho_neg, rho_pos, bx, by, bz);
    if (st) return st;
    if (kappa_override)
        memcpy(kappa, kappa_override, sizeof(double) * (size_t)n * n * n);
    else if ((st = orc_curvature(n, phi, kappa)))
        return st;
    if ((st = orc_jump(n, phi, kappa, rho_neg, rho_pos, sigma, jterm)))
        return st;
    return orc_rhs(n, f, jterm, b, mean_out);
}
