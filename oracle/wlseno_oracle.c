/*
 * WLS-ENO oracle -- numerical core.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
 * of what the WLS-ENO finite-volume path computes.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code with the GPU library.
 *
 * It follows the paper (Liu & Jiao, "WLS-ENO", arXiv:1602.02694) step by step:
 *   - Taylor/cell-average system about the cell centroid: Sec. 3.2, the 2-D and
 *     3-D cell-average equations (1-D: Sec. 3.1.1, eq. average_eq).  The
 *     factorials are read as 1/(k! l! m!) inside the sum, with 1/|tau_j| outside.
 *   - non-smoothness indicator beta and weights omega: Sec. 3.1.2, eqs.
 *     (smoothness indicator) and (weight); W = diag(omega).  In 2-D/3-D the
 *     centre's indicator is the minimum over its facet neighbours.
 *   - column scaling S = diag(1/||column||) of W A and QR with column pivoting,
 *     rank-truncated pseudo-inverse: Sec. 3.3.2, eq. (scaled_WLS) and the
 *     two pseudo-inverse formulas that follow it.
 *   - evaluation at facet quadrature points: end of Sec. 3.2.
 *   - Lax-Friedrichs flux: Sec. 1, eq. (flux); FV update eq. (fvm) read with
 *     1/|tau_i|.
 *   - third-order TVD Runge-Kutta: Sec. 4.2.1, eq. (3rd-order-Runge-Kutta).
 *
 * Compiled with -O2 -ffp-contract=off; per-cell loops may run under OpenMP.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXDIM 3
#define OR_MAXM 35
#define OR_MAXN 128
#define OR_MAXV 5
#define OR_MAXF 4
#define OR_MAXQ 8

enum { OR_ADVECTION = 0, OR_BURGERS = 1, OR_EULER = 2 };

typedef struct {
    int dim, p, m, nvars, flux, weight_mode;
    int nc, nq, periodic;
    double period, eps, alpha_w, rank_tol, h, gamma;
    double adv[3];
    const int *exps;      /* m x 3 exponents of the Taylor basis */
    const double *cv;     /* nc x (dim+1) x dim vertex coordinates of each cell */
    const double *cent;   /* nc x dim centroids */
    const double *vol;    /* nc measures */
    const int *nbr;       /* nc x (dim+1): cell across facet lf (opposite vertex lf), -1 on boundary */
    const int *row_ptr;   /* nc+1 stencil CSR, centre first */
    const int *col;
    const double *qx;     /* nc x (dim+1) x nq x dim facet quadrature points */
    const double *qw;     /* nq weights, summing to 1 */
    const double *normal; /* nc x (dim+1) x dim unit outward normals */
    const double *area;   /* nc x (dim+1) facet measures */
} or_problem;

/* ------------------------------------------------------------------ basis */

static double factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= (double)i;
    return f;
}

int or_num_coeffs(int dim, int p)
{
    /* number of monomials of total degree <= p-1 in dim variables */
    int count = 0;
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < (dim >= 2 ? p : 1); ++b)
            for (int c = 0; c < (dim >= 3 ? p : 1); ++c)
                if (a + b + c <= p - 1) ++count;
    return count;
}

/* Graded order: total degree ascending; within a degree, exponent tuples in
 * descending lexicographic order (x power first). */
int or_basis(int dim, int p, int *exps)
{
    int k = 0;
    for (int q = 0; q <= p - 1; ++q) {
        if (dim == 1) {
            exps[3 * k] = q; exps[3 * k + 1] = 0; exps[3 * k + 2] = 0; ++k;
        } else if (dim == 2) {
            for (int a = q; a >= 0; --a) {
                exps[3 * k] = a; exps[3 * k + 1] = q - a; exps[3 * k + 2] = 0; ++k;
            }
        } else {
            for (int a = q; a >= 0; --a)
                for (int b = q - a; b >= 0; --b) {
                    exps[3 * k] = a; exps[3 * k + 1] = b; exps[3 * k + 2] = q - a - b; ++k;
                }
        }
    }
    return k;
}

/* Nearest periodic image of a 1-D difference. */
static double wrap(const or_problem *P, double d)
{
    if (P->periodic) {
        double L = P->period;
        if (d > 0.5 * L) d -= L;
        else if (d < -0.5 * L) d += L;
    }
    return d;
}

/* ------------------------------------------------- exact simplex averages */

/* Average over the simplex with vertices `verts` ((dim+1) x dim) of
 *   prod_d (x_d - c_d)^{a_d} / a_d!.
 * Each factor (x_d - c_d) is affine, so with barycentric coordinates lambda,
 *   prod_t l_t(x) = sum over maps s:{1..q}->{0..dim} of prod_t lambda_{s(t)} l_t(V_{s(t)}),
 * and the simplex integral of lambda^alpha is |T| dim! alpha! / (dim+|alpha|)!.
 * The sum runs over all (dim+1)^q maps. */
double or_simplex_avg_monomial(int dim, const double *verts, const double *c, const int *a)
{
    int q = 0, fac_dim[8];
    for (int d = 0; d < dim; ++d)
        for (int e = 0; e < a[d]; ++e) fac_dim[q++] = d;
    if (q == 0) return 1.0;
    int nv = dim + 1;
    long total = 1;
    for (int t = 0; t < q; ++t) total *= nv;
    double sum = 0.0;
    int s[8];
    for (long code = 0; code < total; ++code) {
        long rem = code;
        for (int t = 0; t < q; ++t) { s[t] = (int)(rem % nv); rem /= nv; }
        int mult[4] = {0, 0, 0, 0};
        double prod = 1.0;
        for (int t = 0; t < q; ++t) {
            mult[s[t]] += 1;
            prod *= verts[s[t] * dim + fac_dim[t]] - c[fac_dim[t]];
        }
        double mf = 1.0;
        for (int v = 0; v < nv; ++v) mf *= factorial(mult[v]);
        sum += mf * prod;
    }
    double avg = sum * factorial(dim) / factorial(dim + q);
    double af = 1.0;
    for (int d = 0; d < dim; ++d) af *= factorial(a[d]);
    return avg / af;
}

/* ---------------------------------------------------- per-cell pieces */

static int stencil_size(const or_problem *P, int i) { return P->row_ptr[i + 1] - P->row_ptr[i]; }

/* Vertices of cell j shifted to the periodic image nearest cell i (1-D). */
static void image_vertices(const or_problem *P, int i, int j, double *out)
{
    int nv = P->dim + 1;
    double shift = 0.0;
    if (P->periodic) {
        double d = P->cent[j] - P->cent[i];
        shift = wrap(P, d) - d;
    }
    for (int v = 0; v < nv; ++v)
        for (int d = 0; d < P->dim; ++d)
            out[v * P->dim + d] = P->cv[((size_t)j * nv + v) * P->dim + d] + (d == 0 ? shift : 0.0);
}

/* A (n x m): averages over each stencil cell of the Taylor monomials about x_i. */
void or_cell_matrix(const or_problem *P, int i, double *A)
{
    int n = stencil_size(P, i), m = P->m;
    const int *rows = P->col + P->row_ptr[i];
    double verts[(OR_MAXDIM + 1) * OR_MAXDIM];
    const double *ci = P->cent + (size_t)i * P->dim;
    for (int r = 0; r < n; ++r) {
        image_vertices(P, i, rows[r], verts);
        for (int k = 0; k < m; ++k)
            A[r * m + k] = or_simplex_avg_monomial(P->dim, verts, ci, P->exps + 3 * k);
    }
}

/* Row weights omega for cell i from one scalar field u (length nc). */
void or_cell_weights(const or_problem *P, int i, const double *u, double *w)
{
    int n = stencil_size(P, i);
    const int *rows = P->col + P->row_ptr[i];
    if (P->weight_mode == 1) {
        for (int r = 0; r < n; ++r) w[r] = 1.0;
        return;
    }
    double eh2 = P->eps * P->h * P->h;
    double ui = u[i];
    /* beta of the centre: the smallest indicator among its facet neighbours */
    double beta_i = -1.0;
    for (int lf = 0; lf <= P->dim; ++lf) {
        int j = P->nbr[(size_t)i * (P->dim + 1) + lf];
        if (j < 0) continue;
        double b = (u[j] - ui) * (u[j] - ui) + eh2;
        if (beta_i < 0.0 || b < beta_i) beta_i = b;
    }
    if (beta_i < 0.0) beta_i = eh2;
    for (int r = 0; r < n; ++r) {
        int j = rows[r];
        if (j == i) {
            w[r] = P->alpha_w / beta_i;
        } else {
            double b = (u[j] - ui) * (u[j] - ui) + eh2;
            w[r] = 1.0 / b;
        }
    }
}

/* Solve min || W A S d - W b ||_2 with Householder QR and column pivoting,
 * truncating to the numerical rank r = #{k : |R_kk| > tol |R_11|}; returns r
 * and v = S E [R_{1:r,1:r}^{-1} (Q^T W b)_{1:r}; 0]. rdiag (length min(n,m))
 * receives the diagonal of R, perm the column order E. */
int or_wls_qrcp_solve(int n, int m, const double *A, const double *w, const double *b,
                      double tol, double *v, double *rdiag, int *perm_out)
{
    double M[OR_MAXN][OR_MAXM], rhs[OR_MAXN], s[OR_MAXM], y[OR_MAXM];
    int perm[OR_MAXM];
    for (int r = 0; r < n; ++r) {
        for (int k = 0; k < m; ++k) M[r][k] = w[r] * A[r * m + k];
        rhs[r] = w[r] * b[r];
    }
    for (int k = 0; k < m; ++k) {
        double ss = 0.0;
        for (int r = 0; r < n; ++r) ss += M[r][k] * M[r][k];
        double nrm = sqrt(ss);
        s[k] = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int r = 0; r < n; ++r) M[r][k] *= s[k];
        perm[k] = k;
    }
    int kmax = n < m ? n : m;
    for (int k = 0; k < kmax; ++k) {
        /* pivot: largest exactly recomputed partial column norm, first on ties */
        int best = k;
        double bn = -1.0;
        for (int c = k; c < m; ++c) {
            double eta = 0.0;
            for (int r = k; r < n; ++r) eta += M[r][c] * M[r][c];
            if (eta > bn) { bn = eta; best = c; }
        }
        if (best != k) {
            for (int r = 0; r < n; ++r) { double t = M[r][k]; M[r][k] = M[r][best]; M[r][best] = t; }
            int t = perm[k]; perm[k] = perm[best]; perm[best] = t;
        }
        /* Householder reflector H = I - tau v v^T with v_k = 1 (LAPACK convention) */
        double alpha = M[k][k], xn2 = 0.0;
        for (int r = k + 1; r < n; ++r) xn2 += M[r][k] * M[r][k];
        double tau, beta;
        if (xn2 == 0.0) {
            tau = 0.0;
            beta = alpha;
        } else {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tau = (beta - alpha) / beta;
            double scal = 1.0 / (alpha - beta);
            for (int r = k + 1; r < n; ++r) M[r][k] *= scal;
        }
        M[k][k] = beta;
        if (tau != 0.0) {
            for (int c = k + 1; c < m; ++c) {
                double ws = M[k][c];
                for (int r = k + 1; r < n; ++r) ws += M[r][k] * M[r][c];
                M[k][c] -= tau * ws;
                for (int r = k + 1; r < n; ++r) M[r][c] -= tau * M[r][k] * ws;
            }
            double ws = rhs[k];
            for (int r = k + 1; r < n; ++r) ws += M[r][k] * rhs[r];
            rhs[k] -= tau * ws;
            for (int r = k + 1; r < n; ++r) rhs[r] -= tau * M[r][k] * ws;
        }
    }
    for (int k = 0; k < kmax; ++k) {
        if (rdiag) rdiag[k] = M[k][k];
    }
    int rank = 0;
    double r11 = kmax > 0 ? fabs(M[0][0]) : 0.0;
    while (rank < kmax && fabs(M[rank][rank]) > tol * r11) ++rank;
    for (int k = rank - 1; k >= 0; --k) {
        double acc = rhs[k];
        for (int c = k + 1; c < rank; ++c) acc -= M[k][c] * y[c];
        y[k] = acc / M[k][k];
    }
    for (int k = 0; k < m; ++k) v[k] = 0.0;
    for (int k = 0; k < rank; ++k) v[perm[k]] = s[perm[k]] * y[k];
    if (perm_out)
        for (int k = 0; k < m; ++k) perm_out[k] = perm[k];
    return rank;
}

/* sum_k v_k prod_d dx_d^{a_kd} / a_kd! */
double or_eval_taylor(int dim, int m, const int *exps, const double *v, const double *dx)
{
    double acc = 0.0;
    for (int k = 0; k < m; ++k) {
        double term = v[k];
        for (int d = 0; d < dim; ++d) {
            int a = exps[3 * k + d];
            term *= pow(dx[d], (double)a) / factorial(a);
        }
        acc += term;
    }
    return acc;
}

/* ------------------------------------------------------------- physics */

static double euler_pressure(const or_problem *P, const double *U)
{
    double rho = U[0], ke = 0.0;
    for (int d = 0; d < P->dim; ++d) ke += U[1 + d] * U[1 + d];
    ke = 0.5 * ke / rho;
    return (P->gamma - 1.0) * (U[P->dim + 1] - ke);
}

/* physical normal flux F(U).n for every component */
static void normal_flux(const or_problem *P, const double *U, const double *n, double *F)
{
    if (P->flux == OR_ADVECTION) {
        double an = 0.0;
        for (int d = 0; d < P->dim; ++d) an += P->adv[d] * n[d];
        F[0] = an * U[0];
    } else if (P->flux == OR_BURGERS) {
        double sn = 0.0;
        for (int d = 0; d < P->dim; ++d) sn += n[d];
        F[0] = 0.5 * U[0] * U[0] * sn;
    } else {
        int D = P->dim;
        double rho = U[0], pr = euler_pressure(P, U), vn = 0.0;
        for (int d = 0; d < D; ++d) vn += U[1 + d] / rho * n[d];
        F[0] = rho * vn;
        for (int d = 0; d < D; ++d) F[1 + d] = U[1 + d] * vn + pr * n[d];
        F[D + 1] = (U[D + 1] + pr) * vn;
    }
}

/* normal spectral radius at a state (used for the Lax-Friedrichs alpha) */
static double spectral_radius(const or_problem *P, const double *U, const double *n)
{
    if (P->flux == OR_ADVECTION) {
        double an = 0.0;
        for (int d = 0; d < P->dim; ++d) an += P->adv[d] * n[d];
        return fabs(an);
    } else if (P->flux == OR_BURGERS) {
        double sn = 0.0;
        for (int d = 0; d < P->dim; ++d) sn += n[d];
        return fabs(U[0] * sn);
    } else {
        double rho = U[0], pr = euler_pressure(P, U), vn = 0.0;
        for (int d = 0; d < P->dim; ++d) vn += U[1 + d] / rho * n[d];
        return fabs(vn) + sqrt(P->gamma * pr / rho);
    }
}

/* --------------------------------------------------------- reconstruction */

static int faces_per_cell(const or_problem *P) { return P->dim + 1; }

static size_t fval_index(const or_problem *P, int var, int i, int lf, int q)
{
    int F = faces_per_cell(P);
    return (((size_t)var * P->nc + i) * F + lf) * P->nq + q;
}

/* Reconstruct one cell for every variable: coefficients, own facet values. */
static void reconstruct_cell(const or_problem *P, int i, const double *u, double *coef,
                             double *fval, int *rank, unsigned char *fallback)
{
    int n = stencil_size(P, i), m = P->m, V = P->nvars, F = faces_per_cell(P), D = P->dim;
    const int *rows = P->col + P->row_ptr[i];
    double A[OR_MAXN * OR_MAXM], w[OR_MAXN], b[OR_MAXN];
    double v[OR_MAXV][OR_MAXM];
    or_cell_matrix(P, i, A);
    for (int var = 0; var < V; ++var) {
        const double *uv = u + (size_t)var * P->nc;
        or_cell_weights(P, i, uv, w);
        for (int r = 0; r < n; ++r) b[r] = uv[rows[r]];
        int rk = or_wls_qrcp_solve(n, m, A, w, b, P->rank_tol, v[var], NULL, NULL);
        if (rank) rank[(size_t)var * P->nc + i] = rk;
    }
    /* facet values of the reconstruction */
    double vals[OR_MAXV][OR_MAXF][OR_MAXQ];
    for (int lf = 0; lf < F; ++lf)
        for (int q = 0; q < P->nq; ++q) {
            const double *x = P->qx + (((size_t)i * F + lf) * P->nq + q) * D;
            double dx[OR_MAXDIM];
            for (int d = 0; d < D; ++d) dx[d] = x[d] - P->cent[(size_t)i * D + d];
            for (int var = 0; var < V; ++var)
                vals[var][lf][q] = or_eval_taylor(D, m, P->exps, v[var], dx);
        }
    /* Euler: keep the cell averages if any facet state is not physical */
    int fb = 0;
    if (P->flux == OR_EULER) {
        for (int lf = 0; lf < F && !fb; ++lf)
            for (int q = 0; q < P->nq && !fb; ++q) {
                double U[OR_MAXV];
                for (int var = 0; var < V; ++var) U[var] = vals[var][lf][q];
                if (!(U[0] > 0.0) || !(euler_pressure(P, U) > 0.0)) fb = 1;
            }
        if (fb) {
            for (int var = 0; var < V; ++var) {
                double ub = u[(size_t)var * P->nc + i];
                for (int k = 0; k < m; ++k) v[var][k] = 0.0;
                v[var][0] = ub;
                for (int lf = 0; lf < F; ++lf)
                    for (int q = 0; q < P->nq; ++q) vals[var][lf][q] = ub;
            }
        }
    }
    if (fallback) fallback[i] = (unsigned char)fb;
    for (int var = 0; var < V; ++var) {
        if (coef)
            for (int k = 0; k < m; ++k) coef[((size_t)var * P->nc + i) * m + k] = v[var][k];
        if (fval)
            for (int lf = 0; lf < F; ++lf)
                for (int q = 0; q < P->nq; ++q) fval[fval_index(P, var, i, lf, q)] = vals[var][lf][q];
    }
}

/* u: nvars x nc.  coef: nvars x nc x m.  fval: nvars x nc x (dim+1) x nq. */
int or_reconstruct(const or_problem *P, const double *u, double *coef, double *fval, int *rank,
                   unsigned char *fallback)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < P->nc; ++i) reconstruct_cell(P, i, u, coef, fval, rank, fallback);
    return 0;
}

/* Reconstruct only the listed cells (outputs are indexed by cell id as above). */
int or_reconstruct_cells(const or_problem *P, const double *u, int ncells, const int *cells,
                         double *coef, double *fval, int *rank, unsigned char *fallback)
{
#pragma omp parallel for schedule(static)
    for (int t = 0; t < ncells; ++t) reconstruct_cell(P, cells[t], u, coef, fval, rank, fallback);
    return 0;
}

/* Lax-Friedrichs numerical flux for all components. */
static void lf_flux(const or_problem *P, const double *um, const double *up, const double *n,
                    double alpha, double *out)
{
    double Fm[OR_MAXV], Fp[OR_MAXV];
    normal_flux(P, um, n, Fm);
    normal_flux(P, up, n, Fp);
    for (int var = 0; var < P->nvars; ++var)
        out[var] = 0.5 * ((Fm[var] + Fp[var]) - alpha * (up[var] - um[var]));
}

/* Global Lax-Friedrichs alpha: the largest normal spectral radius over every
 * cell's own facet-point states (the outside states are other cells' own). */
static double global_alpha(const or_problem *P, const double *fval)
{
    int F = faces_per_cell(P), V = P->nvars, D = P->dim;
    double amax = 0.0;
    for (int i = 0; i < P->nc; ++i)
        for (int lf = 0; lf < F; ++lf)
            for (int q = 0; q < P->nq; ++q) {
                double U[OR_MAXV];
                for (int var = 0; var < V; ++var) U[var] = fval[fval_index(P, var, i, lf, q)];
                double a = spectral_radius(P, U, P->normal + ((size_t)i * F + lf) * D);
                if (a > amax) amax = a;
            }
    return amax;
}

/* dudt_i = -(1/|tau_i|) sum_facets |f| sum_q w_q Fhat(u-, u+, n) for the listed
 * cells, given every cell's coefficients and own facet values. */
static void divergence_cell(const or_problem *P, int i, const double *u, const double *coef,
                            const double *fval, const unsigned char *fallback, double alpha,
                            double *dudt)
{
    int F = faces_per_cell(P), V = P->nvars, D = P->dim, m = P->m;
    double tot[OR_MAXV];
    for (int var = 0; var < V; ++var) tot[var] = 0.0;
    for (int lf = 0; lf < F; ++lf) {
        int j = P->nbr[(size_t)i * F + lf];
        const double *n = P->normal + ((size_t)i * F + lf) * D;
        double facc[OR_MAXV];
        for (int var = 0; var < V; ++var) facc[var] = 0.0;
        for (int q = 0; q < P->nq; ++q) {
            double um[OR_MAXV], up[OR_MAXV], fh[OR_MAXV];
            for (int var = 0; var < V; ++var) um[var] = fval[fval_index(P, var, i, lf, q)];
            if (j < 0) {
                for (int var = 0; var < V; ++var) up[var] = um[var];   /* transmissive */
            } else {
                const double *x = P->qx + (((size_t)i * F + lf) * P->nq + q) * D;
                double dx[OR_MAXDIM];
                for (int d = 0; d < D; ++d) dx[d] = x[d] - P->cent[(size_t)j * D + d];
                dx[0] = wrap(P, dx[0]);
                for (int var = 0; var < V; ++var) {
                    if (fallback && fallback[j])
                        up[var] = u[(size_t)var * P->nc + j];
                    else
                        up[var] = or_eval_taylor(D, m, P->exps, coef + ((size_t)var * P->nc + j) * m, dx);
                }
            }
            double a = alpha;
            if (P->flux == OR_ADVECTION) a = spectral_radius(P, um, n);
            lf_flux(P, um, up, n, a, fh);
            for (int var = 0; var < V; ++var) facc[var] += P->qw[q] * fh[var];
        }
        for (int var = 0; var < V; ++var) tot[var] += P->area[(size_t)i * F + lf] * facc[var];
    }
    for (int var = 0; var < V; ++var) dudt[(size_t)var * P->nc + i] = -tot[var] / P->vol[i];
}

/* Full right-hand side L(u).  alpha_out (nullable) receives the LF alpha used
 * (0 for linear advection, where alpha is per facet). */
int or_rhs(const or_problem *P, const double *u, double *dudt, double *alpha_out)
{
    size_t ncoef = (size_t)P->nvars * P->nc * P->m;
    size_t nfv = (size_t)P->nvars * P->nc * faces_per_cell(P) * P->nq;
    double *coef = (double *)malloc(ncoef * sizeof(double));
    double *fval = (double *)malloc(nfv * sizeof(double));
    unsigned char *fb = (unsigned char *)calloc((size_t)P->nc, 1);
    if (!coef || !fval || !fb) { free(coef); free(fval); free(fb); return -1; }
    or_reconstruct(P, u, coef, fval, NULL, fb);
    double alpha = 0.0;
    if (P->flux != OR_ADVECTION) alpha = global_alpha(P, fval);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < P->nc; ++i) divergence_cell(P, i, u, coef, fval, fb, alpha, dudt);
    if (alpha_out) *alpha_out = alpha;
    free(coef); free(fval); free(fb);
    return 0;
}

/* n steps of the third-order TVD Runge-Kutta scheme, in place on u. */
int or_rk3(const or_problem *P, double *u, double dt, int nsteps)
{
    size_t N = (size_t)P->nvars * P->nc;
    double *L = (double *)malloc(N * sizeof(double));
    double *k1 = (double *)malloc(N * sizeof(double));
    double *k2 = (double *)malloc(N * sizeof(double));
    if (!L || !k1 || !k2) { free(L); free(k1); free(k2); return -1; }
    for (int s = 0; s < nsteps; ++s) {
        if (or_rhs(P, u, L, NULL)) goto fail;
        for (size_t t = 0; t < N; ++t) k1[t] = u[t] + dt * L[t];
        if (or_rhs(P, k1, L, NULL)) goto fail;
        for (size_t t = 0; t < N; ++t) k2[t] = 0.75 * u[t] + 0.25 * k1[t] + 0.25 * dt * L[t];
        if (or_rhs(P, k2, L, NULL)) goto fail;
        for (size_t t = 0; t < N; ++t)
            u[t] = (1.0 / 3.0) * u[t] + (2.0 / 3.0) * k2[t] + (2.0 / 3.0) * dt * L[t];
    }
    free(L); free(k1); free(k2);
    return 0;
fail:
    free(L); free(k1); free(k2);
    return -1;
}
