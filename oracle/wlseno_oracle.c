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
 * The arithmetic type `real` is double; building with -DOR_REAL='long double'
 * gives the same algorithm in x87 extended precision, used only to measure
 * the FP64 rounding floor of individual cells.  A third build compiles this
 * file as C++ with oracle/tangent.hpp force-included, -DOR_REAL=or_dual and
 * -DOR_TANGENT: the same algorithm on forward-mode dual numbers, giving the
 * exact directional derivative of the right-hand side and of the RK3
 * trajectory with every branch held at the point (or_rhs_tangent,
 * or_rk3_tangent at the end of this file).  Arrays crossing the API are
 * double in every build.
 */
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXDIM 3
#ifndef OR_MAXM
#define OR_MAXM 35
#endif
#ifndef OR_MAXN
#define OR_MAXN 128
#endif
#define OR_MAXV 5
#define OR_MAXF 4
#define OR_MAXQ 8
#define OR_PIVOT_TIE 1e-10

#ifndef OR_REAL
#define OR_REAL double
#endif
typedef OR_REAL real;
/* Geometry (vertex coordinates, monomial averages, facet-point offsets) never
 * depends on the cell averages: in the tangent build it stays plain double,
 * which gives the same values as the FP64 build without dual-number work. */
#ifndef OR_GREAL
#define OR_GREAL OR_REAL
#endif
typedef OR_GREAL greal;

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_ADVECTION = 0, OR_BURGERS = 1, OR_EULER = 2 };

typedef struct {
    int dim, p, m, nvars, flux, weight_mode;
    int nc, nq, periodic;
    int bc;               /* boundary facets: outside state 0 = inside state; 1 = zero; 2 = far[];
                             3 = (Euler) inside state with the normal momentum reversed (slip wall) */
    int characteristic;   /* Euler: 0 reconstruct conserved components; 1 characteristic fields per facet */
    double period, eps, alpha_w, rank_tol, h, gamma;
    double adv[3];
    double far[OR_MAXV];  /* bc = 2 outside state */
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
    const int *pool_ptr;  /* balance: enlarged stencils (CSR, centre first, canonical order) */
    const int *pool_col;
    int balance;          /* scalar fluxes: refit out-of-range cells on a balanced stencil */
    double period_y;      /* 2-D periodic meshes: period along y (period: along x) */
    int lf_alpha;         /* 1: local (Rusanov) alpha per facet point for Burgers and Euler */
    const double *h_cell; /* nullable: h in eps h^2 per cell (else the mesh's h) */
} or_problem;

/* Threads the per-cell loops use (1 without OpenMP). */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Use n threads in later per-cell loops (timing on one core); returns the
 * previous count. */
int or_set_num_threads(int n)
{
    int prev = or_num_threads();
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#endif
    return prev;
}

/* ------------------------------------------------------------------ basis */

static greal factorial(int k)
{
    greal f = 1.0;
    for (int i = 2; i <= k; ++i) f *= (greal)i;
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

/* Nearest periodic image of a coordinate difference along `axis` (1-D
 * circle: axis 0; 2-D periodic square: axes 0 and 1). */
static greal wrap(const or_problem *P, int axis, greal d)
{
    if (P->periodic) {
        greal L = axis == 0 ? P->period : (axis == 1 ? P->period_y : 0.0);
        if (L > 0.0) {
            if (d > 0.5 * L) d -= L;
            else if (d < -0.5 * L) d += L;
        }
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
static greal simplex_avg(int dim, const greal *verts, const greal *c, const int *a)
{
    int q = 0, fac_dim[8];
    for (int d = 0; d < dim; ++d)
        for (int e = 0; e < a[d]; ++e) fac_dim[q++] = d;
    if (q == 0) return 1.0;
    int nv = dim + 1;
    long total = 1;
    for (int t = 0; t < q; ++t) total *= nv;
    greal sum = 0.0;
    int s[8];
    for (long code = 0; code < total; ++code) {
        long rem = code;
        for (int t = 0; t < q; ++t) { s[t] = (int)(rem % nv); rem /= nv; }
        int mult[4] = {0, 0, 0, 0};
        greal prod = 1.0;
        for (int t = 0; t < q; ++t) {
            mult[s[t]] += 1;
            prod *= verts[s[t] * dim + fac_dim[t]] - c[fac_dim[t]];
        }
        greal mf = 1.0;
        for (int v = 0; v < nv; ++v) mf *= factorial(mult[v]);
        sum += mf * prod;
    }
    greal avg = sum * factorial(dim) / factorial(dim + q);
    greal af = 1.0;
    for (int d = 0; d < dim; ++d) af *= factorial(a[d]);
    return avg / af;
}

double or_simplex_avg_monomial(int dim, const double *verts, const double *c, const int *a)
{
    greal vr[(OR_MAXDIM + 1) * OR_MAXDIM], cr[OR_MAXDIM];
    for (int t = 0; t < (dim + 1) * dim; ++t) vr[t] = verts[t];
    for (int d = 0; d < dim; ++d) cr[d] = c[d];
    return (double)simplex_avg(dim, vr, cr, a);
}

/* ---------------------------------------------------- per-cell pieces */

static int stencil_size(const or_problem *P, int i) { return P->row_ptr[i + 1] - P->row_ptr[i]; }

/* Vertices of cell j shifted to the periodic image nearest cell i. */
static void image_vertices(const or_problem *P, int i, int j, greal *out)
{
    int nv = P->dim + 1;
    greal shift[OR_MAXDIM] = {0.0, 0.0, 0.0};
    if (P->periodic)
        for (int d = 0; d < P->dim; ++d) {
            greal dd = (greal)P->cent[(size_t)j * P->dim + d] - (greal)P->cent[(size_t)i * P->dim + d];
            shift[d] = wrap(P, d, dd) - dd;
        }
    for (int v = 0; v < nv; ++v)
        for (int d = 0; d < P->dim; ++d)
            out[v * P->dim + d] = (greal)P->cv[((size_t)j * nv + v) * P->dim + d] + shift[d];
}

/* A (n x m): averages over each stencil cell of the Taylor monomials about x_i. */
/* Rows of the cell-average system for stencil cells rows[0..n). */
static void cell_matrix_rows(const or_problem *P, int i, const int *rows, int n, real *A)
{
    int m = P->m;
    greal verts[(OR_MAXDIM + 1) * OR_MAXDIM], ci[OR_MAXDIM];
    for (int d = 0; d < P->dim; ++d) ci[d] = P->cent[(size_t)i * P->dim + d];
    for (int r = 0; r < n; ++r) {
        image_vertices(P, i, rows[r], verts);
        for (int k = 0; k < m; ++k) A[r * m + k] = simplex_avg(P->dim, verts, ci, P->exps + 3 * k);
    }
}

static void cell_matrix(const or_problem *P, int i, real *A)
{
    cell_matrix_rows(P, i, P->col + P->row_ptr[i], stencil_size(P, i), A);
}

void or_cell_matrix(const or_problem *P, int i, double *A)
{
    real Ar[OR_MAXN * OR_MAXM];
    cell_matrix(P, i, Ar);
    for (int t = 0; t < stencil_size(P, i) * P->m; ++t) A[t] = (double)Ar[t];
}

/* Row weights omega for cell i from the values of one scalar field: ui at the
 * centre, us[r] at stencil row r, unb[lf] at the facet neighbour across lf
 * (read only where that neighbour exists). */
static void weights_from_values(const or_problem *P, int i, int n, const int *rows, real ui, const real *us,
                                const real *unb, real *w)
{
    if (P->weight_mode == 1) {
        for (int r = 0; r < n; ++r) w[r] = 1.0;
        return;
    }
    real h = P->h_cell ? (real)P->h_cell[i] : (real)P->h;
    real eh2 = (real)P->eps * h * h;
    /* beta of the centre: the smallest indicator among its facet neighbours */
    real beta_i = -1.0;
    for (int lf = 0; lf <= P->dim; ++lf) {
        int j = P->nbr[(size_t)i * (P->dim + 1) + lf];
        if (j < 0) continue;
        real b = (unb[lf] - ui) * (unb[lf] - ui) + eh2;
        if (beta_i < 0.0 || b < beta_i) beta_i = b;
    }
    if (beta_i < 0.0) beta_i = eh2;
    for (int r = 0; r < n; ++r) {
        if (rows[r] == i) {
            w[r] = (real)P->alpha_w / beta_i;
        } else {
            real b = (us[r] - ui) * (us[r] - ui) + eh2;
            w[r] = 1.0 / b;
        }
    }
}

/* Row weights omega for cell i from one scalar field u (length nc). */
static void cell_weights(const or_problem *P, int i, const real *u, real *w)
{
    int n = stencil_size(P, i);
    const int *rows = P->col + P->row_ptr[i];
    real us[OR_MAXN], unb[OR_MAXF];
    for (int r = 0; r < n; ++r) us[r] = u[rows[r]];
    for (int lf = 0; lf <= P->dim; ++lf) {
        int j = P->nbr[(size_t)i * (P->dim + 1) + lf];
        unb[lf] = j >= 0 ? u[j] : 0.0;
    }
    weights_from_values(P, i, n, rows, u[i], us, unb, w);
}

void or_cell_weights(const or_problem *P, int i, const double *u, double *w)
{
    /* only the stencil's and the facet neighbours' entries of u are read */
    real *ur = (real *)calloc((size_t)P->nc, sizeof(real));
    real wr[OR_MAXN];
    const int *rows = P->col + P->row_ptr[i];
    for (int r = 0; r < stencil_size(P, i); ++r) ur[rows[r]] = u[rows[r]];
    for (int lf = 0; lf <= P->dim; ++lf) {
        int j = P->nbr[(size_t)i * (P->dim + 1) + lf];
        if (j >= 0) ur[j] = u[j];
    }
    cell_weights(P, i, ur, wr);
    for (int r = 0; r < stencil_size(P, i); ++r) w[r] = (double)wr[r];
    free(ur);
}

/* Solve min || W A S d - W b ||_2 with Householder QR and column pivoting,
 * truncating to the numerical rank r = #{k : |R_kk| > tol |R_11|}; returns r
 * and v = S E [R_{1:r,1:r}^{-1} (Q^T W b)_{1:r}; 0]. rdiag (length min(n,m))
 * receives the diagonal of R, perm the column order E. */
static int qrcp_solve(int n, int m, const real *A, const real *w, const real *b, real tol, real *v,
                      real *rdiag, int *perm_out)
{
    real M[OR_MAXN][OR_MAXM], rhs[OR_MAXN], s[OR_MAXM], y[OR_MAXM];
    int perm[OR_MAXM];
    for (int r = 0; r < n; ++r) {
        for (int k = 0; k < m; ++k) M[r][k] = w[r] * A[r * m + k];
        rhs[r] = w[r] * b[r];
    }
    for (int k = 0; k < m; ++k) {
        real ss = 0.0;
        for (int r = 0; r < n; ++r) ss += M[r][k] * M[r][k];
        real nrm = sqrt(ss);
        s[k] = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int r = 0; r < n; ++r) M[r][k] *= s[k];
        perm[k] = k;
    }
    int kmax = n < m ? n : m;
    for (int k = 0; k < kmax; ++k) {
        /* pivot: the largest exactly recomputed partial column norm; columns
         * within a relative OR_PIVOT_TIE of the largest count as tied and the
         * lowest index wins (after column scaling every norm is 1 at the first
         * step, and rounding must not decide the order) */
        real eta[OR_MAXM], bn = 0.0;
        for (int c = k; c < m; ++c) {
            eta[c] = 0.0;
            for (int r = k; r < n; ++r) eta[c] += M[r][c] * M[r][c];
            if (eta[c] > bn) bn = eta[c];
        }
        int best = k;
        for (int c = m - 1; c >= k; --c)
            if (eta[c] >= bn * (1.0 - OR_PIVOT_TIE)) best = c;
        if (best != k) {
            for (int r = 0; r < n; ++r) { real t = M[r][k]; M[r][k] = M[r][best]; M[r][best] = t; }
            int t = perm[k]; perm[k] = perm[best]; perm[best] = t;
        }
        /* Householder reflector H = I - tau v v^T with v_k = 1 (LAPACK convention) */
        real alpha = M[k][k], xn2 = 0.0;
        for (int r = k + 1; r < n; ++r) xn2 += M[r][k] * M[r][k];
        real tau, beta;
        if (xn2 == 0.0) {
            tau = 0.0;
            beta = alpha;
        } else {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tau = (beta - alpha) / beta;
            real scal = 1.0 / (alpha - beta);
            for (int r = k + 1; r < n; ++r) M[r][k] *= scal;
        }
        M[k][k] = beta;
        if (tau != 0.0) {
            for (int c = k + 1; c < m; ++c) {
                real ws = M[k][c];
                for (int r = k + 1; r < n; ++r) ws += M[r][k] * M[r][c];
                M[k][c] -= tau * ws;
                for (int r = k + 1; r < n; ++r) M[r][c] -= tau * M[r][k] * ws;
            }
            real ws = rhs[k];
            for (int r = k + 1; r < n; ++r) ws += M[r][k] * rhs[r];
            rhs[k] -= tau * ws;
            for (int r = k + 1; r < n; ++r) rhs[r] -= tau * M[r][k] * ws;
        }
    }
    for (int k = 0; k < kmax; ++k) {
        if (rdiag) rdiag[k] = M[k][k];
    }
    int rank = 0;
    real r11 = kmax > 0 ? fabs(M[0][0]) : 0.0;
    while (rank < kmax && fabs(M[rank][rank]) > tol * r11) ++rank;
    for (int k = rank - 1; k >= 0; --k) {
        real acc = rhs[k];
        for (int c = k + 1; c < rank; ++c) acc -= M[k][c] * y[c];
        y[k] = acc / M[k][k];
    }
    for (int k = 0; k < m; ++k) v[k] = 0.0;
    for (int k = 0; k < rank; ++k) v[perm[k]] = s[perm[k]] * y[k];
    if (perm_out)
        for (int k = 0; k < m; ++k) perm_out[k] = perm[k];
    return rank;
}

int or_wls_qrcp_solve(int n, int m, const double *A, const double *w, const double *b, double tol,
                      double *v, double *rdiag, int *perm_out)
{
    real Ar[OR_MAXN * OR_MAXM], wr[OR_MAXN], br[OR_MAXN], vr[OR_MAXM], rd[OR_MAXM];
    for (int t = 0; t < n * m; ++t) Ar[t] = A[t];
    for (int r = 0; r < n; ++r) { wr[r] = w[r]; br[r] = b[r]; }
    int rank = qrcp_solve(n, m, Ar, wr, br, tol, vr, rd, perm_out);
    for (int k = 0; k < m; ++k) v[k] = (double)vr[k];
    if (rdiag)
        for (int k = 0; k < (n < m ? n : m); ++k) rdiag[k] = (double)rd[k];
    return rank;
}

/* sum_k v_k prod_d dx_d^{a_kd} / a_kd! */
static real eval_taylor(int dim, int m, const int *exps, const real *v, const greal *dx)
{
    real acc = 0.0;
    for (int k = 0; k < m; ++k) {
        real term = v[k];
        for (int d = 0; d < dim; ++d) {
            int a = exps[3 * k + d];
            term *= pow(dx[d], (greal)a) / factorial(a);
        }
        acc += term;
    }
    return acc;
}

double or_eval_taylor(int dim, int m, const int *exps, const double *v, const double *dx)
{
    real vr[OR_MAXM];
    greal xr[OR_MAXDIM];
    for (int k = 0; k < m; ++k) vr[k] = v[k];
    for (int d = 0; d < dim; ++d) xr[d] = dx[d];
    return (double)eval_taylor(dim, m, exps, vr, xr);
}

/* ------------------------------------------------------------- physics */

static real euler_pressure(const or_problem *P, const real *U)
{
    real rho = U[0], ke = 0.0;
    for (int d = 0; d < P->dim; ++d) ke += U[1 + d] * U[1 + d];
    ke = 0.5 * ke / rho;
    return ((real)P->gamma - 1.0) * (U[P->dim + 1] - ke);
}

/* physical normal flux F(U).n for every component */
static void normal_flux(const or_problem *P, const real *U, const real *n, real *F)
{
    if (P->flux == OR_ADVECTION) {
        real an = 0.0;
        for (int d = 0; d < P->dim; ++d) an += (real)P->adv[d] * n[d];
        F[0] = an * U[0];
    } else if (P->flux == OR_BURGERS) {
        real sn = 0.0;
        for (int d = 0; d < P->dim; ++d) sn += n[d];
        F[0] = 0.5 * U[0] * U[0] * sn;
    } else {
        int D = P->dim;
        real rho = U[0], pr = euler_pressure(P, U), vn = 0.0;
        for (int d = 0; d < D; ++d) vn += U[1 + d] / rho * n[d];
        F[0] = rho * vn;
        for (int d = 0; d < D; ++d) F[1 + d] = U[1 + d] * vn + pr * n[d];
        F[D + 1] = (U[D + 1] + pr) * vn;
    }
}

/* normal spectral radius at a state (used for the Lax-Friedrichs alpha) */
static real spectral_radius(const or_problem *P, const real *U, const real *n)
{
    if (P->flux == OR_ADVECTION) {
        real an = 0.0;
        for (int d = 0; d < P->dim; ++d) an += (real)P->adv[d] * n[d];
        return fabs(an);
    } else if (P->flux == OR_BURGERS) {
        real sn = 0.0;
        for (int d = 0; d < P->dim; ++d) sn += n[d];
        return fabs(U[0] * sn);
    } else {
        real rho = U[0], pr = euler_pressure(P, U), vn = 0.0;
        for (int d = 0; d < P->dim; ++d) vn += U[1 + d] / rho * n[d];
        return fabs(vn) + sqrt((real)P->gamma * pr / rho);
    }
}

/* Characteristic decomposition of the Euler system along the unit normal n
 * (Sec. 5.2: the eigen-decomposition of the flux Jacobian, R^{-1} f' R =
 * Lambda).  Fields, in order: q_n - c, q_n (entropy), in 2-D q_n (shear,
 * along the tangent t = (-n_y, n_x)), q_n + c, with q_n = v.n, c the speed of
 * sound and H the enthalpy at the state U.  R (V x V, row-major) holds the
 * right eigenvectors as columns -- in 1-D exactly the paper's R(u) -- and L
 * its inverse, the left eigenvectors as rows (b1 = (gamma-1)/c^2,
 * b2 = |v|^2 b1 / 2). */
static void char_basis(const or_problem *P, const real *U, const real *n, real *L, real *R)
{
    int D = P->dim, V = D + 2, kc = V - 1;
    real g = (real)P->gamma, rho = U[0], vel[OR_MAXDIM], q2 = 0.0, qn = 0.0;
    for (int d = 0; d < D; ++d) {
        vel[d] = U[1 + d] / rho;
        q2 += vel[d] * vel[d];
        qn += vel[d] * n[d];
    }
    real pr = euler_pressure(P, U);
    real c = sqrt(g * pr / rho), H = (U[D + 1] + pr) / rho;
    real b1 = (g - 1.0) / (c * c), b2 = 0.5 * q2 * b1;
    for (int t = 0; t < V * V; ++t) L[t] = R[t] = 0.0;
    /* q_n - c */
    R[0 * V + 0] = 1.0;
    for (int d = 0; d < D; ++d) R[(1 + d) * V + 0] = vel[d] - c * n[d];
    R[(D + 1) * V + 0] = H - c * qn;
    L[0 * V + 0] = 0.5 * (b2 + qn / c);
    for (int d = 0; d < D; ++d) L[0 * V + 1 + d] = 0.5 * (-b1 * vel[d] - n[d] / c);
    L[0 * V + D + 1] = 0.5 * b1;
    /* q_n, entropy */
    R[0 * V + 1] = 1.0;
    for (int d = 0; d < D; ++d) R[(1 + d) * V + 1] = vel[d];
    R[(D + 1) * V + 1] = 0.5 * q2;
    L[1 * V + 0] = 1.0 - b2;
    for (int d = 0; d < D; ++d) L[1 * V + 1 + d] = b1 * vel[d];
    L[1 * V + D + 1] = -b1;
    /* q_n, shear (2-D) */
    if (D == 2) {
        real t[2] = {-n[1], n[0]};
        real qt = vel[0] * t[0] + vel[1] * t[1];
        R[1 * V + 2] = t[0];
        R[2 * V + 2] = t[1];
        R[3 * V + 2] = qt;
        L[2 * V + 0] = -qt;
        L[2 * V + 1] = t[0];
        L[2 * V + 2] = t[1];
    }
    /* q_n + c */
    R[0 * V + kc] = 1.0;
    for (int d = 0; d < D; ++d) R[(1 + d) * V + kc] = vel[d] + c * n[d];
    R[(D + 1) * V + kc] = H + c * qn;
    L[kc * V + 0] = 0.5 * (b2 - qn / c);
    for (int d = 0; d < D; ++d) L[kc * V + 1 + d] = 0.5 * (-b1 * vel[d] + n[d] / c);
    L[kc * V + D + 1] = 0.5 * b1;
}

int or_char_basis(int dim, double gamma, const double *U, const double *n, double *L, double *R)
{
    if (dim < 1 || dim > 2) return -1;
    or_problem P;
    memset(&P, 0, sizeof P);
    P.dim = dim;
    P.gamma = gamma;
    int V = dim + 2;
    real Ur[OR_MAXV], nr[OR_MAXDIM], Lr[OR_MAXV * OR_MAXV], Rr[OR_MAXV * OR_MAXV];
    for (int t = 0; t < V; ++t) Ur[t] = U[t];
    for (int d = 0; d < dim; ++d) nr[d] = n[d];
    char_basis(&P, Ur, nr, Lr, Rr);
    for (int t = 0; t < V * V; ++t) {
        L[t] = (double)Lr[t];
        R[t] = (double)Rr[t];
    }
    return 0;
}

/* Euler normal flux F(U).n of one state (pins). */
int or_euler_normal_flux(int dim, double gamma, const double *U, const double *n, double *F)
{
    if (dim < 1 || dim > 3) return -1;
    or_problem P;
    memset(&P, 0, sizeof P);
    P.dim = dim;
    P.gamma = gamma;
    P.flux = OR_EULER;
    real Ur[OR_MAXV], nr[OR_MAXDIM], Fr[OR_MAXV];
    for (int t = 0; t < dim + 2; ++t) Ur[t] = U[t];
    for (int d = 0; d < dim; ++d) nr[d] = n[d];
    normal_flux(&P, Ur, nr, Fr);
    for (int t = 0; t < dim + 2; ++t) F[t] = (double)Fr[t];
    return 0;
}

/* --------------------------------------------------------- reconstruction */

static int faces_per_cell(const or_problem *P) { return P->dim + 1; }

static size_t fval_index(const or_problem *P, int var, int i, int lf, int q)
{
    int F = faces_per_cell(P);
    return (((size_t)var * P->nc + i) * F + lf) * P->nq + q;
}

static void load_normal(const or_problem *P, int i, int lf, real *n)
{
    for (int d = 0; d < P->dim; ++d) n[d] = P->normal[((size_t)i * faces_per_cell(P) + lf) * P->dim + d];
}

/* Balanced stencil (end of Sec. 3.2): from the enlarged stencil of cell i
 * (centre first, then by distance), keep the centre and the nearest cells
 * on either side of the line/plane through the centroid orthogonal to the
 * gradient g, ceil((n-1)/2) with g.(x_j - x_i) > 0 and floor((n-1)/2) with
 * g.(x_j - x_i) <= 0; a side with too few cells leaves its share to the
 * other.  Returns the number of rows written to out (centre first, then in
 * the enlarged stencil's order). */
static int balanced_rows(const or_problem *P, int i, const real *g, int n, int *out)
{
    const int *pool = P->pool_col + P->pool_ptr[i];
    int np = P->pool_ptr[i + 1] - P->pool_ptr[i], D = P->dim;
    unsigned char plus[2 * OR_MAXN];
    int cp = 0, cm = 0;
    for (int r = 1; r < np; ++r) {
        int j = pool[r];
        real s = 0.0;
        for (int d = 0; d < D; ++d) {
            greal dd = (greal)P->cent[(size_t)j * D + d] - (greal)P->cent[(size_t)i * D + d];
            dd = wrap(P, d, dd);
            s += g[d] * dd;
        }
        plus[r] = s > 0.0;
        if (plus[r]) ++cp; else ++cm;
    }
    int qp = n / 2, qm = (n - 1) / 2;
    if (cp < qp) { qm += qp - cp; qp = cp; }
    if (cm < qm) { qp += qm - cm; qm = cm; }
    int k = 0, tp = 0, tm = 0;
    out[k++] = i;
    for (int r = 1; r < np; ++r) {
        if (plus[r] ? tp < qp : tm < qm) {
            if (plus[r]) ++tp; else ++tm;
            out[k++] = pool[r];
        }
    }
    return k;
}

int or_balanced_rows(const or_problem *P, int i, const double *g, int n, int *out)
{
    real gr[OR_MAXDIM];
    for (int d = 0; d < P->dim; ++d) gr[d] = g[d];
    return balanced_rows(P, i, gr, n, out);
}

/* Reconstruct one cell for every variable: coefficients, own facet values. */
static void reconstruct_cell(const or_problem *P, int i, const real *u, real *coef, real *fval,
                             int *rank, unsigned char *fallback, unsigned char *rebal)
{
    int n = stencil_size(P, i), m = P->m, V = P->nvars, F = faces_per_cell(P), D = P->dim;
    const int *rows = P->col + P->row_ptr[i];
    real A[OR_MAXN * OR_MAXM], w[OR_MAXN], b[OR_MAXN];
    real v[OR_MAXV][OR_MAXM];
    real vals[OR_MAXV][OR_MAXF][OR_MAXQ];
    cell_matrix(P, i, A);
    if (P->flux == OR_EULER && P->characteristic) {
        /* characteristic-wise (Sec. 5.2): for each facet, decompose along its
         * normal at the facet state (mean of the two cells' averages; the
         * cell's own average on the boundary), reconstruct every field with its
         * own weights, evaluate at the facet's points and map back with R.
         * There is no single polynomial per component: coefficients are NaN,
         * the rank is the smallest over the facets. */
        for (int var = 0; var < V; ++var) {
            for (int k = 0; k < m; ++k) v[var][k] = NAN;
            if (rank) rank[(size_t)var * P->nc + i] = m + 1;
        }
        for (int lf = 0; lf < F; ++lf) {
            int jn = P->nbr[(size_t)i * F + lf];
            real Ub[OR_MAXV], nn[OR_MAXDIM], Lc[OR_MAXV * OR_MAXV], Rc[OR_MAXV * OR_MAXV];
            for (int c = 0; c < V; ++c) {
                real ui = u[(size_t)c * P->nc + i];
                Ub[c] = jn >= 0 ? 0.5 * (ui + u[(size_t)c * P->nc + jn]) : ui;
            }
            load_normal(P, i, lf, nn);
            char_basis(P, Ub, nn, Lc, Rc);
            real wq[OR_MAXV][OR_MAXQ];
            for (int k = 0; k < V; ++k) {
                /* field k of every stencil cell and facet neighbour */
                real unb[OR_MAXF], ui = 0.0, vk[OR_MAXM];
                for (int r = 0; r < n; ++r) {
                    real t = 0.0;
                    for (int c = 0; c < V; ++c) t += Lc[k * V + c] * u[(size_t)c * P->nc + rows[r]];
                    b[r] = t;
                }
                for (int c = 0; c < V; ++c) ui += Lc[k * V + c] * u[(size_t)c * P->nc + i];
                for (int f2 = 0; f2 < F; ++f2) {
                    int j = P->nbr[(size_t)i * F + f2];
                    real t = 0.0;
                    if (j >= 0)
                        for (int c = 0; c < V; ++c) t += Lc[k * V + c] * u[(size_t)c * P->nc + j];
                    unb[f2] = t;
                }
                weights_from_values(P, i, n, rows, ui, b, unb, w);
                int rk = qrcp_solve(n, m, A, w, b, P->rank_tol, vk, NULL, NULL);
                if (rank && rk < rank[(size_t)k * P->nc + i]) rank[(size_t)k * P->nc + i] = rk;
                for (int q = 0; q < P->nq; ++q) {
                    const double *x = P->qx + (((size_t)i * F + lf) * P->nq + q) * D;
                    greal dx[OR_MAXDIM];
                    for (int d = 0; d < D; ++d) dx[d] = (greal)x[d] - (greal)P->cent[(size_t)i * D + d];
                    wq[k][q] = eval_taylor(D, m, P->exps, vk, dx);
                }
            }
            for (int q = 0; q < P->nq; ++q)
                for (int c = 0; c < V; ++c) {
                    real t = 0.0;
                    for (int k = 0; k < V; ++k) t += Rc[c * V + k] * wq[k][q];
                    vals[c][lf][q] = t;
                }
        }
    } else {
        for (int var = 0; var < V; ++var) {
            const real *uv = u + (size_t)var * P->nc;
            cell_weights(P, i, uv, w);
            for (int r = 0; r < n; ++r) b[r] = uv[rows[r]];
            int rk = qrcp_solve(n, m, A, w, b, P->rank_tol, v[var], NULL, NULL);
            if (rank) rank[(size_t)var * P->nc + i] = rk;
        }
        /* facet values of the reconstruction */
        for (int lf = 0; lf < F; ++lf)
            for (int q = 0; q < P->nq; ++q) {
                const double *x = P->qx + (((size_t)i * F + lf) * P->nq + q) * D;
                greal dx[OR_MAXDIM];
                for (int d = 0; d < D; ++d) dx[d] = (greal)x[d] - (greal)P->cent[(size_t)i * D + d];
                for (int var = 0; var < V; ++var) vals[var][lf][q] = eval_taylor(D, m, P->exps, v[var], dx);
            }
        if (P->balance && V == 1) {
            /* out of the stencil's range (beyond a rounding band)?  Then fit
             * again on a balanced stencil (end of Sec. 3.2), once. */
            real mn = u[rows[0]], mx = u[rows[0]];
            for (int r = 1; r < n; ++r) {
                real t = u[rows[r]];
                if (t < mn) mn = t;
                if (t > mx) mx = t;
            }
            real band = 1e-10 * (mx - mn) + 1e-14 * (fabs(mx) > fabs(mn) ? fabs(mx) : fabs(mn));
            int out = 0;
            for (int lf = 0; lf < F; ++lf)
                for (int q = 0; q < P->nq; ++q)
                    if (vals[0][lf][q] > mx + band || vals[0][lf][q] < mn - band) out = 1;
            if (out) {
                real g[OR_MAXDIM];
                for (int d = 0; d < D; ++d) g[d] = v[0][1 + d];
                int rows2[OR_MAXN];
                int n2 = balanced_rows(P, i, g, n, rows2);
                real A2[OR_MAXN * OR_MAXM], us[OR_MAXN], unb[OR_MAXF];
                cell_matrix_rows(P, i, rows2, n2, A2);
                for (int r = 0; r < n2; ++r) us[r] = u[rows2[r]];
                for (int f2 = 0; f2 < F; ++f2) {
                    int j = P->nbr[(size_t)i * F + f2];
                    unb[f2] = j >= 0 ? u[j] : 0.0;
                }
                weights_from_values(P, i, n2, rows2, u[i], us, unb, w);
                int rk = qrcp_solve(n2, m, A2, w, us, P->rank_tol, v[0], NULL, NULL);
                if (rank) rank[i] = rk;
                for (int lf = 0; lf < F; ++lf)
                    for (int q = 0; q < P->nq; ++q) {
                        const double *x = P->qx + (((size_t)i * F + lf) * P->nq + q) * D;
                        greal dx[OR_MAXDIM];
                        for (int d = 0; d < D; ++d) dx[d] = (greal)x[d] - (greal)P->cent[(size_t)i * D + d];
                        vals[0][lf][q] = eval_taylor(D, m, P->exps, v[0], dx);
                    }
                if (rebal) rebal[i] = 1;
            }
        }
    }
    /* Euler: keep the cell averages if any facet state is not physical */
    int fb = 0;
    if (P->flux == OR_EULER) {
        for (int lf = 0; lf < F && !fb; ++lf)
            for (int q = 0; q < P->nq && !fb; ++q) {
                real U[OR_MAXV];
                for (int var = 0; var < V; ++var) U[var] = vals[var][lf][q];
                if (!(U[0] > 0.0) || !(euler_pressure(P, U) > 0.0)) fb = 1;
            }
        if (fb) {
            for (int var = 0; var < V; ++var) {
                real ub = u[(size_t)var * P->nc + i];
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

static real *to_real(const double *x, size_t n)
{
    real *r = (real *)malloc((n ? n : 1) * sizeof(real));
    if (r)
        for (size_t t = 0; t < n; ++t) r[t] = x[t];
    return r;
}

static void to_double(const real *x, double *out, size_t n)
{
    for (size_t t = 0; t < n; ++t) out[t] = (double)x[t];
}

/* Reconstruct the listed cells (all cells when cells == NULL); outputs are
 * indexed by cell id.  u: nvars x nc.  coef: nvars x nc x m.  fval: nvars x nc
 * x (dim+1) x nq. */
static int reconstruct_api(const or_problem *P, const double *u, int ncells, const int *cells, double *coef,
                           double *fval, int *rank, unsigned char *fallback, unsigned char *rebal)
{
    size_t nu = (size_t)P->nvars * P->nc;
    size_t ncoef = nu * P->m, nfv = nu * faces_per_cell(P) * P->nq;
    real *ur = to_real(u, nu);
    real *cr = (real *)calloc(ncoef ? ncoef : 1, sizeof(real));
    real *fr = (real *)calloc(nfv ? nfv : 1, sizeof(real));
    if (!ur || !cr || !fr) { free(ur); free(cr); free(fr); return -1; }
    int count = cells ? ncells : P->nc;
#pragma omp parallel for schedule(static)
    for (int t = 0; t < count; ++t) reconstruct_cell(P, cells ? cells[t] : t, ur, cr, fr, rank, fallback, rebal);
    if (coef) to_double(cr, coef, ncoef);
    if (fval) to_double(fr, fval, nfv);
    free(ur); free(cr); free(fr);
    return 0;
}

int or_reconstruct(const or_problem *P, const double *u, double *coef, double *fval, int *rank,
                   unsigned char *fallback, unsigned char *rebal)
{
    return reconstruct_api(P, u, 0, NULL, coef, fval, rank, fallback, rebal);
}

int or_reconstruct_cells(const or_problem *P, const double *u, int ncells, const int *cells,
                         double *coef, double *fval, int *rank, unsigned char *fallback, unsigned char *rebal)
{
    return reconstruct_api(P, u, ncells, cells, coef, fval, rank, fallback, rebal);
}

/* Lax-Friedrichs numerical flux for all components. */
static void lf_flux(const or_problem *P, const real *um, const real *up, const real *n, real alpha, real *out)
{
    real Fm[OR_MAXV], Fp[OR_MAXV];
    normal_flux(P, um, n, Fm);
    normal_flux(P, up, n, Fp);
    for (int var = 0; var < P->nvars; ++var)
        out[var] = 0.5 * ((Fm[var] + Fp[var]) - alpha * (up[var] - um[var]));
}

/* Global Lax-Friedrichs alpha: the largest normal spectral radius over every
 * cell's own facet-point states (the outside states are other cells' own). */
static real global_alpha(const or_problem *P, const real *fval)
{
    int F = faces_per_cell(P), V = P->nvars;
    real amax = 0.0;
    for (int i = 0; i < P->nc; ++i)
        for (int lf = 0; lf < F; ++lf)
            for (int q = 0; q < P->nq; ++q) {
                real U[OR_MAXV], n[OR_MAXDIM];
                for (int var = 0; var < V; ++var) U[var] = fval[fval_index(P, var, i, lf, q)];
                load_normal(P, i, lf, n);
                real a = spectral_radius(P, U, n);
                if (a > amax) amax = a;
            }
    return amax;
}

/* dudt_i = -(1/|tau_i|) sum_facets |f| sum_q w_q Fhat(u-, u+, n), given every
 * cell's coefficients and own facet values. */
static void divergence_cell(const or_problem *P, int i, const real *u, const real *coef, const real *fval,
                            const unsigned char *fallback, real alpha, real *dudt)
{
    int F = faces_per_cell(P), V = P->nvars, D = P->dim, m = P->m;
    real tot[OR_MAXV];
    for (int var = 0; var < V; ++var) tot[var] = 0.0;
    for (int lf = 0; lf < F; ++lf) {
        int j = P->nbr[(size_t)i * F + lf];
        real n[OR_MAXDIM];
        load_normal(P, i, lf, n);
        real facc[OR_MAXV];
        for (int var = 0; var < V; ++var) facc[var] = 0.0;
        for (int q = 0; q < P->nq; ++q) {
            real um[OR_MAXV], up[OR_MAXV], fh[OR_MAXV];
            for (int var = 0; var < V; ++var) um[var] = fval[fval_index(P, var, i, lf, q)];
            if (j < 0) {
                /* transmissive (u+ = u-), or a zero far field (u+ = 0): with the
                 * upwind flux of linear advection, outflow unchanged and no inflow */
                for (int var = 0; var < V; ++var)
                    up[var] = P->bc == 0 ? um[var] : (P->bc == 2 ? (real)P->far[var] : 0.0);
                if (P->bc == 3) {
                    /* slip wall: mirror image of the inside state */
                    real mn = 0.0;
                    for (int d = 0; d < D; ++d) mn += um[1 + d] * n[d];
                    up[0] = um[0];
                    for (int d = 0; d < D; ++d) up[1 + d] = um[1 + d] - 2.0 * mn * n[d];
                    up[D + 1] = um[D + 1];
                }
            } else if (P->flux == OR_EULER && P->characteristic) {
                /* per-facet reconstructions: the neighbour's own value at the
                 * same point, found as its nearest facet point on a facet it
                 * shares with cell i */
                const double *x = P->qx + (((size_t)i * F + lf) * P->nq + q) * D;
                int bf = -1, bq = -1;
                greal bd = 0.0;
                for (int f2 = 0; f2 < F; ++f2) {
                    if (P->nbr[(size_t)j * F + f2] != i) continue;
                    for (int q2 = 0; q2 < P->nq; ++q2) {
                        const double *y = P->qx + (((size_t)j * F + f2) * P->nq + q2) * D;
                        greal dd = 0.0;
                        for (int d = 0; d < D; ++d) {
                            greal e = (greal)y[d] - (greal)x[d];
                            e = wrap(P, d, e);
                            dd += e * e;
                        }
                        if (bf < 0 || dd < bd) { bf = f2; bq = q2; bd = dd; }
                    }
                }
                for (int var = 0; var < V; ++var) up[var] = fval[fval_index(P, var, j, bf, bq)];
            } else {
                const double *x = P->qx + (((size_t)i * F + lf) * P->nq + q) * D;
                greal dx[OR_MAXDIM];
                for (int d = 0; d < D; ++d) dx[d] = (greal)x[d] - (greal)P->cent[(size_t)j * D + d];
                for (int d = 0; d < D; ++d) dx[d] = wrap(P, d, dx[d]);
                for (int var = 0; var < V; ++var) {
                    if (fallback && fallback[j])
                        up[var] = u[(size_t)var * P->nc + j];
                    else
                        up[var] = eval_taylor(D, m, P->exps, coef + ((size_t)var * P->nc + j) * m, dx);
                }
            }
            real a = alpha;
            if (P->flux == OR_ADVECTION) {
                a = spectral_radius(P, um, n);
            } else if (P->lf_alpha == 1) {
                /* local (Rusanov): the larger spectral radius of the two states */
                real ra = spectral_radius(P, um, n), rb = spectral_radius(P, up, n);
                a = ra > rb ? ra : rb;
            }
            lf_flux(P, um, up, n, a, fh);
            for (int var = 0; var < V; ++var) facc[var] += (real)P->qw[q] * fh[var];
        }
        for (int var = 0; var < V; ++var) tot[var] += (real)P->area[(size_t)i * F + lf] * facc[var];
    }
    for (int var = 0; var < V; ++var) dudt[(size_t)var * P->nc + i] = -tot[var] / (real)P->vol[i];
}

/* Full right-hand side L(u) in working precision. */
static int rhs_real(const or_problem *P, const real *u, real *dudt, real *alpha_out)
{
    size_t ncoef = (size_t)P->nvars * P->nc * P->m;
    size_t nfv = (size_t)P->nvars * P->nc * faces_per_cell(P) * P->nq;
    real *coef = (real *)malloc(ncoef * sizeof(real));
    real *fval = (real *)malloc(nfv * sizeof(real));
    unsigned char *fb = (unsigned char *)calloc((size_t)P->nc, 1);
    if (!coef || !fval || !fb) { free(coef); free(fval); free(fb); return -1; }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < P->nc; ++i) reconstruct_cell(P, i, u, coef, fval, NULL, fb, NULL);
    real alpha = 0.0;
    if (P->flux != OR_ADVECTION) alpha = global_alpha(P, fval);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < P->nc; ++i) divergence_cell(P, i, u, coef, fval, fb, alpha, dudt);
    if (alpha_out) *alpha_out = alpha;
    free(coef); free(fval); free(fb);
    return 0;
}

/* L(u); alpha_out (nullable) receives the LF alpha used (0 for linear
 * advection, where alpha is per facet). */
int or_rhs(const or_problem *P, const double *u, double *dudt, double *alpha_out)
{
    size_t N = (size_t)P->nvars * P->nc;
    real *ur = to_real(u, N), *Lr = (real *)malloc(N * sizeof(real)), a = 0.0;
    if (!ur || !Lr) { free(ur); free(Lr); return -1; }
    int st = rhs_real(P, ur, Lr, &a);
    if (!st) to_double(Lr, dudt, N);
    if (alpha_out) *alpha_out = (double)a;
    free(ur); free(Lr);
    return st;
}

/* n steps of the third-order TVD Runge-Kutta scheme, in place on the
 * working-precision state U (carried in working precision between stages
 * and steps):
 *   k1 = u + dt L(u);  k2 = 3/4 u + 1/4 k1 + 1/4 dt L(k1);
 *   u  = 1/3 u + 2/3 k2 + 2/3 dt L(k2). */
static int rk3_real(const or_problem *P, real *U, real dt, int nsteps)
{
    size_t N = (size_t)P->nvars * P->nc;
    int st = -1;
    real *L = (real *)malloc(N * sizeof(real));
    real *k1 = (real *)malloc(N * sizeof(real));
    real *k2 = (real *)malloc(N * sizeof(real));
    if (!L || !k1 || !k2) goto done;
    for (int s = 0; s < nsteps; ++s) {
        if (rhs_real(P, U, L, NULL)) goto done;
        for (size_t t = 0; t < N; ++t) k1[t] = U[t] + dt * L[t];
        if (rhs_real(P, k1, L, NULL)) goto done;
        for (size_t t = 0; t < N; ++t) k2[t] = 0.75 * U[t] + 0.25 * k1[t] + 0.25 * dt * L[t];
        if (rhs_real(P, k2, L, NULL)) goto done;
        for (size_t t = 0; t < N; ++t)
            U[t] = ((real)1.0 / 3.0) * U[t] + ((real)2.0 / 3.0) * k2[t] + ((real)2.0 / 3.0) * dt * L[t];
    }
    st = 0;
done:
    free(L); free(k1); free(k2);
    return st;
}

int or_rk3(const or_problem *P, double *u, double dt_in, int nsteps)
{
    size_t N = (size_t)P->nvars * P->nc;
    real *U = to_real(u, N);
    if (!U) return -1;
    int st = rk3_real(P, U, (real)dt_in, nsteps);
    if (!st) to_double(U, u, N);
    free(U);
    return st;
}

#ifdef OR_TANGENT
/* ------------------------------------------------------------- tangents */

/* Directions per call (the dual number's width). */
int or_ndir(void) { return OR_NDIR; }

/* The state u (nvars x nc) with ndir directions du (ndir x nvars x nc); the
 * dual numbers carry ndir derivatives from here on. */
static real *seed_state(const double *u, const double *du, int ndir, size_t N)
{
    or_nd = ndir > 0 ? ndir : 1;
    real *U = (real *)malloc((N ? N : 1) * sizeof(real));
    if (U)
        for (size_t t = 0; t < N; ++t) U[t] = or_seed(u[t], du + t, ndir, N);
    return U;
}

static void split_state(const real *U, int ndir, size_t N, double *u, double *du)
{
    for (size_t t = 0; t < N; ++t) {
        u[t] = U[t].v;
        for (int k = 0; k < ndir; ++k) du[(size_t)k * N + t] = U[t].d[k];
    }
}

/* L(u) and its directional derivatives J(u) du_k, k < ndir <= or_ndir(). */
int or_rhs_tangent(const or_problem *P, const double *u, const double *du, int ndir, double *dudt,
                   double *ddudt)
{
    size_t N = (size_t)P->nvars * P->nc;
    if (ndir < 0 || ndir > OR_NDIR) return -2;
    real *U = seed_state(u, du, ndir, N);
    real *L = (real *)malloc((N ? N : 1) * sizeof(real));
    int st = -1;
    if (U && L) st = rhs_real(P, U, L, NULL);
    if (!st) split_state(L, ndir, N, dudt, ddudt);
    free(U); free(L);
    return st;
}

/* nsteps RK3 steps in place on u, and in place on the directions du:
 * du_k <- (d u(T) / d u0) du_k, the exact tangent of the trajectory. */
int or_rk3_tangent(const or_problem *P, double *u, double *du, int ndir, double dt, int nsteps)
{
    size_t N = (size_t)P->nvars * P->nc;
    if (ndir < 0 || ndir > OR_NDIR) return -2;
    real *U = seed_state(u, du, ndir, N);
    if (!U) return -1;
    int st = rk3_real(P, U, (real)dt, nsteps);
    if (!st) split_state(U, ndir, N, u, du);
    free(U);
    return st;
}
#endif

#ifdef __cplusplus
}
#endif
