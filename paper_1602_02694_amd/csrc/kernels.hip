// WLS-ENO device kernels for gfx950 (MI355X).
//
//  k_reconstruct : one cell per group of 4 lanes (a DPP quad).  Each lane holds
//                  RPL rows of the cell's weighted, column-scaled Taylor system
//                  in registers; column norms and Householder dot products are
//                  reduced across the quad with DPP quad_perm butterflies, so
//                  every lane of a cell sees bitwise-identical sums and takes
//                  the same pivot decisions.  Output: the degree p-1
//                  polynomial evaluated at the cell's own facet points
//                  (Sec. 3.1-3.3 of the paper).
//  k_update      : one thread per cell.  Lax-Friedrichs flux at every facet
//                  point (Sec. 1, eq. flux), computed by both cells of a facet
//                  from identical operands in the orientation of the facet's
//                  lower-numbered cell, so the two contributions are exact
//                  negatives (conservative, deterministic, no atomics); then
//                  L_i = -(1/|tau_i|) sum_f |f| sum_q w_q Fhat and the TVD RK3
//                  stage combination (Sec. 4.2.1).
//  k_permute     : user order <-> device (reverse Cuthill-McKee) order.
//
// All arithmetic is FP64 on the vector ALUs: these are tiny independent
// least-squares solves, not a dense contraction, so MFMA does not apply.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "internal.hpp"

#define WLSENO_HD __device__
#include "grid_sync.hpp"

namespace wlseno {
namespace {

constexpr int kFluxAdv = WLSENO_FLUX_ADVECTION;
constexpr double kPivotTie = 1e-10;
constexpr int kFluxBurgers = WLSENO_FLUX_BURGERS;
constexpr int kFluxEuler = WLSENO_FLUX_EULER;
// Euler reconstructed in characteristic fields per facet (a kernel variant,
// not a flux of the interface: the flux itself is the Euler one)
constexpr int kFluxEulerChar = 16;

constexpr int binom(int n, int k)
{
    int r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

template <int DIM, int P>
struct Basis {
    static constexpr int M = binom(P - 1 + DIM, DIM);
    int e[M][3];
    constexpr Basis() : e{}
    {
        int k = 0;
        for (int q = 0; q <= P - 1; ++q) {
            if (DIM == 1) {
                e[k][0] = q; e[k][1] = 0; e[k][2] = 0; ++k;
            } else if (DIM == 2) {
                for (int a = q; a >= 0; --a) { e[k][0] = a; e[k][1] = q - a; e[k][2] = 0; ++k; }
            } else {
                for (int a = q; a >= 0; --a)
                    for (int b = q - a; b >= 0; --b) { e[k][0] = a; e[k][1] = b; e[k][2] = q - a - b; ++k; }
            }
        }
    }
    constexpr int deg(int k) const { return e[k][0] + e[k][1] + e[k][2]; }
    // beta_t <= alpha_k componentwise
    constexpr bool le(int t, int k) const
    {
        return e[t][0] <= e[k][0] && e[t][1] <= e[k][1] && e[t][2] <= e[k][2];
    }
};

template <int DIM, int P>
constexpr int num_q() { return DIM == 1 ? 1 : (DIM == 2 ? ((P + 1) / 2 > 1 ? (P + 1) / 2 : 1) : 3); }

// Geometry record stride: centroid + moments of degree 2..P-1, padded to even.
template <int DIM, int P>
constexpr int geo_stride()
{
    int s = DIM + (Basis<DIM, P>::M - 1 - DIM);
    return (s & 1) ? s + 1 : s;
}

// ------------------------------------------------------------ lane exchange

template <int CTRL>
__device__ __forceinline__ double dpp_d(double x)
{
    int lo = __double2loint(x);
    int hi = __double2hiint(x);
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 4 lanes of a quad; identical bits in all four lanes.
__device__ __forceinline__ double quad_sum(double x)
{
    x = x + dpp_d<0xB1>(x);   // quad_perm [1,0,3,2]
    x = x + dpp_d<0x4E>(x);   // quad_perm [2,3,0,1]
    return x;
}

// Value of lane l of the quad (l is a constant after unrolling).
__device__ __forceinline__ double quad_bcast(double x, int l)
{
    switch (l & 3) {
    case 0: return dpp_d<0x00>(x);
    case 1: return dpp_d<0x55>(x);
    case 2: return dpp_d<0xAA>(x);
    default: return dpp_d<0xFF>(x);
    }
}

// Sum over a group of G = 2, 4, 8 or 16 lanes.  Beyond the quad, partial sums
// are exchanged with row_half_mirror (lane i <-> 7-i) and row_mirror
// (i <-> 15-i): every lane adds the same two operands, so all lanes of the
// group hold identical bits.
template <int G>
__device__ __forceinline__ double group_sum(double x)
{
    if constexpr (G == 2) return x + dpp_d<0xB1>(x);   // quad_perm [1,0,3,2]
    x = quad_sum(x);
    if constexpr (G >= 8) x = x + dpp_d<0x141>(x);
    if constexpr (G >= 16) x = x + dpp_d<0x140>(x);
    return x;
}

// Maximum / minimum over a group of G lanes (same exchange pattern as group_sum).
template <int G>
__device__ __forceinline__ double group_max(double x)
{
    x = fmax(x, dpp_d<0xB1>(x));
    if constexpr (G >= 4) x = fmax(x, dpp_d<0x4E>(x));
    if constexpr (G >= 8) x = fmax(x, dpp_d<0x141>(x));
    if constexpr (G >= 16) x = fmax(x, dpp_d<0x140>(x));
    return x;
}

template <int G>
__device__ __forceinline__ double group_min(double x)
{
    x = fmin(x, dpp_d<0xB1>(x));
    if constexpr (G >= 4) x = fmin(x, dpp_d<0x4E>(x));
    if constexpr (G >= 8) x = fmin(x, dpp_d<0x141>(x));
    if constexpr (G >= 16) x = fmin(x, dpp_d<0x140>(x));
    return x;
}

template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long x)
{
    int lo = (int)(unsigned)(x & 0xffffffffull);
    int hi = (int)(unsigned)(x >> 32);
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo;
}

// Bitwise OR over a group of G lanes.
template <int G>
__device__ __forceinline__ unsigned long long group_or(unsigned long long x)
{
    x |= dpp_u64<0xB1>(x);
    if constexpr (G >= 4) x |= dpp_u64<0x4E>(x);
    if constexpr (G >= 8) x |= dpp_u64<0x141>(x);
    if constexpr (G >= 16) x |= dpp_u64<0x140>(x);
    return x;
}

// Value of lane l (constant after unrolling) of the group, for lane g.
template <int G>
__device__ __forceinline__ double group_bcast(double x, int l, int g)
{
    if constexpr (G == 2) {
        // lane l of this lane's pair: quad_perm [0,0,2,2] or [1,1,3,3]
        return (l & 1) ? dpp_d<0xF5>(x) : dpp_d<0xA0>(x);
    }
    const double t = quad_bcast(x, l & 3);          // lane l&3 of this lane's quad
    if constexpr (G == 4) {
        return t;
    } else if constexpr (G == 8) {
        const double o = dpp_d<0x141>(t);           // ... of the other quad of the 8
        return ((g >> 2) == (l >> 2)) ? t : o;
    } else {
        // quads reachable: own (q), half mirror (q^1), mirror (q^3), both (q^2)
        const double t1 = dpp_d<0x141>(t);
        const double t2 = dpp_d<0x140>(t);
        const double t3 = dpp_d<0x140>(t1);
        const int d = (g >> 2) ^ (l >> 2);
        return d == 0 ? t : (d == 1 ? t1 : (d == 3 ? t2 : t3));
    }
}

// Maximum over the wavefront, valid in lane 0: DPP within rows of 16, then
// the four row results read back by lane.
__device__ __forceinline__ double wave_max(double x)
{
    x = fmax(x, dpp_d<0xB1>(x));
    x = fmax(x, dpp_d<0x4E>(x));
    x = fmax(x, dpp_d<0x141>(x));
    x = fmax(x, dpp_d<0x140>(x));
    double m = x;
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        const int lo = __builtin_amdgcn_readlane(__double2loint(x), 16 * r);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(x), 16 * r);
        m = fmax(m, __hiloint2double(hi, lo));
    }
    return m;
}

// pw[d][a] = x_d^a / a!
template <int DIM, int P>
__device__ __forceinline__ void scaled_powers(const double (&x)[DIM], double (&pw)[DIM][P])
{
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        pw[d][0] = 1.0;
#pragma unroll
        for (int a = 1; a < P; ++a) pw[d][a] = pw[d][a - 1] * x[d] * (1.0 / a);
    }
}

// Point q of a 1-D or 2-D facet with end points a and b (relative to the
// centroid): 1-D the point itself; 2-D Gauss-Legendre nodes along the edge.
template <int DIM, int Q>
__device__ __forceinline__ void edge_point(const double (&a)[DIM], const double (&b)[DIM], int q, double (&x)[DIM])
{
    if constexpr (DIM == 1) {
        x[0] = a[0];
    } else {
        double t;
        if constexpr (Q == 1) {
            t = 0.5;
        } else if constexpr (Q == 2) {
            // Gauss-Legendre nodes on [0,1], ascending
            const double h = 0.5 / 1.7320508075688772;   // 1/(2 sqrt 3)
            t = q == 0 ? 0.5 - h : 0.5 + h;
        } else {
            static_assert(Q == 3, "up to three points per edge");
            const double h = 0.38729833462074170;        // sqrt(3/5) / 2
            t = q == 0 ? 0.5 - h : (q == 1 ? 0.5 : 0.5 + h);
        }
#pragma unroll
        for (int d = 0; d < DIM; ++d) x[d] = a[d] + t * (b[d] - a[d]);
    }
}

// Point q of facet lf of a tetrahedron (vertex offsets vr from the centroid):
// the degree-2 rule with barycentric coordinates (2/3, 1/6, 1/6).
template <int DIM, int Q>
__device__ __forceinline__ void facet_point(const double *vr, int lf, int q, double (&x)[DIM])
{
    static_assert(DIM == 3, "tetrahedral facets only");
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const double w = (t == q) ? (2.0 / 3.0) : (1.0 / 6.0);
            s += w * vr[((lf + 1 + t) % 4) * 3 + d];
        }
        x[d] = s;
    }
}

template <int DIM, int Q>
__device__ __forceinline__ double quad_weight(int q)
{
    if constexpr (DIM == 1) return 1.0;
    else if constexpr (DIM == 2) return Q == 1 ? 1.0 : (Q == 2 ? 0.5 : (q == 1 ? 8.0 / 18.0 : 5.0 / 18.0));
    else return 1.0 / 3.0;
}

struct RArgs {
    int64_t nc;
    const double *u, *geo, *vrel, *nsum, *normal;
    const int32_t *spad, *sib, *perm;
    double *fv;
    double *coef_user, *fv_user;
    int32_t *rank_user;
    unsigned long long *alpha_acc;   // this stage's parity: nmesh x spm slots (stride 16)
    const int32_t *mid;              // batches: mesh of each cell (else null)
    const double *eh2_tab;           // batches: eps h^2 per mesh
    const double *eh2_cell;          // h_mode 1: eps h_i^2 per cell (else null)
    int spm;                         // alpha slots per mesh
    double eh2, alpha_w, rank_tol, period, period_y, gamma;
    int weight_mode;
    double *bal_grad;                // balanced-stencil refit: gradients of the first fit
    unsigned long long *bal_count;   // and this stage's list length (read by the refit)
    // stencil-size buckets: cells [cell0[b], cell0[b+1]) run with rpl[b] rows
    // per lane, in workgroups [blk0[b], blk0[b+1])
    int64_t cell0[kMaxBuckets + 1];
    int blk0[kMaxBuckets + 1];
    int64_t spad_off[kMaxBuckets + 1];   // padded stencil table of bucket b
    int stride[kMaxBuckets];             // its entries per cell
};

// 1/x to ~1 ulp: hardware estimate and two Newton steps (x finite, nonzero).
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// 1/sqrt(x) to ~1 ulp (x > 0): hardware estimate and two Newton steps.
__device__ __forceinline__ double rsq_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    return fma(y, e, y);
}

// Workgroups are handed to the 8 XCDs round robin; renumber them so that each
// XCD works on one contiguous range of cells and stencil neighbours share its L2.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int xcd = b & 7, idx = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// ------------------------------------------------------ per-cell solve

// Characteristic decomposition of the 2-D Euler system along the unit normal
// of facet fl of cell c (Sec. 5.1.4 gives R(u) in 1-D; Sec. 5.2.4 applies it
// along facet normals): row v of L = R^{-1} and column v of R at the facet
// state, the mean of the averages of c and of its neighbour across fl (c's own
// average on the boundary).  Fields: q_n - c, q_n (entropy), q_n (shear, along
// (-n_y, n_x)), q_n + c.
__device__ __forceinline__ void char_vectors(const double *u, const double *normal, const int32_t *sib, int64_t N,
                                             int64_t c, int fl, int v, double gamma, double (&Lr)[4],
                                             double (&Rc)[4])
{
    const int32_t sbf = sib[(int64_t)fl * N + c];
    const int64_t nb = sbf >= 0 ? (int64_t)(sbf >> 2) : c;
    double U[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double ui = u[(int64_t)k * N + c], uj = u[(int64_t)k * N + nb];
        U[k] = sbf >= 0 ? 0.5 * (ui + uj) : ui;
    }
    double nx = normal[((int64_t)fl * N + c) * 2 + 0], ny = normal[((int64_t)fl * N + c) * 2 + 1];
    const double il = 1.0 / sqrt(nx * nx + ny * ny);
    nx *= il;
    ny *= il;
    const double rho = U[0], ux = U[1] / rho, uy = U[2] / rho;
    const double q2 = ux * ux + uy * uy, qn = ux * nx + uy * ny;
    const double pr = (gamma - 1.0) * (U[3] - 0.5 * (U[1] * U[1] + U[2] * U[2]) / rho);
    const double cs = sqrt(gamma * pr / rho), H = (U[3] + pr) / rho;
    const double b1 = (gamma - 1.0) / (cs * cs), b2 = 0.5 * q2 * b1;
    if (v == 0) {
        Rc[0] = 1.0; Rc[1] = ux - cs * nx; Rc[2] = uy - cs * ny; Rc[3] = H - cs * qn;
        Lr[0] = 0.5 * (b2 + qn / cs); Lr[1] = 0.5 * (-b1 * ux - nx / cs); Lr[2] = 0.5 * (-b1 * uy - ny / cs);
        Lr[3] = 0.5 * b1;
    } else if (v == 1) {
        Rc[0] = 1.0; Rc[1] = ux; Rc[2] = uy; Rc[3] = 0.5 * q2;
        Lr[0] = 1.0 - b2; Lr[1] = b1 * ux; Lr[2] = b1 * uy; Lr[3] = -b1;
    } else if (v == 2) {
        const double qt = -ux * ny + uy * nx;
        Rc[0] = 0.0; Rc[1] = -ny; Rc[2] = nx; Rc[3] = qt;
        Lr[0] = -qt; Lr[1] = -ny; Lr[2] = nx; Lr[3] = 0.0;
    } else {
        Rc[0] = 1.0; Rc[1] = ux + cs * nx; Rc[2] = uy + cs * ny; Rc[3] = H + cs * qn;
        Lr[0] = 0.5 * (b2 - qn / cs); Lr[1] = 0.5 * (-b1 * ux + nx / cs); Lr[2] = 0.5 * (-b1 * uy + ny / cs);
        Lr[3] = 0.5 * b1;
    }
}

// Centroid offset of a stencil cell (record gxs: centroid, then moments) from
// x_c, wrapped to the nearest periodic image on a periodic line (period) or
// square (period along x, period_y along y).
template <int DIM>
__device__ __forceinline__ void centroid_offset(const double *gxs, const double (&xc)[DIM], double period,
                                                double period_y, double (&dl)[DIM])
{
#pragma unroll
    for (int d = 0; d < DIM; ++d) dl[d] = gxs[d] - xc[d];
    if constexpr (DIM <= 2) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const double L = d == 0 ? period : period_y;
            if (L > 0.0) dl[d] = dl[d] > 0.5 * L ? dl[d] - L : (dl[d] < -0.5 * L ? dl[d] + L : dl[d]);
        }
    }
}

// Average over a stencil cell of every Taylor monomial about x_c, from its
// centroid offset dl and centred moments nu(a) = mu(a)/a! (2 <= |a| <= p-1):
//   sum_{t <= k} (dl^{a_k - a_t} / (a_k - a_t)!) nu(a_t),  nu(0) = 1, nu(|a| = 1) = 0.
template <int DIM, int P>
__device__ __forceinline__ void taylor_row(const double (&dl)[DIM], const double *nu, double (&row)[Basis<DIM, P>::M])
{
    constexpr Basis<DIM, P> B{};
    constexpr int M = Basis<DIM, P>::M;
    double pw[DIM][P];
    scaled_powers<DIM, P>(dl, pw);
#pragma unroll
    for (int k = 0; k < M; ++k) {
        double acc = 1.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) acc *= pw[d][B.e[k][d]];
#pragma unroll
        for (int t = 1 + DIM; t < M; ++t) {
            if (B.le(t, k)) {
                double ph = nu[t - 1 - DIM];
#pragma unroll
                for (int d = 0; d < DIM; ++d) ph *= pw[d][B.e[k][d] - B.e[t][d]];
                acc += ph;
            }
        }
        row[k] = acc;
    }
}

// Column scaling S = diag(1 / ||(W A)_k||): sc[k], and A <- A S.
template <int M, int G, int RPL>
__device__ __forceinline__ void scale_columns(double (&A)[RPL][M], double (&sc)[M])
{
#pragma unroll
    for (int k = 0; k < M; ++k) {
        double t = 0.0;
#pragma unroll
        for (int s = 0; s < RPL; ++s) t = fma(A[s][k], A[s][k], t);
        t = group_sum<G>(t);
        sc[k] = t > 0.0 ? rsq_nr(t) : 0.0;
#pragma unroll
        for (int s = 0; s < RPL; ++s) A[s][k] *= sc[k];
    }
}

// Householder QR with column pivoting of the rows A (row r = s G + g in lane
// g, slot s) and right-hand side bv, in place.  R row k goes to lane k % G,
// slot k / G of Rs (with (Q^T b)_k in cs); rd = diag R, rinv = 1 / diag R,
// pm = the column order, sc is permuted along.
template <int M, int G, int RPL, int RS>
__device__ __forceinline__ void qrcp(double (&A)[RPL][M], double (&bv)[RPL], double (&sc)[M], int g, int (&pm)[M],
                                     double (&rd)[M], double (&rinv)[M], double (&Rs)[RS][M], double (&cs)[RS])
{
    // Householder QR with column pivoting.  Rows < k are retired into the
    // owner lane's R store (Rs, cs) and zeroed in A, so every reduction runs
    // over all slots without row predicates.  Column exchanges and row
    // retirement run under lane masks (cells of a wave pivot independently);
    // an exchange no cell of the wave needs is skipped.
#pragma unroll
    for (int k = 0; k < M; ++k) pm[k] = k;
#pragma unroll
    for (int s = 0; s < RS; ++s) {
        cs[s] = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) Rs[s][k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
        double best;
        if (k == 0) {
            // After the scaling every nonzero column has unit norm and column 0
            // (the weights themselves) is never zero, so under the tie rule the
            // first pivot is always column 0: no search, no exchange.
            double t = 0.0;
#pragma unroll
            for (int s = 0; s < RPL; ++s) t = fma(A[s][0], A[s][0], t);
            best = group_sum<G>(t);
        } else {
            double eta[M];
#pragma unroll
            for (int cc = k; cc < M; ++cc) {
                double t = 0.0;
#pragma unroll
                for (int s = 0; s < RPL; ++s) t = fma(A[s][cc], A[s][cc], t);
                eta[cc] = group_sum<G>(t);
            }
            // pivot: lowest column index among those within a relative kPivotTie
            // of the largest partial norm (rounding must not order ties)
            double mx[M];
#pragma unroll
            for (int cc = k; cc < M; ++cc) mx[cc] = eta[cc];
#pragma unroll
            for (int w = 1; w < M - k; w *= 2)
#pragma unroll
                for (int cc = k; cc + w < M; cc += 2 * w) mx[cc] = fmax(mx[cc], mx[cc + w]);
            const double tie = mx[k] * (1.0 - kPivotTie);
            unsigned msk = 0u;
#pragma unroll
            for (int cc = k; cc < M; ++cc) msk |= (eta[cc] >= tie) ? (1u << cc) : 0u;
            const int piv = msk ? __builtin_ctz(msk) : k;
            best = eta[k];
#pragma unroll
            for (int cc = k + 1; cc < M; ++cc) {
                if (piv == cc) {
                    best = eta[cc];
#pragma unroll
                    for (int s = 0; s < RPL; ++s) {
                        const double t0 = A[s][k];
                        A[s][k] = A[s][cc];
                        A[s][cc] = t0;
                    }
                    // a pivot exchanges whole columns: the R entries of retired rows too
#pragma unroll
                    for (int s = 0; s < RS; ++s) {
                        if (s * G < k) {
                            const double t0 = Rs[s][k];
                            Rs[s][k] = Rs[s][cc];
                            Rs[s][cc] = t0;
                        }
                    }
                    const double s0 = sc[k];
                    sc[k] = sc[cc];
                    sc[cc] = s0;
                    const int p0 = pm[k];
                    pm[k] = pm[cc];
                    pm[cc] = p0;
                }
            }
        }
        const double alpha = group_bcast<G>(A[k / G][k], k % G, g);
        const bool nz = best > 0.0;
        // beta = -sign(alpha) ||x||, and 1/beta, from one reciprocal square root
        const double rs = nz ? rsq_nr(best) : 0.0;
        const double beta = nz ? -copysign(best * rs, alpha) : 0.0;
        const double rb = -copysign(rs, alpha);
        const double tau = (beta - alpha) * rb;
        const double scal = nz ? rcp_nr(alpha - beta) : 0.0;
        const bool own = g == (k % G);
        double v[RPL];
#pragma unroll
        for (int s = 0; s < RPL; ++s) v[s] = A[s][k] * scal;
        v[k / G] = own ? 1.0 : v[k / G];
#pragma unroll
        for (int cc = k + 1; cc < M; ++cc) {
            double t = 0.0;
#pragma unroll
            for (int s = 0; s < RPL; ++s) t = fma(v[s], A[s][cc], t);
            const double tw = tau * group_sum<G>(t);
#pragma unroll
            for (int s = 0; s < RPL; ++s) A[s][cc] = fma(-tw, v[s], A[s][cc]);
        }
        {
            double t = 0.0;
#pragma unroll
            for (int s = 0; s < RPL; ++s) t = fma(v[s], bv[s], t);
            const double tw = tau * group_sum<G>(t);
#pragma unroll
            for (int s = 0; s < RPL; ++s) bv[s] = fma(-tw, v[s], bv[s]);
        }
        rd[k] = beta;
        rinv[k] = rb;
        if (own) {
#pragma unroll
            for (int cc = k + 1; cc < M; ++cc) {
                Rs[k / G][cc] = A[k / G][cc];
                A[k / G][cc] = 0.0;
            }
            cs[k / G] = bv[k / G];
            bv[k / G] = 0.0;
        }
    }
}

// Numerical rank: leading k with |R_kk| > tol |R_11|.
template <int M>
__device__ __forceinline__ int num_rank(const double (&rd)[M], double tol)
{
    const double thr = tol * fabs(rd[0]);
    int rank = 0;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        ok = ok && (fabs(rd[k]) > thr);
        rank += ok ? 1 : 0;
    }
    return rank;
}

// Back substitution R_{1:r,1:r} y = c_{1:r} (c_k held by the owner lane of
// row k), y_k = 0 beyond the rank; y ends up in every lane of the group.
template <int M, int G, int RS>
__device__ __forceinline__ void back_solve(const double (&Rs)[RS][M], const double (&cs)[RS], const double (&rinv)[M],
                                           int rank, int g, double (&y)[M])
{
#pragma unroll
    for (int k = M - 1; k >= 0; --k) {
        double acc = cs[k / G];
#pragma unroll
        for (int j = k + 1; j < M; ++j) acc = fma(-Rs[k / G][j], y[j], acc);
        const double yk = group_bcast<G>(acc, k % G, g) * rinv[k];
        y[k] = (k < rank) ? yk : 0.0;
    }
}

// --------------------------------------------------------------- K1
// Reconstruction of one cell by a group of G lanes (g = lane in the group),
// component by component (V = 1, or DIM + 2 conserved variables for Euler).
// Threads per workgroup of the per-cell kernels: one wavefront in 2-D, so
// that a small mesh's few waves spread over all CUs instead of filling a
// fraction of them four at a time (19.6 k triangles: 9.1 against 10.2 us per
// launch); four in 3-D (64 measured 2% slower).
constexpr int recon_block(int dim) { return dim == 3 ? 256 : 64; }

// BAL: scalar fluxes, also store each cell's gradient for the balanced-stencil
// refit (a variant of its own, so that the plain kernels carry none of it).
template <int DIM, int P, int G, int RPL, int FLUX, bool BAL = false>
__device__ __forceinline__ void reconstruct_cell(const RArgs &a, int64_t cell, int64_t cell_begin, int64_t cell_end,
                                                 const int32_t *spad, int stride, int g, double *lds, int slot)
{
    constexpr Basis<DIM, P> B{};
    constexpr int M = Basis<DIM, P>::M;
    constexpr int F = DIM + 1;
    constexpr int Q = num_q<DIM, P>();
    constexpr int NMOM = M - 1 - DIM;
    constexpr int GS = geo_stride<DIM, P>();
    constexpr int RS = (M + G - 1) / G;
    constexpr bool CHAR = FLUX == kFluxEulerChar;
    constexpr bool EULER = FLUX == kFluxEuler || CHAR;
    static_assert(!CHAR || DIM == 2, "characteristic fields: 2-D only");
    constexpr int V = EULER ? DIM + 2 : 1;
    // solves per cell: one per component, or (characteristic) one per field and facet
    constexpr int NIT = CHAR ? V * F : V;
    constexpr int CPB = recon_block(DIM) / G;

    const bool live = cell < cell_end;
    const int64_t c = live ? cell : cell_end - 1;
    const int32_t *srow = spad + (c - cell_begin) * stride;
    const int64_t N = a.nc;
    const int32_t mesh = a.mid ? a.mid[c] : 0;
    const double eh2 = a.eh2_cell ? a.eh2_cell[c] : (a.mid ? a.eh2_tab[mesh] : a.eh2);

    const double *gc = a.geo + c * GS;
    double xc[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) xc[d] = gc[d];
    // 1-D and 2-D: the end points of this lane's facets, relative to the
    // centroid (1-D: the facet point itself; 2-D: the edge's two vertices).
    // With one facet per lane they are loaded up front, so that their latency
    // overlaps the gather; with more, at the evaluation (registers).
    constexpr int FPL = (F + G - 1) / G;   // facets per lane (lane g: g, g+G, ...)
    constexpr bool kEarly = FPL == 1;
    double ea[FPL][DIM], eb[FPL][DIM];
    auto load_ends = [&](int t) {
        const int lf = g + t * G < F ? g + t * G : F - 1;
        const int ia = DIM == 1 ? (lf == 0 ? 1 : 0) : (lf == 2 ? 0 : lf + 1);
        const int ib = DIM == 1 ? ia : (lf == 0 ? 2 : lf - 1);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            ea[t][d] = a.vrel[(c * F + ia) * DIM + d];
            eb[t][d] = a.vrel[(c * F + ib) * DIM + d];
        }
    };
    if constexpr (DIM < 3 && kEarly) load_ends(0);
    // Loads run unconditionally (indices clamped into the cell's own records)
    // so that every load of a phase is in flight at once: first the facet
    // siblings and stencil ids, then the neighbours' averages and geometry.
    int32_t sb[F];
#pragma unroll
    for (int lf = 0; lf < F; ++lf) sb[lf] = a.sib[lf * N + c];
    int32_t jid[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int r = s * G + g;
        jid[s] = srow[r < stride ? r : stride - 1];
    }
    int32_t jrow[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int r = s * G + g;
        jrow[s] = (live && r < stride && jid[s] >= 0) ? jid[s] : -1;
    }
    // Burgers: sum of the unit normal's components; Euler: the area-scaled
    // normal, on this lane's facets (for the Lax-Friedrichs alpha bound)
    double nsm[FPL];
    double nrm[EULER ? FPL : 1][DIM];
#pragma unroll
    for (int t = 0; t < FPL; ++t) {
        const int lf = g + t * G < F ? g + t * G : F - 1;
        if constexpr (FLUX == kFluxBurgers) nsm[t] = a.nsum[lf * N + c];
        if constexpr (EULER) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) nrm[t][d] = a.normal[(lf * N + c) * DIM + d];
        }
    }
    double *lfv = lds + (CPB * M) + slot * (V * F * Q);   // systems: this cell's facet values, [V][F][Q]
    double am = 0.0;   // Lax-Friedrichs alpha bound over this lane's facet points
    const bool user = live && (a.fv_user || a.rank_user || a.coef_user);
    const int64_t uid = user ? (int64_t)a.perm[c] : 0;

    int rkm = 0;   // characteristic: smallest rank of a field over the facets
#pragma unroll 1
    for (int it = 0; it < NIT; ++it) {
    // component v, or (characteristic) field v of facet fl
    const int v = CHAR ? it / F : it;
    const int fl = CHAR ? it - v * F : 0;
    double Lr[4], Rc[4];
    if constexpr (CHAR) char_vectors(a.u, a.normal, a.sib, N, c, fl, v, a.gamma, Lr, Rc);
    auto field = [&](int64_t j) -> double {
        if constexpr (CHAR) {
            double t = Lr[0] * a.u[j];
#pragma unroll
            for (int k = 1; k < V; ++k) t = fma(Lr[k], a.u[(int64_t)k * N + j], t);
            return t;
        } else {
            return a.u[(int64_t)v * N + j];
        }
    };
    const double uc = field(c);
    double unb[F];
#pragma unroll
    for (int lf = 0; lf < F; ++lf) unb[lf] = field(sb[lf] >= 0 ? (sb[lf] >> 2) : c);
    double ug[RPL], gx[RPL][DIM + NMOM];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int64_t j = jrow[s] >= 0 ? (int64_t)jrow[s] : c;
        ug[s] = field(j);
#pragma unroll
        for (int t = 0; t < DIM + NMOM; ++t) gx[s][t] = a.geo[j * GS + t];
    }

    // indicator of the centre: smallest over its facet neighbours
    double bmin = -1.0;
#pragma unroll
    for (int lf = 0; lf < F; ++lf) {
        const double du = unb[lf] - uc;
        const double bt = du * du + eh2;
        bmin = (sb[lf] >= 0 && (bmin < 0.0 || bt < bmin)) ? bt : bmin;
    }
    bmin = bmin < 0.0 ? eh2 : bmin;

    // centroid offsets in place of the centroids; on a periodic mesh, to the
    // nearest image (a branch the whole wave takes or skips)
#pragma unroll
    for (int s = 0; s < RPL; ++s)
#pragma unroll
        for (int d = 0; d < DIM; ++d) gx[s][d] -= xc[d];
    if constexpr (DIM <= 2) {
        if (a.period > 0.0 || a.period_y > 0.0) {
#pragma unroll
            for (int s = 0; s < RPL; ++s)
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    const double L = d == 0 ? a.period : a.period_y;
                    const double x = gx[s][d];
                    if (L > 0.0) gx[s][d] = x > 0.5 * L ? x - L : (x < -0.5 * L ? x + L : x);
                }
        }
    }

    // weighted rows  W A  and  W u
    double A[RPL][M], bv[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int r = s * G + g;
        const bool valid = jrow[s] >= 0;
        double dl[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) dl[d] = gx[s][d];
        const double uj = ug[s];
        double row[M];
        taylor_row<DIM, P>(dl, gx[s] + DIM, row);
        double w = 1.0;
        if (a.weight_mode == 0) {
            const double du = uj - uc;
            const double num = (r == 0) ? a.alpha_w : 1.0;
            const double den = (r == 0) ? bmin : du * du + eh2;
            w = num * rcp_nr(den);
        }
        w = valid ? w : 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) A[s][k] = w * row[k];
        bv[s] = w * uj;
    }

    double sc[M];
    scale_columns<M, G, RPL>(A, sc);
    int pm[M];
    double rd[M], rinv[M];
    double Rs[RS][M], cs[RS];
    qrcp<M, G, RPL, RS>(A, bv, sc, g, pm, rd, rinv, Rs, cs);

    // numerical rank and back substitution on the leading r x r block
    const int rank = num_rank<M>(rd, a.rank_tol);
    double y[M];
    back_solve<M, G, RS>(Rs, cs, rinv, rank, g, y);

    // coefficients in the original basis order, v = S E y, through LDS: lane g
    // stores the entries k = g, g+G, ... at their original positions
    double *lc = lds + slot * M;
#pragma unroll
    for (int k = 0; k < M; ++k)
        if ((k % G) == g) lc[pm[k]] = sc[k] * y[k];
    // the G lanes of a cell are in one wavefront, whose LDS accesses complete
    // in order: a wavefront-scope fence suffices
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double coef[M];
#pragma unroll
    for (int o = 0; o < M; ++o) coef[o] = lc[o];
    if constexpr (CHAR) {
        rkm = fl == 0 ? rank : min(rkm, rank);
        if (live && a.rank_user && g == 0 && fl == F - 1) a.rank_user[(int64_t)v * N + uid] = rkm;
        // facet fl only, by the lane that holds its values: field v at its
        // points, mapped back with column v of R and summed over the fields
        if (g == fl % G) {
            const int ia = fl == 2 ? 0 : fl + 1, ib = fl == 0 ? 2 : fl - 1;
            double pa[DIM], pb[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                pa[d] = a.vrel[(c * F + ia) * DIM + d];
                pb[d] = a.vrel[(c * F + ib) * DIM + d];
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                double x[DIM];
                edge_point<DIM, Q>(pa, pb, q, x);
                double pw[DIM][P];
                scaled_powers<DIM, P>(x, pw);
                double val = 0.0;
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    double ph = coef[k];
#pragma unroll
                    for (int d = 0; d < DIM; ++d) ph *= pw[d][B.e[k][d]];
                    val += ph;
                }
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    double *dst = lfv + (k * F + fl) * Q + q;
                    *dst = v == 0 ? Rc[k] * val : fma(Rc[k], val, *dst);
                }
            }
        }
    } else {
    if (live && a.rank_user && g == 0) a.rank_user[(int64_t)v * N + uid] = rank;

    // evaluate at the facet points: lane g handles facets g, g+G, ...
#pragma unroll
    for (int t = 0; t < FPL; ++t) {
        const int lf0 = g + t * G;
        if (FPL * G > F && lf0 >= F) break;   // lanes beyond the last facet
        const int lf = lf0 < F ? lf0 : 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double x[DIM];
            if constexpr (DIM < 3 && !kEarly) {
                if (q == 0) load_ends(t);
            }
            if constexpr (DIM < 3)
                edge_point<DIM, Q>(ea[t], eb[t], q, x);
            else
                facet_point<DIM, Q>(a.vrel + c * F * DIM, lf, q, x);
            double pw[DIM][P];
            scaled_powers<DIM, P>(x, pw);
            double val = 0.0;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                double ph = coef[k];
#pragma unroll
                for (int d = 0; d < DIM; ++d) ph *= pw[d][B.e[k][d]];
                val += ph;
            }
            if constexpr (V == 1) {
                // scalar: straight out, with the Burgers alpha bound
                if (live) {
                    a.fv[(lf * N + c) * Q + q] = val;
                    if (a.fv_user) a.fv_user[(uid * F + lf) * Q + q] = val;
                    if constexpr (FLUX == kFluxBurgers) am = fmax(am, fabs(val * nsm[t]));
                }
            } else {
                lfv[(v * F + lf) * Q + q] = val;
            }
        }
    }
    if (live && a.coef_user) {
#pragma unroll
        for (int o = 0; o < M; ++o)
            if ((o % G) == g) a.coef_user[((int64_t)v * N + uid) * M + o] = coef[o];
    }
    if constexpr (V == 1 && BAL) {
        // balanced-stencil refit: the first fit's gradient, for the cells the
        // range check will list
        if (live && g == 0) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) a.bal_grad[c * DIM + d] = coef[1 + d];
        }
    }
    }   // component-wise evaluation
    }   // solves

    if constexpr (V > 1) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // Euler: keep the cell averages at every facet point when any facet
    // state of the reconstruction has non-positive density or pressure
    bool fallback = false;
    {
        double bad = 0.0;
#pragma unroll
        for (int t = 0; t < FPL; ++t) {
            const int lf0 = g + t * G;
            if (FPL * G > F && lf0 >= F) break;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                double U[V];
#pragma unroll
                for (int v = 0; v < V; ++v) U[v] = lfv[(v * F + lf0) * Q + q];
                double ke = 0.0;
#pragma unroll
                for (int d = 0; d < DIM; ++d) ke += U[1 + d] * U[1 + d];
                ke = 0.5 * ke / U[0];
                const double pr = (a.gamma - 1.0) * (U[DIM + 1] - ke);
                bad = (U[0] > 0.0 && pr > 0.0) ? bad : 1.0;
            }
        }
        fallback = group_sum<G>(bad) > 0.0;
    }

    // facet values out, Lax-Friedrichs alpha bound over this lane's points
#pragma unroll
    for (int t = 0; t < FPL; ++t) {
        const int lf0 = g + t * G;
        if (FPL * G > F && lf0 >= F) break;
        const int lf = lf0 < F ? lf0 : 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double U[V];
#pragma unroll
            for (int v = 0; v < V; ++v) U[v] = fallback ? a.u[(int64_t)v * N + c] : lfv[(v * F + lf) * Q + q];
            if (live) {
#pragma unroll
                for (int v = 0; v < V; ++v) a.fv[((v * F + lf) * N + c) * Q + q] = U[v];
                if (a.fv_user) {
#pragma unroll
                    for (int v = 0; v < V; ++v) a.fv_user[(((int64_t)v * N + uid) * F + lf) * Q + q] = U[v];
                }
                if constexpr (EULER) {
                    // |v.n| + c with the unit normal n = m / |m|
                    double mn = 0.0, mm = 0.0;
#pragma unroll
                    for (int d = 0; d < DIM; ++d) {
                        mn += U[1 + d] * nrm[t][d];
                        mm += nrm[t][d] * nrm[t][d];
                    }
                    double ke = 0.0;
#pragma unroll
                    for (int d = 0; d < DIM; ++d) ke += U[1 + d] * U[1 + d];
                    ke = 0.5 * ke / U[0];
                    const double pr = (a.gamma - 1.0) * (U[DIM + 1] - ke);
                    const double sr = fabs(mn / U[0]) / sqrt(mm) + sqrt(a.gamma * pr / U[0]);
                    am = fmax(am, sr);   // fmax ignores a NaN bound
                }
            }
        }
    }
    if (!CHAR && live && a.coef_user && fallback) {
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int o = 0; o < M; ++o)
                if ((o % G) == g)
                    a.coef_user[((int64_t)v * N + uid) * M + o] = o == 0 ? a.u[(int64_t)v * N + c] : 0.0;
    }
    }   // systems

    if constexpr (FLUX != kFluxAdv) {
        // global Lax-Friedrichs alpha of the cell's mesh: the wave maximum into
        // one of the mesh's slots; a wave that spans meshes (batches, at mesh
        // boundaries) posts lane by lane
        const int wv = (int)((blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) % a.spm);
        const int m0 = __builtin_amdgcn_readfirstlane(mesh);
        if (__ballot(mesh != m0) == 0) {
            am = wave_max(am);
            if ((threadIdx.x & 63) == 0)
                atomicMax(a.alpha_acc + ((int64_t)m0 * a.spm + wv) * 16, (unsigned long long)__double_as_longlong(am));
        } else if (am > 0.0) {
            atomicMax(a.alpha_acc + ((int64_t)mesh * a.spm + wv) * 16, (unsigned long long)__double_as_longlong(am));
        }
    }
}

// LDS of a reconstruction workgroup: per cell M coefficients; for the Euler
// system also its facet values [V][F][Q].
template <int DIM, int P, int FLUX, int G>
constexpr int recon_lds()
{
    return (recon_block(DIM) / G) *
           (Basis<DIM, P>::M +
            (FLUX == kFluxEuler || FLUX == kFluxEulerChar ? (DIM + 2) * (DIM + 1) * num_q<DIM, P>() : 0));
}

// Logical workgroup L of the reconstruction: 256/G (3-D) or 64/G (1-D, 2-D)
// cells of one stencil-size bucket, G lanes per cell.
template <int DIM, int P, int FLUX, int G, int R0, int R1, int R2, bool BAL = false>
__device__ __forceinline__ void reconstruct_block(const RArgs &a, int L, double *lds)
{
    constexpr int CPB = recon_block(DIM) / G;   // cells per workgroup
    const int g = (int)(threadIdx.x % G);
    const int slot = (int)(threadIdx.x / G);
    if (L < a.blk0[1]) {
        const int64_t cell = a.cell0[0] + (int64_t)(L - a.blk0[0]) * CPB + slot;
        reconstruct_cell<DIM, P, G, R0, FLUX, BAL>(a, cell, a.cell0[0], a.cell0[1], a.spad + a.spad_off[0], a.stride[0], g,
                                              lds, slot);
    } else if (L < a.blk0[2]) {
        const int64_t cell = a.cell0[1] + (int64_t)(L - a.blk0[1]) * CPB + slot;
        reconstruct_cell<DIM, P, G, R1, FLUX, BAL>(a, cell, a.cell0[1], a.cell0[2], a.spad + a.spad_off[1], a.stride[1], g,
                                              lds, slot);
    } else {
        const int64_t cell = a.cell0[2] + (int64_t)(L - a.blk0[2]) * CPB + slot;
        reconstruct_cell<DIM, P, G, R2, FLUX, BAL>(a, cell, a.cell0[2], a.cell0[3], a.spad + a.spad_off[2], a.stride[2], g,
                                              lds, slot);
    }
}

template <int DIM, int P, int FLUX, int G, int R0, int R1, int R2, bool BAL = false>
__global__ void __launch_bounds__(recon_block(DIM)) k_reconstruct(RArgs a)
{
    __shared__ double lds[recon_lds<DIM, P, FLUX, G>()];
    reconstruct_block<DIM, P, FLUX, G, R0, R1, R2, BAL>(a, xcd_block((int)blockIdx.x, (int)gridDim.x), lds);
}

// Balanced-stencil refit (end of Sec. 3.2) of the cells listed by
// k_reconstruct: from each cell's enlarged stencil (centre first, then by
// distance) keep the centroid and the nearest cells on both sides of the
// line/plane through it orthogonal to the first fit's gradient,
// ceil((n-1)/2) with g.(x_j - x_i) > 0 and floor((n-1)/2) otherwise (a short
// side leaves its share to the other), and fit again.  Lane g of a cell
// classifies enlarged-stencil entries g, g+G, ...; the sides are 128-bit
// masks in stencil order, OR-ed over the group, so the choice is a prefix
// count.
// Range check of the first fit (one thread per cell): a cell whose facet
// values leave [min, max] of its stencil's averages by more than a rounding
// band goes on the refit list; every other cell posts its Lax-Friedrichs alpha
// bound (the first fit posted into scratch slots, so that the refit's values,
// not the discarded ones, bound alpha).
struct FArgs {
    int64_t nc;
    const double *u, *fv, *nsum;
    const int32_t *sptr, *scol, *mid;
    unsigned long long *alpha_acc, *count;
    int32_t *list;
    int spm;
};

template <int DIM, int Q, int FLUX>
__global__ void __launch_bounds__(256) k_flag(FArgs a)
{
    constexpr int F = DIM + 1;
    const int64_t N = a.nc;
    const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool live = i0 < N;
    const int64_t c = live ? i0 : N - 1;
    double lo = a.u[c], hi = lo;
    // the stencil's averages in batches of 16 independent loads (clamped
    // indices repeat the centre), so that their latencies overlap
    const int32_t t0 = a.sptr[c], t1 = a.sptr[c + 1];
    for (int32_t tb = t0; tb < t1; tb += 16) {
        int32_t id[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) id[k] = tb + k < t1 ? a.scol[tb + k] : (int32_t)c;
        double v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = a.u[id[k]];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            lo = fmin(lo, v[k]);
            hi = fmax(hi, v[k]);
        }
    }
    double vlo = INFINITY, vhi = -INFINITY, am = 0.0;
#pragma unroll
    for (int lf = 0; lf < F; ++lf) {
        const double nsm = FLUX == kFluxBurgers ? a.nsum[lf * N + c] : 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double v = a.fv[(lf * N + c) * Q + q];
            vlo = fmin(vlo, v);
            vhi = fmax(vhi, v);
            am = fmax(am, fabs(v * nsm));
        }
    }
    const double band = 1e-10 * (hi - lo) + 1e-14 * fmax(fabs(hi), fabs(lo));
    if (live && (vhi > hi + band || vlo < lo - band)) {
        am = 0.0;   // the refit posts this cell's bound
        const unsigned long long k = atomicAdd(a.count, 1ull);
        if (k < (unsigned long long)N) a.list[k] = (int32_t)c;
    }
    if (!live) am = 0.0;
    if constexpr (FLUX == kFluxBurgers) {
        const int32_t mesh = a.mid ? a.mid[c] : 0;
        const int wv = (int)((blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) % a.spm);
        const int m0 = __builtin_amdgcn_readfirstlane(mesh);
        if (__ballot(mesh != m0) == 0) {
            am = wave_max(am);
            if ((threadIdx.x & 63) == 0)
                atomicMax(a.alpha_acc + ((int64_t)m0 * a.spm + wv) * 16, (unsigned long long)__double_as_longlong(am));
        } else if (am > 0.0) {
            atomicMax(a.alpha_acc + ((int64_t)mesh * a.spm + wv) * 16, (unsigned long long)__double_as_longlong(am));
        }
    }
}

struct BArgs {
    const unsigned long long *count;
    const int32_t *list, *pool, *sptr;
    const double *grad;
    int pool_cap;
};

__device__ __forceinline__ unsigned long long lowest_bits(unsigned long long x, int k)
{
    unsigned long long y = 0ull;
    for (int t = 0; t < k && x; ++t) {
        const unsigned long long low = x & (~x + 1ull);
        y |= low;
        x ^= low;
    }
    return y;
}

template <int DIM, int P, int FLUX, int G, int RPL>
__global__ void __launch_bounds__(recon_block(DIM)) k_rebalance(RArgs a, BArgs b)
{
    constexpr int CPB = recon_block(DIM) / G;
    constexpr int GS = geo_stride<DIM, P>();
    __shared__ double lds[CPB * Basis<DIM, P>::M];
    __shared__ int32_t rows[CPB][RPL * G];
    const int g = (int)(threadIdx.x % G);
    const int slot = (int)(threadIdx.x / G);
    const int64_t total = (int64_t)*b.count;
    const int64_t cnt = total < a.nc ? total : a.nc;
    // whole wavefronts past the end of the list leave at once
    const int64_t first = (int64_t)blockIdx.x * CPB + (int64_t)(threadIdx.x / 64) * (64 / G);
    if (first >= cnt) return;
    const int64_t idx = (int64_t)blockIdx.x * CPB + slot;
    const bool live = idx < cnt;
    const int64_t c = b.list[live ? idx : cnt - 1];
    double gr[DIM], xc[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        gr[d] = b.grad[c * DIM + d];
        xc[d] = a.geo[c * GS + d];
    }
    const int32_t *pool = b.pool + c * b.pool_cap;
    unsigned long long mp[2] = {0ull, 0ull}, mm[2] = {0ull, 0ull};
    // entries g, g+G, ... in batches of 8 independent loads (clamped to the
    // centre), so that their latencies overlap
    for (int rb = g; rb < b.pool_cap; rb += 8 * G) {
        int32_t jj[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int r = rb + k * G;
            jj[k] = r < b.pool_cap ? pool[r] : -1;
        }
        double gx[8][DIM];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int64_t j = jj[k] >= 0 ? (int64_t)jj[k] : c;
#pragma unroll
            for (int d = 0; d < DIM; ++d) gx[k][d] = a.geo[j * GS + d];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int r = rb + k * G;
            if (r == 0 || jj[k] < 0) continue;   // the centre; padding or past the end
            double dl[DIM];
            centroid_offset<DIM>(gx[k], xc, a.period, a.period_y, dl);
            double sd = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) sd += gr[d] * dl[d];
            const unsigned long long bit = 1ull << (r & 63);
            if (sd > 0.0)
                mp[r >> 6] |= bit;
            else
                mm[r >> 6] |= bit;
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        mp[h] = group_or<G>(mp[h]);
        mm[h] = group_or<G>(mm[h]);
    }
    const int cp = __popcll(mp[0]) + __popcll(mp[1]);
    const int cm = __popcll(mm[0]) + __popcll(mm[1]);
    const int n = b.sptr[c + 1] - b.sptr[c];
    int qp = n / 2, qm = (n - 1) / 2;
    if (cp < qp) {
        qm += qp - cp;
        qp = cp;
    }
    if (cm < qm) {
        qp += qm - cm;
        qm = cm;
    }
    unsigned long long acc[2];
    {
        const int p0 = __popcll(mp[0]) < qp ? __popcll(mp[0]) : qp;
        const int m0 = __popcll(mm[0]) < qm ? __popcll(mm[0]) : qm;
        acc[0] = lowest_bits(mp[0], p0) | lowest_bits(mm[0], m0);
        acc[1] = lowest_bits(mp[1], qp - p0) | lowest_bits(mm[1], qm - m0);
    }
    const int n2 = 1 + __popcll(acc[0]) + __popcll(acc[1]);
    int32_t *rw = rows[slot];
    if (g == 0) rw[0] = (int32_t)c;
    for (int r = g; r < b.pool_cap; r += G) {
        const unsigned long long w = acc[r >> 6];
        if ((w >> (r & 63)) & 1ull) {
            const int below = (r >= 64 ? __popcll(acc[0]) : 0) + __popcll(w & ((1ull << (r & 63)) - 1ull));
            rw[1 + below] = pool[r];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // cell range [c, c + 1): a lane past the end of the list passes c + 1, which
    // reconstruct_cell clamps back to c (a listed cell), and stores nothing
    reconstruct_cell<DIM, P, G, RPL, FLUX>(a, live ? c : c + 1, c, c + 1, rw, n2, g, lds, slot);
}

// ------------------------------------------------------------ adjoint
// Transposed Jacobian of the advection right-hand side, v -> J(u)^T v, in two
// kernels: k_adjoint writes, per cell i, the contribution of (dL/du)^T v
// through cell i's reconstruction to every cell its stencil reads (one value
// per stencil slot, one per facet slot for the centre weight's
// smallest-indicator neighbour), each into the receiving cell's contiguous
// segment; k_adjoint_gather sums every segment in a fixed order.

struct AArgs {
    int64_t nc, npad;
    const double *u, *v;               // state and cotangent of L(u), device order
    const double *geo, *vrel, *normal, *rvol;
    const int32_t *spad, *sib;
    double *contrib;                   // contributions, in transposed-stencil order
    const int32_t *tpos;               // position in contrib of each padded slot, then of each facet slot
    double eh2, alpha_w, rank_tol, period, period_y;
    int weight_mode, bc;
    double vel[3];
    int64_t cell0[kMaxBuckets + 1];
    int blk0[kMaxBuckets + 1];
    int64_t spad_off[kMaxBuckets + 1];
    int stride[kMaxBuckets];
};

template <int DIM, int P, int G, int RPL>
__device__ __forceinline__ void adjoint_cell(const AArgs &a, int64_t cell, int64_t cell_begin, int64_t cell_end,
                                             int64_t pad_off, int stride, int g, double *lds, int slot)
{
    constexpr Basis<DIM, P> B{};
    constexpr int M = Basis<DIM, P>::M;
    constexpr int F = DIM + 1;
    constexpr int Q = num_q<DIM, P>();
    constexpr int GS = geo_stride<DIM, P>();
    constexpr int RS = (M + G - 1) / G;
    constexpr int FPL = (F + G - 1) / G;
    constexpr int CPB = 256 / G;

    const bool live = cell < cell_end;
    const int64_t c = live ? cell : cell_end - 1;
    const int32_t *srow = a.spad + pad_off + (c - cell_begin) * stride;
    const int64_t N = a.nc;
    const double eh2 = a.eh2;

    double xc[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) xc[d] = a.geo[c * GS + d];
    const double uc = a.u[c];
    int32_t sb[F];
#pragma unroll
    for (int lf = 0; lf < F; ++lf) sb[lf] = a.sib[lf * N + c];
    int32_t jrow[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int r = s * G + g;
        const int32_t j = srow[r < stride ? r : stride - 1];
        jrow[s] = (live && r < stride && j >= 0) ? j : -1;
    }
    // centre indicator: smallest over the facet neighbours (first one on ties)
    double bmin = -1.0, unbmin = uc;
    int lfmin = -1;
#pragma unroll
    for (int lf = 0; lf < F; ++lf) {
        const double un = a.u[sb[lf] >= 0 ? (sb[lf] >> 2) : c];
        const double du = un - uc;
        const double bt = du * du + eh2;
        const bool take = sb[lf] >= 0 && (bmin < 0.0 || bt < bmin);
        bmin = take ? bt : bmin;
        unbmin = take ? un : unbmin;
        lfmin = take ? lf : lfmin;
    }
    bmin = bmin < 0.0 ? eh2 : bmin;

    // the forward solve again: weighted rows, scaling, QRCP, coefficients
    double A[RPL][M], bv[RPL], wt[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int r = s * G + g;
        const int64_t j = jrow[s] >= 0 ? (int64_t)jrow[s] : c;
        double dl[DIM];
        centroid_offset<DIM>(a.geo + j * GS, xc, a.period, a.period_y, dl);
        double row[M];
        taylor_row<DIM, P>(dl, a.geo + j * GS + DIM, row);
        const double uj = a.u[j];
        double w = 1.0;
        if (a.weight_mode == 0) {
            const double du = uj - uc;
            const double num = (r == 0) ? a.alpha_w : 1.0;
            const double den = (r == 0) ? bmin : du * du + eh2;
            w = num * rcp_nr(den);
        }
        w = jrow[s] >= 0 ? w : 0.0;
        wt[s] = w;
#pragma unroll
        for (int k = 0; k < M; ++k) A[s][k] = w * row[k];
        bv[s] = w * uj;
    }
    double sc[M];
    scale_columns<M, G, RPL>(A, sc);
    int pm[M];
    double rd[M], rinv[M];
    double Rs[RS][M], cs[RS];
    qrcp<M, G, RPL, RS>(A, bv, sc, g, pm, rd, rinv, Rs, cs);
    const int rank = num_rank<M>(rd, a.rank_tol);
    double y[M];
    back_solve<M, G, RS>(Rs, cs, rinv, rank, g, y);
    double *lc = lds + slot * M;            // coefficients, then lambda
    double *lg = lds + (CPB + slot) * M;    // cotangent of the coefficients
#pragma unroll
    for (int k = 0; k < M; ++k)
        if ((k % G) == g) lc[pm[k]] = sc[k] * y[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double coef[M];
#pragma unroll
    for (int o = 0; o < M; ++o) coef[o] = lc[o];

    // cotangent of this cell's facet values: facet point value a enters its
    // own cell's L with -rvol_i w_q dF/da and the neighbour's with
    // +rvol_j w_q dF/da (upwind flux with the area-scaled normal m)
    const double vi = a.v[c], rvi = a.rvol[c];
    double gco[M];
#pragma unroll
    for (int k = 0; k < M; ++k) gco[k] = 0.0;
#pragma unroll
    for (int t = 0; t < FPL; ++t) {
        const int lf0 = g + t * G;
        const bool has = lf0 < F;
        const int lf = has ? lf0 : 0;
        const int32_t sj = sb[lf];
        double am = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) am += a.vel[d] * a.normal[(lf * N + c) * DIM + d];
        const int64_t jn = sj >= 0 ? (int64_t)(sj >> 2) : c;   // clamped: loads stay in bounds
        const double vj = sj >= 0 ? a.v[jn] : 0.0;
        const double rvj = sj >= 0 ? a.rvol[jn] : 0.0;
        // boundary: F = am a (transmissive) or 1/2 (am + |am|) a (zero outside state)
        const double dfb = a.bc ? 0.5 * (am + fabs(am)) : am;
        const double coefa = sj >= 0 ? 0.5 * (am + fabs(am)) * (rvj * vj - rvi * vi) : -rvi * vi * dfb;
        double ea[DIM], eb[DIM];
        if constexpr (DIM < 3) {
            const int ia = DIM == 1 ? (lf == 0 ? 1 : 0) : (lf == 2 ? 0 : lf + 1);
            const int ib = DIM == 1 ? ia : (lf == 0 ? 2 : lf - 1);
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                ea[d] = a.vrel[(c * F + ia) * DIM + d];
                eb[d] = a.vrel[(c * F + ib) * DIM + d];
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double x[DIM];
            if constexpr (DIM < 3)
                edge_point<DIM, Q>(ea, eb, q, x);
            else
                facet_point<DIM, Q>(a.vrel + c * F * DIM, lf, q, x);
            double pw[DIM][P];
            scaled_powers<DIM, P>(x, pw);
            const double ga = (has && live) ? quad_weight<DIM, Q>(q) * coefa : 0.0;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                double ph = ga;
#pragma unroll
                for (int d = 0; d < DIM; ++d) ph *= pw[d][B.e[k][d]];
                gco[k] += ph;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < M; ++k) gco[k] = group_sum<G>(gco[k]);

    // lambda = S E_r (R^T R)^-1 E_r^T S gco on the leading rank columns:
    // forward substitution R^T z = E^T S gco, then R l = z
    if (g == 0) {
#pragma unroll
        for (int o = 0; o < M; ++o) lg[o] = gco[o];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double z[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < k; ++j) t += (g == (j % G)) ? Rs[j / G][k] * z[j] : 0.0;
        t = group_sum<G>(t);
        const double gy = sc[k] * lg[pm[k]];
        z[k] = (k < rank) ? (gy - t) * rinv[k] : 0.0;
    }
    double lam[M];
#pragma unroll
    for (int k = M - 1; k >= 0; --k) {
        double acc = z[k];
#pragma unroll
        for (int j = k + 1; j < M; ++j) acc = fma(-Rs[k / G][j], lam[j], acc);
        const double lk = group_bcast<G>(acc, k % G, g) * rinv[k];
        lam[k] = (k < rank) ? lk : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < M; ++k)
        if ((k % G) == g) lc[pm[k]] = sc[k] * lam[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double lo[M];
#pragma unroll
    for (int o = 0; o < M; ++o) lo[o] = lc[o];

    // contributions: b = W u_S gives W^2 A lambda; the weights give
    // 2 w (A lambda) (u_S - A v) through d w / d u
    double to_c = 0.0, to_nb = 0.0;
    double slotv[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int r = s * G + g;
        const bool valid = jrow[s] >= 0;
        const int64_t j = valid ? (int64_t)jrow[s] : c;
        double dl[DIM];
        centroid_offset<DIM>(a.geo + j * GS, xc, a.period, a.period_y, dl);
        double row[M];
        taylor_row<DIM, P>(dl, a.geo + j * GS + DIM, row);
        const double uj = a.u[j];
        double al = 0.0, av = 0.0;
#pragma unroll
        for (int o = 0; o < M; ++o) {
            al = fma(row[o], lo[o], al);
            av = fma(row[o], coef[o], av);
        }
        const double w = wt[s];
        const double bbar = w * w * al;
        const double wbar = 2.0 * w * al * (uj - av);
        double own = bbar;
        if (a.weight_mode == 0 && valid) {
            if (r == 0) {
                // w_0 = alpha_w / beta_min, beta_min = (u_nb - u_i)^2 + eps h^2
                const double d = lfmin >= 0 ? 2.0 * (unbmin - uc) : 0.0;
                const double dw = -w * w / a.alpha_w;   // d w_0 / d beta
                to_nb += wbar * dw * d;
                to_c -= wbar * dw * d;
            } else {
                // w_r = 1 / beta_r, beta_r = (u_j - u_i)^2 + eps h^2
                const double d = 2.0 * (uj - uc);
                own += wbar * (-w * w) * d;
                to_c += wbar * (w * w) * d;
            }
        }
        slotv[s] = valid ? own : 0.0;
    }
    to_c = group_sum<G>(to_c);
    to_nb = group_sum<G>(to_nb);
    if (live) {
        // each slot that reads a cell has a place in that cell's contiguous
        // segment of contrib (tpos < 0: padding, or a boundary facet)
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            const int r = s * G + g;
            if (r < stride) {
                const int32_t t = a.tpos[pad_off + (c - cell_begin) * stride + r];
                if (t >= 0) a.contrib[t] = slotv[s] + (r == 0 ? to_c : 0.0);
            }
        }
        if (g == 0) {
#pragma unroll
            for (int lf = 0; lf < F; ++lf) {
                const int32_t t = a.tpos[a.npad + lf * N + c];
                if (t >= 0) a.contrib[t] = lf == lfmin ? to_nb : 0.0;
            }
        }
    }
}

template <int DIM, int P, int G, int R0, int R1, int R2>
__global__ void __launch_bounds__(256) k_adjoint(AArgs a)
{
    constexpr int CPB = 256 / G;
    __shared__ double lds[2 * CPB * Basis<DIM, P>::M];
    const int L = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int g = (int)(threadIdx.x % G);
    const int slot = (int)(threadIdx.x / G);
    if (L < a.blk0[1]) {
        const int64_t cell = a.cell0[0] + (int64_t)(L - a.blk0[0]) * CPB + slot;
        adjoint_cell<DIM, P, G, R0>(a, cell, a.cell0[0], a.cell0[1], a.spad_off[0], a.stride[0], g, lds, slot);
    } else if (L < a.blk0[2]) {
        const int64_t cell = a.cell0[1] + (int64_t)(L - a.blk0[1]) * CPB + slot;
        adjoint_cell<DIM, P, G, R1>(a, cell, a.cell0[1], a.cell0[2], a.spad_off[1], a.stride[1], g, lds, slot);
    } else {
        const int64_t cell = a.cell0[2] + (int64_t)(L - a.blk0[2]) * CPB + slot;
        adjoint_cell<DIM, P, G, R2>(a, cell, a.cell0[2], a.cell0[3], a.spad_off[2], a.stride[2], g, lds, slot);
    }
}

// out = A x + B y + C z + D sum of cell j's segment of contrib, per cell j
// (device order, segments in increasing source order); null vectors count as zero.
__global__ void __launch_bounds__(256) k_adjoint_gather(int64_t nc, const int64_t *tptr, const double *contrib,
                                                        const double *x, const double *y, const double *z,
                                                        double *out, double A, double B, double C, double D)
{
    const int64_t j = (int64_t)xcd_block((int)blockIdx.x, (int)gridDim.x) * 256 + threadIdx.x;
    if (j >= nc) return;
    double s = 0.0;
    for (int64_t t = tptr[j]; t < tptr[j + 1]; ++t) s += contrib[t];
    double o = D * s;
    if (x) o += A * x[j];
    if (y) o += B * y[j];
    if (z) o += C * z[j];
    out[j] = o;
}

// --------------------------------------------------------------- K2/K3
struct UArgs {
    int64_t nc;
    const double *fv, *snormal, *rvol;    // snormal = |f| n, [F][N][DIM]
    const int32_t *sib, *qperm;
    const double *u0, *prev;
    double *out;
    const unsigned long long *alpha_rd;   // this stage's parity (nmesh x spm slots, stride 16)
    unsigned long long *alpha_clr;        // next stage's parity, cleared by block 0
    const int32_t *mid;                   // batches: mesh of each cell (else null)
    const double *dt_tab;                 // batches: time step per mesh (Cdt is then the coefficient)
    const double *dt_one;                 // one mesh: its time step, if Cdt is the coefficient (else null)
    int spm, nslot;                       // slots per mesh, slots per parity
    double A, B, Cdt;
    double vel[3];
    double gamma;
    int mode;
    int bc;
    int local_alpha;   // 1: Rusanov alpha per facet point
    double far[5];     // bc = 2: outside state
};

// Euler normal flux F(U).m for the area-scaled normal m (linear in m).
template <int DIM, int V>
__device__ __forceinline__ void euler_flux(const double (&U)[V], const double (&m)[DIM], double gamma, double (&f)[V])
{
    const double rho = U[0];
    double ke = 0.0, vm = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        ke += U[1 + d] * U[1 + d];
        vm += U[1 + d] / rho * m[d];
    }
    ke = 0.5 * ke / rho;
    const double pr = (gamma - 1.0) * (U[DIM + 1] - ke);
    f[0] = rho * vm;
#pragma unroll
    for (int d = 0; d < DIM; ++d) f[1 + d] = U[1 + d] * vm + pr * m[d];
    f[DIM + 1] = (U[DIM + 1] + pr) * vm;
}

// |f| times the Lax-Friedrichs flux for the area-scaled normal m = |f| n, for
// every component: out = 1/2 [(F(ua) + F(ub)).m - alpha |m| (ub - ua)], with
// alpha = |a.n| per facet for advection and the global bound otherwise.
template <int DIM, int FLUX, int V>
__device__ __forceinline__ void lf_flux(const double (&ua)[V], const double (&ub)[V], const double (&m)[DIM],
                                        double alpha, const double (&vel)[3], double gamma, double (&out)[V])
{
    if constexpr (FLUX == kFluxAdv) {
        double am = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) am += vel[d] * m[d];
        out[0] = 0.5 * ((am * ua[0] + am * ub[0]) - fabs(am) * (ub[0] - ua[0]));
    } else if constexpr (FLUX == kFluxBurgers) {
        double sm = 0.0, mm = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            sm += m[d];
            mm += m[d] * m[d];
        }
        const double af = alpha * sqrt(mm);
        out[0] = 0.5 * ((0.5 * ua[0] * ua[0] * sm + 0.5 * ub[0] * ub[0] * sm) - af * (ub[0] - ua[0]));
    } else {
        double mm = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) mm += m[d] * m[d];
        const double af = alpha * sqrt(mm);
        double fa[V], fb[V];
        euler_flux<DIM, V>(ua, m, gamma, fa);
        euler_flux<DIM, V>(ub, m, gamma, fb);
#pragma unroll
        for (int v = 0; v < V; ++v) out[v] = 0.5 * ((fa[v] + fb[v]) - af * (ub[v] - ua[v]));
    }
}

// Local (Rusanov) alpha at a facet point: the larger normal spectral radius of
// its two states, for the area-scaled normal m (per unit normal).
template <int DIM, int FLUX, int V>
__device__ __forceinline__ double point_alpha(const double (&ua)[V], const double (&ub)[V], const double (&m)[DIM],
                                              double gamma)
{
    double mm = 0.0, sm = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        mm += m[d] * m[d];
        sm += m[d];
    }
    const double im = 1.0 / sqrt(mm);
    if constexpr (FLUX == kFluxBurgers) {
        return fmax(fabs(ua[0] * sm), fabs(ub[0] * sm)) * im;
    } else {
        double r[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const double *U = side == 0 ? ua : ub;
            double vm = 0.0, ke = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                vm += U[1 + d] * m[d];
                ke += U[1 + d] * U[1 + d];
            }
            const double pr = (gamma - 1.0) * (U[DIM + 1] - 0.5 * ke / U[0]);
            r[side] = fabs(vm / U[0]) * im + sqrt(gamma * pr / U[0]);
        }
        return fmax(r[0], r[1]);
    }
}

// Logical workgroup lb of the flux/update: cells lb BS .. lb BS + BS - 1.
template <int DIM, int Q, int FLUX, int BS>
__device__ __forceinline__ void update_block(const UArgs &a, int lb)
{
    constexpr int F = DIM + 1;
    constexpr int V = FLUX == kFluxEuler ? DIM + 2 : 1;
    // 64-bit cell indices: [V][F][N][Q] offsets pass 2^32 well within 288 GB
    const int64_t N = a.nc;
    const int64_t c0 = (int64_t)lb * BS + threadIdx.x;
    const bool live = c0 < N;
    const int64_t c = live ? c0 : N - 1;   // lanes past the end work on the last cell, store nothing
    if constexpr (FLUX != kFluxAdv) {
        if (lb == 0)
            for (int t = (int)threadIdx.x; t < a.nslot; t += BS) a.alpha_clr[t * 16] = 0ull;
    }
    // every load is issued up front (indices clamped into this cell's own
    // records for boundary facets), then the fluxes are formed
    int32_t sb[F];
    double m[F][DIM];
#pragma unroll
    for (int lf = 0; lf < F; ++lf) {
        sb[lf] = a.sib[lf * N + c];
#pragma unroll
        for (int d = 0; d < DIM; ++d) m[lf][d] = a.snormal[(lf * N + c) * DIM + d];
    }
    const double rv = a.rvol[c];
    double alpha = 0.0;
    double cdt = a.Cdt;
    if (!a.mid && a.dt_one) cdt = a.Cdt * a.dt_one[0];
    if (a.mid) {
        const int32_t mesh = a.mid[c];
        cdt = a.Cdt * a.dt_tab[mesh];
        if constexpr (FLUX != kFluxAdv) {
            for (int t = 0; t < a.spm; ++t)
                alpha = fmax(alpha, __longlong_as_double((long long)a.alpha_rd[((int64_t)mesh * a.spm + t) * 16]));
        }
    } else if constexpr (FLUX != kFluxAdv) {
        // one mesh: its 64 slots, one per lane, reduced over the wave
        const double v = __longlong_as_double((long long)a.alpha_rd[(threadIdx.x & 63) * 16]);
        const double w = wave_max(v);
        alpha = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(w)),
                                 __builtin_amdgcn_readfirstlane(__double2loint(w)));
    }
    double own[V][F][Q], oth[V][F][Q];
    bool owner[F];
    int32_t qp[F];
#pragma unroll
    for (int lf = 0; lf < F; ++lf) {
        const bool inner = sb[lf] >= 0;
        const int64_t j = inner ? (int64_t)(sb[lf] >> 2) : c;
        const int l2 = inner ? (sb[lf] & 3) : lf;
        owner[lf] = c < j;
        qp[lf] = 0;
        if constexpr (DIM == 3) qp[lf] = inner ? (owner[lf] ? a.qperm[lf * N + c] : a.qperm[l2 * N + j]) : 0;
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                own[v][lf][q] = a.fv[((v * F + lf) * N + c) * Q + q];
                oth[v][lf][q] = a.fv[((v * F + l2) * N + j) * Q + q];
            }
    }
    double vel[3] = {a.vel[0], a.vel[1], a.vel[2]};
    double tot[V];
#pragma unroll
    for (int v = 0; v < V; ++v) tot[v] = 0.0;
#pragma unroll
    for (int lf = 0; lf < F; ++lf) {
        double facc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) facc[v] = 0.0;
        if (sb[lf] < 0) {
            // boundary: outside state = inside state (transmissive), zero, a
            // given far-field state, or (Euler) the inside state mirrored at a
            // slip wall: normal momentum reversed
            double mq = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) mq += m[lf][d] * m[lf][d];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                double uo[V], ux[V], fl[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    uo[v] = own[v][lf][q];
                    ux[v] = a.bc == 0 ? uo[v] : (a.bc == 2 ? a.far[v] : 0.0);
                }
                if constexpr (V > 1) {
                    if (a.bc == 3) {
                        double mn = 0.0;
#pragma unroll
                        for (int d = 0; d < DIM; ++d) mn += uo[1 + d] * m[lf][d];
                        const double s = 2.0 * mn / mq;
                        ux[0] = uo[0];
#pragma unroll
                        for (int d = 0; d < DIM; ++d) ux[1 + d] = uo[1 + d] - s * m[lf][d];
                        ux[DIM + 1] = uo[DIM + 1];
                    }
                }
                double al = alpha;
                if constexpr (FLUX != kFluxAdv) {
                    if (a.local_alpha) al = point_alpha<DIM, FLUX, V>(uo, ux, m[lf], a.gamma);
                }
                lf_flux<DIM, FLUX, V>(uo, ux, m[lf], al, vel, a.gamma, fl);
#pragma unroll
                for (int v = 0; v < V; ++v) facc[v] += quad_weight<DIM, Q>(q) * fl[v];
            }
        } else {
            // both cells evaluate the facet from identical operands in the
            // orientation of the lower-numbered cell; the other one negates
            const bool ow = owner[lf];
            double mm[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) mm[d] = ow ? m[lf][d] : -m[lf][d];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                // the sibling's point matching point q: reversed along an edge in 2-D
                const int qo = DIM == 3 ? ((qp[lf] >> (2 * q)) & 3) : (Q - 1 - q);
                double ua[V], ub[V], fl[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    // 3-D: qo is data, so select among the three points
                    double own_qo = own[v][lf][0], oth_q = oth[v][lf][0];
#pragma unroll
                    for (int t = 1; t < Q; ++t) {
                        own_qo = qo == t ? own[v][lf][t] : own_qo;
                    }
                    oth_q = oth[v][lf][q];
                    double oth_qo = oth[v][lf][0];
#pragma unroll
                    for (int t = 1; t < Q; ++t) oth_qo = qo == t ? oth[v][lf][t] : oth_qo;
                    ua[v] = ow ? own[v][lf][q] : oth_q;
                    ub[v] = ow ? oth_qo : own_qo;
                }
                double al = alpha;
                if constexpr (FLUX != kFluxAdv) {
                    if (a.local_alpha) al = point_alpha<DIM, FLUX, V>(ua, ub, mm, a.gamma);
                }
                lf_flux<DIM, FLUX, V>(ua, ub, mm, al, vel, a.gamma, fl);
#pragma unroll
                for (int v = 0; v < V; ++v) facc[v] += quad_weight<DIM, Q>(q) * fl[v];
            }
#pragma unroll
            for (int v = 0; v < V; ++v) facc[v] = ow ? facc[v] : -facc[v];
        }
#pragma unroll
        for (int v = 0; v < V; ++v) tot[v] += facc[v];
    }
    if (!live) return;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int64_t vc = v * N + c;
        const double L = -tot[v] * rv;
        a.out[vc] = a.mode == 0 ? L : a.A * a.u0[vc] + a.B * a.prev[vc] + cdt * L;
    }
}

template <int DIM, int Q, int FLUX, int BS>
__global__ void __launch_bounds__(BS) k_update(UArgs a)
{
    update_block<DIM, Q, FLUX, BS>(a, xcd_block((int)blockIdx.x, (int)gridDim.x));
}

// ---------------------------------------------------- persistent steps
// n TVD RK3 steps in one cooperative launch: every stage is a reconstruction
// phase, a device-wide barrier, a flux/update phase and another barrier, with
// the same logical workgroups, coefficients and alpha-slot parities as the
// stage launches (so the results are the same bits).  Physical workgroup b
// runs on XCD b % 8; each phase's logical workgroups are split into 8
// contiguous ranges, one per XCD, dealt out round robin among that XCD's
// workgroups, as xcd_block does for a plain launch.

struct DevSyncOps {
    static __device__ void add_release(unsigned *p, unsigned v)
    {
        __hip_atomic_fetch_add(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    static __device__ void acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
    static __device__ unsigned load_relaxed(unsigned *p)
    {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    static __device__ void store_relaxed(unsigned *p, unsigned v)
    {
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    static __device__ void pause() { __builtin_amdgcn_s_sleep(2); }
};

struct SArgs {
    RArgs r;                      // reconstruction (state and alpha parity set per stage)
    UArgs up;                     // flux/update (buffers and coefficients set per stage)
    double *u, *k;                // state and stage buffer, device order
    unsigned long long *alpha;    // both parities of alpha slots
    double h;                     // stage scale (the time step; 1 for batches)
    int nsteps, nb_rec, nb_upd;
    unsigned *count, *err;        // barrier arrivals, failure flag (separate 128-byte lines)
    unsigned max_polls;
};

// Logical workgroups [lo, hi) of XCD x when n are split into 8 contiguous ranges.
__device__ __forceinline__ void xcd_range(int n, int x, int &lo, int &hi)
{
    const int per = n >> 3, rem = n & 7;
    lo = x * per + (x < rem ? x : rem);
    hi = lo + per + (x < rem ? 1 : 0);
}

// One wavefront per workgroup: lane 0 arrives for it; false if the barrier failed.
__device__ __forceinline__ bool grid_barrier(const SArgs &a, unsigned epoch)
{
    __syncthreads();
    int ok = 1;
    if (threadIdx.x == 0) ok = arrive_and_wait<DevSyncOps>(a.count, a.err, gridDim.x, epoch, a.max_polls) ? 1 : 0;
    ok = __shfl(ok, 0);
    // lane 0 acquired; the workgroup barrier orders the other lanes after it
    __syncthreads();
    return ok != 0;
}

template <int DIM, int P, int FLUX, int G, int R0, int R1, int R2>
__global__ void __launch_bounds__(64) k_steps(SArgs a)
{
    static_assert(recon_block(DIM) == 64, "one-wavefront reconstruction workgroups");
    constexpr int Q = num_q<DIM, P>();
    __shared__ double lds[recon_lds<DIM, P, FLUX, G>()];
    const int x = (int)(blockIdx.x & 7u), i0 = (int)(blockIdx.x >> 3), nx = (int)(gridDim.x >> 3);
    const int64_t nsl = (int64_t)a.up.nslot * 16;
    unsigned epoch = 0;
    int par = 0;
    for (int s = 0; s < a.nsteps; ++s) {
        for (int st = 0; st < 3; ++st) {
            RArgs r = a.r;
            r.u = st == 0 ? a.u : a.k;
            r.alpha_acc = a.alpha + par * nsl;
            int lo, hi;
            xcd_range(a.nb_rec, x, lo, hi);
            for (int L = lo + i0; L < hi; L += nx) reconstruct_block<DIM, P, FLUX, G, R0, R1, R2>(r, L, lds);
            if (!grid_barrier(a, ++epoch)) return;
            // k1 = u + h L(u); k2 = 3/4 u + 1/4 k1 + 1/4 h L(k1); u = 1/3 u + 2/3 k2 + 2/3 h L(k2)
            UArgs up = a.up;
            up.u0 = a.u;
            up.prev = st == 0 ? a.u : a.k;
            up.out = st == 2 ? a.u : a.k;
            up.A = st == 0 ? 1.0 : (st == 1 ? 0.75 : 1.0 / 3.0);
            up.B = st == 0 ? 0.0 : (st == 1 ? 0.25 : 2.0 / 3.0);
            up.Cdt = st == 0 ? a.h : (st == 1 ? 0.25 * a.h : 2.0 / 3.0 * a.h);
            up.mode = 1;
            up.alpha_rd = a.alpha + par * nsl;
            up.alpha_clr = a.alpha + (par ^ 1) * nsl;
            xcd_range(a.nb_upd, x, lo, hi);
            for (int L = lo + i0; L < hi; L += nx) update_block<DIM, Q, FLUX, 64>(up, L);
            if (!grid_barrier(a, ++epoch)) return;
            par ^= 1;
        }
    }
}

// ------------------------------------------------------------- helpers
__global__ void k_clear_u32(unsigned *p, int n)
{
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t < n) p[t] = 0u;
}

// Device order d <-> user index perm[d]; user arrays have component stride
// ustride (the user's cell count: all cells of a batch with several dims).
__global__ void k_permute(int64_t nc, int nvars, const int32_t *perm, const double *in, double *out,
                          int to_device, int64_t ustride)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nc * nvars) return;
    const int64_t v = t / nc, d = t - v * nc;
    const int64_t u = perm[d];
    if (to_device)
        out[v * nc + d] = in[v * ustride + u];
    else
        out[v * ustride + u] = in[v * nc + d];
}

// Smallest index of a non-finite entry of p[0, n) into *first (left at its
// initial all-ones value if there is none).
__global__ void k_first_nonfinite(int64_t n, const double *p, unsigned long long *first)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(p[i])) atomicMin(first, (unsigned long long)i);
}

__global__ void k_set_u64(unsigned long long *p, unsigned long long v) { *p = v; }

__global__ void k_clear_alpha(unsigned long long *alpha, int nslot)
{
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t < nslot) alpha[(int64_t)t * 16] = 0ull;
}

// ------------------------------------------------------------ dispatch
inline int blocks_for(int64_t work, int per_block) { return (int)((work + per_block - 1) / per_block); }

// Lanes per cell of the characteristic-field variant (2-D Euler, 4 x 3 solves
// per cell).  Measured on 179k cells: 4 lanes beat 8 and 16 by 1.5x and 2.8x
// at p = 3 and 4 (less per-column work replicated across a cell's lanes);
// p = 5 keeps 16, below which its rows spill.
constexpr int char_lanes(int p) { return p == 5 ? 16 : 4; }

template <int DIM, int P, int G, int R0, int R1, int R2>
int launch_k1(const DevMesh &dm, RArgs args, hipStream_t st)
{
    // workgroup ranges of the buckets for BS/G cells per workgroup
    constexpr int BS = recon_block(DIM);
    int nb = 0;
    for (int b = 0; b < kMaxBuckets; ++b) {
        args.blk0[b] = nb;
        nb += blocks_for(args.cell0[b + 1] - args.cell0[b], BS / G);
    }
    args.blk0[kMaxBuckets] = nb;
    if (nb == 0) return 0;
    if constexpr (DIM >= 2 && P == 3 && G == (DIM == 3 ? 8 : 2)) {
        if (dm.balance) {
            // first fit (alpha bounds into scratch slots, gradients kept), range
            // check and listing, then the refit of the listed cells
            BArgs b;
            b.count = args.bal_count;
            b.list = dm.bal_list;
            b.pool = dm.pool;
            b.sptr = dm.sptr;
            b.grad = args.bal_grad;
            b.pool_cap = dm.pool_cap;
            FArgs f;
            f.nc = dm.nc;
            f.u = args.u;
            f.fv = dm.fv;
            f.nsum = dm.nsum;
            f.sptr = dm.sptr;
            f.scol = dm.scol;
            f.mid = dm.mid;
            f.alpha_acc = args.alpha_acc;
            f.count = args.bal_count;
            f.list = dm.bal_list;
            f.spm = args.spm;
            RArgs a1 = args;
            a1.alpha_acc = dm.bal_alpha;
            const int nb2 = blocks_for(dm.nc, BS / G);
            const int nbf = blocks_for(dm.nc, 256);
            constexpr int Q = num_q<DIM, P>();
            if (dm.flux == kFluxBurgers) {
                hipLaunchKernelGGL((k_reconstruct<DIM, P, kFluxBurgers, G, R0, R1, R2, true>), dim3(nb), dim3(BS), 0,
                                   st, a1);
                hipLaunchKernelGGL((k_flag<DIM, Q, kFluxBurgers>), dim3(nbf), dim3(256), 0, st, f);
                hipLaunchKernelGGL((k_rebalance<DIM, P, kFluxBurgers, G, R2>), dim3(nb2), dim3(BS), 0, st, args, b);
            } else if (dm.flux == kFluxAdv) {
                hipLaunchKernelGGL((k_reconstruct<DIM, P, kFluxAdv, G, R0, R1, R2, true>), dim3(nb), dim3(BS), 0, st,
                                   a1);
                hipLaunchKernelGGL((k_flag<DIM, Q, kFluxAdv>), dim3(nbf), dim3(256), 0, st, f);
                hipLaunchKernelGGL((k_rebalance<DIM, P, kFluxAdv, G, R2>), dim3(nb2), dim3(BS), 0, st, args, b);
            } else {
                return (int)hipErrorInvalidValue;
            }
            return (int)hipGetLastError();
        }
    }
    if (dm.balance) return (int)hipErrorInvalidValue;   // no refit variant for this shape
    if (dm.flux == kFluxBurgers) {
        hipLaunchKernelGGL((k_reconstruct<DIM, P, kFluxBurgers, G, R0, R1, R2>), dim3(nb), dim3(BS), 0, st, args);
    } else if (dm.flux == kFluxEuler) {
        if constexpr (DIM == 2) {
            if (dm.characteristic) {
                // one lane count per order (launch_reconstruct picks it)
                if constexpr (G == char_lanes(P))
                    hipLaunchKernelGGL((k_reconstruct<DIM, P, kFluxEulerChar, G, R0, R1, R2>), dim3(nb), dim3(BS), 0,
                                       st, args);
                else
                    return (int)hipErrorInvalidValue;
            } else {
                hipLaunchKernelGGL((k_reconstruct<DIM, P, kFluxEuler, G, R0, R1, R2>), dim3(nb), dim3(BS), 0, st, args);
            }
        } else {
            return (int)hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL((k_reconstruct<DIM, P, kFluxAdv, G, R0, R1, R2>), dim3(nb), dim3(BS), 0, st, args);
    }
    return (int)hipGetLastError();
}

template <int DIM, int Q>
int launch_k23(const DevMesh &dm, const UArgs &args, hipStream_t st)
{
    // one wavefront per workgroup in 2-D: 19,602 triangles step 3.4% faster
    // (graph-replayed steps; alone a launch is no faster); 2 M triangles the same
    constexpr int BS = DIM == 3 ? 256 : 64;
    const int nb = blocks_for(dm.nc, BS);
    if (dm.flux == kFluxBurgers) {
        hipLaunchKernelGGL((k_update<DIM, Q, kFluxBurgers, BS>), dim3(nb), dim3(BS), 0, st, args);
    } else if (dm.flux == kFluxEuler) {
        if constexpr (DIM == 2)
            hipLaunchKernelGGL((k_update<DIM, Q, kFluxEuler, BS>), dim3(nb), dim3(BS), 0, st, args);
        else
            return (int)hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_update<DIM, Q, kFluxAdv, BS>), dim3(nb), dim3(BS), 0, st, args);
    }
    return (int)hipGetLastError();
}

}  // namespace

template <int DIM, int P, int G, int R0, int R1, int R2>
int launch_adj(AArgs args, hipStream_t st)
{
    int nb = 0;
    for (int b = 0; b < kMaxBuckets; ++b) {
        args.blk0[b] = nb;
        nb += blocks_for(args.cell0[b + 1] - args.cell0[b], 256 / G);
    }
    args.blk0[kMaxBuckets] = nb;
    if (nb == 0) return 0;
    hipLaunchKernelGGL((k_adjoint<DIM, P, G, R0, R1, R2>), dim3(nb), dim3(256), 0, st, args);
    return (int)hipGetLastError();
}

int default_lanes(const DevMesh &dm)
{
    return dm.dim == 3 ? 8 : (dm.dim == 2 && dm.p == 3 ? 2 : (dm.dim == 2 && dm.p == 5 ? 16 : 4));
}

std::vector<int> lane_choices(const DevMesh &dm)
{
    if (dm.balance) return {dm.dim == 3 ? 8 : 2};
    if (dm.dim == 2 && dm.flux == kFluxEuler && dm.characteristic) return {char_lanes(dm.p)};
    if (dm.dim == 2 && dm.p == 3) return {2, 4, 8, 16};
    if (dm.dim == 2 && dm.p == 4) return {4, 8, 16};
    if (dm.dim == 2 && dm.p == 5) return {8, 16};
    if (dm.dim == 3 && dm.p == 3) return {8, 16};
    return {4};
}

bool reconstruct_supported(const DevMesh &dm)
{
    const std::vector<int> v = stencil_capacities(dm.dim, dm.p);
    if (v.empty() || dm.nbuckets != (int)v.size()) return false;
    for (int b = 0; b < dm.nbuckets; ++b)
        if (dm.bucket_cap[b] != v[b]) return false;
    return dm.max_stencil <= v.back();
}

RArgs fill_rargs(const DevMesh &dm, const double *u, int parity, double *coef_user, double *fv_user,
                 int32_t *rank_user)
{
    RArgs a;
    a.nc = dm.nc;
    a.u = u;
    a.geo = dm.geo;
    a.vrel = dm.vrel;
    a.nsum = dm.nsum;
    a.normal = dm.normal;
    a.spad = dm.spad;
    a.sib = dm.sib;
    a.perm = dm.perm;
    a.fv = dm.fv;
    a.coef_user = coef_user;
    a.fv_user = fv_user;
    a.rank_user = rank_user;
    a.alpha_acc = dm.alpha + (size_t)parity * dm.alpha_slots() * 16;
    a.mid = dm.mid;
    a.eh2_tab = dm.eh2_tab;
    a.eh2_cell = dm.eh2_cell;
    a.spm = dm.slots_per_mesh;
    a.eh2 = dm.eh2;
    a.alpha_w = dm.alpha_w;
    a.rank_tol = dm.rank_tol;
    a.period = dm.period;
    a.period_y = dm.period_y;
    a.gamma = dm.gamma;
    a.weight_mode = dm.weight_mode;
    a.bal_grad = dm.bal_grad;
    a.bal_count = dm.bal_count ? dm.bal_count + (size_t)parity * 16 : nullptr;
    // bucket b covers the variant's b-th rows-per-lane value; unused buckets are empty
    for (int b = 0; b <= kMaxBuckets; ++b) {
        a.cell0[b] = dm.bucket_cell0[b < dm.nbuckets ? b : dm.nbuckets];
        a.spad_off[b] = dm.spad_off[b];
        if (b < kMaxBuckets) a.stride[b] = b < dm.nbuckets ? dm.bucket_cap[b] : 0;
    }
    return a;
}

int launch_reconstruct(const DevMesh &dm, const double *u, int parity, double *coef_user, double *fv_user,
                       int32_t *rank_user, void *stream)
{
    RArgs a = fill_rargs(dm, u, parity, coef_user, fv_user, rank_user);
    hipStream_t st = (hipStream_t)stream;
    // rows per lane = ceil(capacity / lanes).  Measured fastest: 2 lanes per
    // cell for 2-D p=3 (6 coefficients), 8 in 3-D (10 coefficients, stencils
    // up to 56 rows), 16 for 2-D p=5 (15 coefficients: fewer lanes spill
    // registers), 4 otherwise.  Fewer lanes replicate less of the
    // per-column work (pivot search, exchanges, broadcasts) across a cell.
    const int lanes = dm.lanes ? dm.lanes : default_lanes(dm);
    if (dm.balance) {
        // the refit list of this stage starts empty
        hipLaunchKernelGGL(k_clear_alpha, dim3(1), dim3(64), 0, st, a.bal_count, 1);
        if (dm.dim == 2 && dm.p == 3) return launch_k1<2, 3, 2, 6, 8, 10>(dm, a, st);
        if (dm.dim == 3 && dm.p == 3) return launch_k1<3, 3, 8, 4, 5, 7>(dm, a, st);
        return (int)hipErrorInvalidValue;
    }
    if (dm.dim == 1) {
        switch (dm.p) {
        case 2: return launch_k1<1, 2, 4, 2, 2, 2>(dm, a, st);
        case 3: return launch_k1<1, 3, 4, 2, 2, 2>(dm, a, st);
        case 4: return launch_k1<1, 4, 4, 2, 2, 2>(dm, a, st);
        case 5: return launch_k1<1, 5, 4, 2, 2, 2>(dm, a, st);
        }
    } else if (dm.dim == 2) {
        if (dm.flux == kFluxEuler && dm.characteristic) {
            switch (dm.p) {
            case 2: return launch_k1<2, 2, char_lanes(2), 2, 2, 2>(dm, a, st);
            case 3: return launch_k1<2, 3, char_lanes(3), 3, 4, 5>(dm, a, st);
            case 4: return launch_k1<2, 4, char_lanes(4), 5, 7, 9>(dm, a, st);
            case 5: return launch_k1<2, 5, char_lanes(5), 2, 2, 3>(dm, a, st);
            }
            return (int)hipErrorInvalidValue;
        }
        if (dm.p == 2) return launch_k1<2, 2, 4, 2, 2, 2>(dm, a, st);
        if (dm.p == 3) {
            if (lanes == 2) return launch_k1<2, 3, 2, 6, 8, 10>(dm, a, st);
            if (lanes == 16) return launch_k1<2, 3, 16, 1, 1, 2>(dm, a, st);
            if (lanes == 8) return launch_k1<2, 3, 8, 2, 2, 3>(dm, a, st);
            return launch_k1<2, 3, 4, 3, 4, 5>(dm, a, st);
        }
        if (dm.p == 4) {
            if (lanes == 16) return launch_k1<2, 4, 16, 2, 2, 3>(dm, a, st);
            if (lanes == 8) return launch_k1<2, 4, 8, 3, 4, 5>(dm, a, st);
            return launch_k1<2, 4, 4, 5, 7, 9>(dm, a, st);
        }
        if (dm.p == 5) {
            if (lanes == 8) return launch_k1<2, 5, 8, 3, 4, 5>(dm, a, st);
            return launch_k1<2, 5, 16, 2, 2, 3>(dm, a, st);
        }
    } else if (dm.dim == 3) {
        if (dm.p == 2) return launch_k1<3, 2, 4, 4, 4, 4>(dm, a, st);
        if (dm.p == 3) {
            if (lanes == 16) return launch_k1<3, 3, 16, 2, 3, 4>(dm, a, st);
            return launch_k1<3, 3, 8, 4, 5, 7>(dm, a, st);
        }
    }
    return (int)hipErrorInvalidValue;
}

UArgs fill_uargs(const DevMesh &dm, const double *u0, const double *prev, double *out, double A, double B,
                 double Cdt, int mode, int parity, const double *dt_one = nullptr)
{
    UArgs a;
    a.nc = dm.nc;
    a.fv = dm.fv;
    a.snormal = dm.normal;
    a.rvol = dm.rvol;
    a.sib = dm.sib;
    a.qperm = dm.qperm;
    a.u0 = u0;
    a.prev = prev;
    a.out = out;
    a.alpha_rd = dm.alpha + (size_t)parity * dm.alpha_slots() * 16;
    a.alpha_clr = dm.alpha + (size_t)(parity ^ 1) * dm.alpha_slots() * 16;
    a.mid = dm.mid;
    a.dt_tab = dm.dt_tab;
    a.dt_one = dt_one;
    a.spm = dm.slots_per_mesh;
    a.nslot = (int)dm.alpha_slots();
    a.A = A;
    a.B = B;
    a.Cdt = Cdt;
    a.vel[0] = dm.vel[0];
    a.vel[1] = dm.vel[1];
    a.vel[2] = dm.vel[2];
    a.gamma = dm.gamma;
    a.mode = mode;
    a.bc = dm.bc;
    for (int v = 0; v < 5; ++v) a.far[v] = dm.far[v];
    a.local_alpha = dm.lf_alpha;
    return a;
}

int launch_update(const DevMesh &dm, const double *u0, const double *prev, double *out, double A, double B,
                  double Cdt, int mode, int parity, void *stream, const double *dt_one)
{
    UArgs a = fill_uargs(dm, u0, prev, out, A, B, Cdt, mode, parity, dt_one);
    hipStream_t st = (hipStream_t)stream;
    if (dm.dim == 1) return launch_k23<1, 1>(dm, a, st);
    if (dm.dim == 2) {
        if (dm.nq == 1) return launch_k23<2, 1>(dm, a, st);
        if (dm.nq == 2) return launch_k23<2, 2>(dm, a, st);
        if (dm.nq == 3) return launch_k23<2, 3>(dm, a, st);
    }
    if (dm.dim == 3 && dm.nq == 3) return launch_k23<3, 3>(dm, a, st);
    return (int)hipErrorInvalidValue;
}

// ---------------------------------------------------- persistent steps
namespace {

template <int DIM, int P, int FLUX, int G, int R0, int R1, int R2>
int launch_steps_t(const DevMesh &dm, double *u, double *k, double h, int nsteps, unsigned *sync, hipStream_t st)
{
    SArgs a;
    a.r = fill_rargs(dm, u, 0, nullptr, nullptr, nullptr);
    constexpr int CPB = recon_block(DIM) / G;
    int nb = 0;
    for (int b = 0; b < kMaxBuckets; ++b) {
        a.r.blk0[b] = nb;
        nb += blocks_for(a.r.cell0[b + 1] - a.r.cell0[b], CPB);
    }
    a.r.blk0[kMaxBuckets] = nb;
    a.up = fill_uargs(dm, u, u, k, 1.0, 0.0, h, 1, 0);
    a.u = u;
    a.k = k;
    a.alpha = dm.alpha;
    a.h = h;
    a.nsteps = nsteps;
    a.nb_rec = nb;
    a.nb_upd = blocks_for(dm.nc, 64);
    a.count = sync;
    a.err = sync + 32;
    // a legitimate wait lasts one phase (microseconds to milliseconds); ~2^22
    // polls of ~64 cycles are a quarter of a second
    a.max_polls = 1u << 22;
    const void *fn = reinterpret_cast<const void *>(&k_steps<DIM, P, FLUX, G, R0, R1, R2>);
    int per_cu = 0, dev = 0, ncu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, 0);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    const int resident = per_cu * ncu;
    int grid = nb > a.nb_upd ? nb : a.nb_upd;
    grid = grid < resident ? grid : resident;
    grid &= ~7;   // whole XCD rounds
    if (grid < 8) return (int)hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(64), 0, st, sync, 64);
    void *args[] = {&a};
    e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(64), args, 0, st);
    if (e != hipSuccess) return (int)e;
    return (int)hipGetLastError();
}

}  // namespace

bool steps_supported(const DevMesh &dm)
{
    const int lanes = dm.lanes ? dm.lanes : 2;
    return dm.dim == 2 && dm.p == 3 && lanes == 2 && !dm.balance && !dm.characteristic &&
           (dm.flux == kFluxAdv || dm.flux == kFluxBurgers) && reconstruct_supported(dm);
}

int launch_steps(const DevMesh &dm, double *u, double *k, double h, int nsteps, unsigned *sync, void *stream)
{
    if (!steps_supported(dm)) return (int)hipErrorInvalidValue;
    hipStream_t st = (hipStream_t)stream;
    if (dm.flux == kFluxBurgers) return launch_steps_t<2, 3, kFluxBurgers, 2, 6, 8, 10>(dm, u, k, h, nsteps, sync, st);
    return launch_steps_t<2, 3, kFluxAdv, 2, 6, 8, 10>(dm, u, k, h, nsteps, sync, st);
}

bool adjoint_supported(const DevMesh &dm)
{
    return dm.flux == WLSENO_FLUX_ADVECTION && dm.nvars == 1 && dm.nmesh == 1 && !dm.balance && !dm.eh2_cell &&
           reconstruct_supported(dm);
}

int launch_adjoint(const DevMesh &dm, const double *u, const double *v, const int32_t *tpos, double *contrib,
                   void *stream)
{
    AArgs a;
    a.nc = dm.nc;
    a.npad = dm.spad_off[kMaxBuckets];
    a.u = u;
    a.v = v;
    a.geo = dm.geo;
    a.vrel = dm.vrel;
    a.normal = dm.normal;
    a.rvol = dm.rvol;
    a.spad = dm.spad;
    a.sib = dm.sib;
    a.tpos = tpos;
    a.contrib = contrib;
    a.eh2 = dm.eh2;
    a.alpha_w = dm.alpha_w;
    a.rank_tol = dm.rank_tol;
    a.period = dm.period;
    a.period_y = dm.period_y;
    a.weight_mode = dm.weight_mode;
    a.bc = dm.bc;
    for (int d = 0; d < 3; ++d) a.vel[d] = dm.vel[d];
    for (int b = 0; b <= kMaxBuckets; ++b) {
        a.cell0[b] = dm.bucket_cell0[b < dm.nbuckets ? b : dm.nbuckets];
        a.spad_off[b] = dm.spad_off[b];
        if (b < kMaxBuckets) a.stride[b] = b < dm.nbuckets ? dm.bucket_cap[b] : 0;
    }
    hipStream_t st = (hipStream_t)stream;
    if (dm.dim == 1) {
        switch (dm.p) {
        case 2: return launch_adj<1, 2, 4, 2, 2, 2>(a, st);
        case 3: return launch_adj<1, 3, 4, 2, 2, 2>(a, st);
        case 4: return launch_adj<1, 4, 4, 2, 2, 2>(a, st);
        case 5: return launch_adj<1, 5, 4, 2, 2, 2>(a, st);
        }
    } else if (dm.dim == 2) {
        if (dm.p == 2) return launch_adj<2, 2, 4, 2, 2, 2>(a, st);
        if (dm.p == 3) return launch_adj<2, 3, 4, 3, 4, 5>(a, st);
        if (dm.p == 4) return launch_adj<2, 4, 8, 3, 4, 5>(a, st);
        if (dm.p == 5) return launch_adj<2, 5, 16, 2, 2, 3>(a, st);
    } else if (dm.dim == 3) {
        if (dm.p == 2) return launch_adj<3, 2, 4, 4, 4, 4>(a, st);
        if (dm.p == 3) return launch_adj<3, 3, 8, 4, 5, 7>(a, st);
    }
    return (int)hipErrorInvalidValue;
}

int launch_adjoint_gather(const DevMesh &dm, const int64_t *tptr, const double *contrib, const double *x,
                          const double *y, const double *z, double *out, double A, double B, double C, double D,
                          void *stream)
{
    hipLaunchKernelGGL(k_adjoint_gather, dim3(blocks_for(dm.nc, 256)), dim3(256), 0, (hipStream_t)stream, dm.nc,
                       tptr, contrib, x, y, z, out, A, B, C, D);
    return (int)hipGetLastError();
}

int launch_permute(const DevMesh &dm, const double *in, double *out, bool to_device_order, void *stream)
{
    const int64_t work = dm.nc * dm.nvars;
    hipLaunchKernelGGL(k_permute, dim3(blocks_for(work, 256)), dim3(256), 0, (hipStream_t)stream, dm.nc,
                       dm.nvars, dm.perm, in, out, to_device_order ? 1 : 0, dm.user_stride ? dm.user_stride : dm.nc);
    return (int)hipGetLastError();
}

// Scratch memory of the allocation-free right-hand side (wlseno_rhs_noalloc):
// one array per GPU in the code object's static device memory, kept until the
// process ends.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

size_t scratch_capacity() { return kScratchBytes; }

int scratch_address(int device, void **out)
{
    static std::mutex mu;
    static void *addr[kScratchDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kScratchDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        hipError_t e = hipSetDevice(device);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess) return (int)e;
        addr[device] = p;
    }
    *out = addr[device];
    return 0;
}

int launch_clear_alpha(const DevMesh &dm, void *stream)
{
    const int n = (int)(2 * dm.alpha_slots());
    hipLaunchKernelGGL(k_clear_alpha, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, dm.alpha, n);
    return (int)hipGetLastError();
}

int first_nonfinite(const double *p, int64_t n, unsigned long long *first_dev, unsigned long long *first_host,
                    void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    k_set_u64<<<1, 1, 0, st>>>(first_dev, ~0ull);
    if (n > 0) {
        const int64_t want = (n + 255) / 256;
        k_first_nonfinite<<<(int)(want < 4096 ? want : 4096), 256, 0, st>>>(n, p, first_dev);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    e = hipMemcpyAsync(first_host, first_dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return (int)e;
    return (int)hipStreamSynchronize(st);
}

}  // namespace wlseno
