/*
 * wlseno.h -- C-ABI of the MI355X WLS-ENO finite-volume library.
 *
 * The library implements, on one AMD Instinct MI355X (gfx950), the per-cell
 * weighted-least-squares essentially non-oscillatory (WLS-ENO) reconstruction
 * of Liu & Jiao (arXiv:1602.02694) and the finite-volume update built on it:
 *
 *   given cell averages u_i on a simplex mesh, for every cell
 *     - gather the stencil's cell averages                    (Sec. 3.1.1, 3.2)
 *     - form the non-smoothness indicators and weights        (Sec. 3.1.2, eqs.
 *       smoothness indicator and weight)
 *     - solve the column-scaled weighted least-squares system for the Taylor
 *       coefficients with Householder QR and column pivoting  (Sec. 3.3.2, eq.
 *       scaled_WLS and the rank-truncated pseudo-inverse)
 *     - evaluate the degree p-1 polynomial at the facet quadrature points
 *                                                             (end of Sec. 3.2)
 *   then apply the Lax-Friedrichs flux (Sec. 1, eq. flux) to form
 *   du_i/dt = -(1/|tau_i|) sum_facets flux (Sec. 1, eq. fvm) and advance with
 *   the third-order TVD Runge-Kutta scheme (Sec. 4.2.1, eq. 3rd-order-RK).
 *
 * Conventions (shared with every caller):
 *   - All floating point is IEEE binary64.  Indices are int32.
 *   - Cell arrays are in the caller's ("user") cell order.  Internally the
 *     library renumbers cells (reverse Cuthill-McKee); that is invisible here.
 *   - Field arrays are structure-of-arrays: u[var * n_cell + cell].
 *   - Local facet lf of a cell is the facet opposite its vertex lf.  Facet
 *     points: 1-D the facet node; 2-D ceil(p/2) Gauss-Legendre points along the
 *     edge from vertex (lf+1)%3 to vertex (lf+2)%3, in increasing parameter;
 *     3-D the 3-point degree-2 rule with weight 2/3 on the facet vertices
 *     (lf+1)%4, (lf+2)%4, (lf+3)%4 in that order.
 *   - Taylor coefficients are in graded order: total degree ascending, then
 *     exponent tuples in descending lexicographic order (x first); entry k
 *     multiplies prod_d (x_d - c_d)^{a_kd} / a_kd! about the cell centroid c.
 *   - Device pointers ("_dev") are caller-owned HIP device memory, borrowed for
 *     the duration of the call.  Host pointers are read (or written) before the
 *     call returns.  Device work is enqueued on the context's stream and the
 *     call returns without waiting; the caller synchronises the stream.
 *   - Every function returns a status and never throws; on failure
 *     wlseno_last_error() describes the cause.  A context must be used from one
 *     host thread at a time.
 */
#ifndef WLSENO_H
#define WLSENO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WLSENO_OK = 0,
    WLSENO_EINVAL = 1,       /* bad argument, bad mesh, stencil too small */
    WLSENO_ENOMEM = 2,       /* host or device allocation failed */
    WLSENO_EDEVICE = 3,      /* a HIP runtime call failed */
    WLSENO_ESTATE = 4,       /* call out of order (e.g. rhs before stencil_build),
                                or a device call on a host-only context */
    WLSENO_EUNSUPPORTED = 5, /* valid request outside the compiled variants */
    WLSENO_ENUMERIC = 6      /* non-finite output (only with wlseno_set_numeric_check) */
} wlseno_status;

/* flux functions */
enum {
    WLSENO_FLUX_ADVECTION = 0, /* F(u) = a u; Lax-Friedrichs alpha = |a.n| per facet */
    WLSENO_FLUX_BURGERS = 1,   /* F(u) = (u^2/2)(1,..,1); alpha = global max |u sum_d n_d| */
    WLSENO_FLUX_EULER = 2      /* 2-D Euler, conserved variables (rho, rho u, rho v, E), gamma-law gas */
};

/* mesh flags */
#define WLSENO_MESH_PERIODIC_1D 1u /* 1-D only: first and last node are one point;
                                       period = x_last - x_first */
#define WLSENO_MESH_PERIODIC_2D 2u /* 2-D only: the mesh fills its bounding box and
                                       closes into a torus: every vertex on the upper
                                       x (y) side has a partner on the lower side with
                                       the identical y (x) coordinate, else EINVAL;
                                       periods = the box's extents */

/* Method parameters.  wlseno_params_default() fills the readings used
 * throughout: eps = 1e-2 and alpha_w = 1.5 (the example values of Sec. 3.1.2),
 * rank_tol = 1e-12 relative to |R_11| (Sec. 3.3.2 leaves it open), unit
 * weights off, automatic lane count. */
typedef struct {
    int32_t p;           /* order: reconstruct polynomials of degree p-1 (1-D: 2..5, 2-D: 2..5, 3-D: 2..3) */
    int32_t n_lo, n_hi;  /* stencil size rule: grow rings until >= n_lo cells, keep the n_hi nearest */
    int32_t flux;        /* WLSENO_FLUX_* */
    int32_t weight_mode; /* 0: WLS-ENO weights (eq. weight); 1: unit weights (plain least squares) */
    int32_t lanes;       /* lanes per cell in the reconstruction kernel: 0 = automatic (2 for
                            2-D p = 3, 16 for 2-D p = 5, 8 in 3-D, 4 otherwise); 2, 4, 8 and 16
                            are compiled for 2-D p = 3, 4, 8 and 16 for 2-D p = 4, 8 and 16
                            for 2-D p = 5 and 3-D p = 3.  Other values are EINVAL; a value not
                            compiled for (dim, p) uses the automatic choice.  Results agree to
                            rounding either way.  Characteristic fields (4 lanes, 16 at
                            p = 5) and the balanced refit use their own fixed choice. */
    double eps;          /* epsilon in beta_j = (u_j - u_i)^2 + eps h^2; must be > 0 with
                            weight_mode 0 (equal averages would give an infinite weight),
                            else EINVAL */
    double alpha_w;      /* centre weight factor alpha > 1 in eq. (weight) */
    double rank_tol;     /* numerical rank: |R_kk| > rank_tol |R_11| */
    double velocity[3];  /* advection velocity a */
    double gamma;        /* ratio of specific heats (Euler) */
    int32_t bc;          /* outside state at boundary facet points: 0 = the inside state
                            (transmissive); 1 = zero (a zero far field: with the upwind flux
                            of linear advection, outflow as before and no inflow; EINVAL for
                            the Euler system); 2 = the constant far_state (inflow from a
                            given free stream); 3 = Euler only: a slip wall, the inside state
                            with the normal momentum reversed.  The Lax-Friedrichs alpha
                            bound is taken over inside states only. */
    int32_t characteristic; /* Euler only (else EINVAL for 1): 0 = reconstruct the conserved
                            components; 1 = reconstruct characteristic fields per facet
                            (Sec. 5.1.4, 5.2.4): for each facet, the eigenvectors of the
                            normal-flux Jacobian at the mean of the two cells' averages (the
                            cell's own on the boundary) project the stencil averages, each
                            field gets its own weights and fit, and R maps the facet-point
                            values back; 4 x (dim+1) solves per cell.  Coefficients are then
                            per facet: wlseno_reconstruct rejects a coefficient output
                            (EINVAL); its rank output is the smallest over the facets. */
    double far_state[5]; /* bc = 2: outside state, n_vars components (Euler: rho, rho v, E) */
    int32_t balance;     /* 1: balanced-stencil refit (end of Sec. 3.2) for advection and
                            Burgers at p = 3 in 2-D and 3-D (else EUNSUPPORTED; EINVAL for
                            the Euler system).  A cell with a facet value outside the range
                            of its stencil's averages (beyond a band of 1e-10 of that range)
                            is fitted once more on a stencil balanced across the line/plane
                            through its centroid orthogonal to the first fit's gradient:
                            from its enlarged stencil (the same ring rule with 2 n_lo, 2 n_hi;
                            2 n_hi <= 128), the centroid plus the nearest ceil((n-1)/2)
                            cells on the gradient's side and floor((n-1)/2) on the other (a
                            short side leaves its share to the other), n its own stencil
                            size.  The lanes setting is then automatic. */
    int32_t lf_alpha;    /* Lax-Friedrichs alpha of Burgers and Euler: 0 = one global bound per
                            stage (per mesh in a batch), the maximum over all facet points of
                            the normal spectral radius; 1 = local (Rusanov): at each facet
                            point the larger spectral radius of its two states.  Linear
                            advection always uses |a.n| per facet. */
    int32_t h_mode;      /* h in eps h^2: 0 = the mesh-mean edge length (per mesh in a batch;
                            1-D: mean width); 1 = each cell's own mean edge length (1-D: its
                            width).  The adjoint requires 0 (EUNSUPPORTED otherwise). */
} wlseno_params;

typedef struct {
    int32_t dim;             /* 1, 2 or 3 */
    int32_t m;               /* Taylor coefficients per cell = C(p-1+dim, dim) */
    int32_t n_vars;          /* field components */
    int32_t faces_per_cell;  /* dim + 1 */
    int32_t points_per_face; /* facet quadrature points */
    int32_t min_stencil, max_stencil;
    int32_t n_mesh;          /* meshes in the context (1 unless built from a batch) */
    int64_t n_cell;
    int64_t nnz;             /* total stencil entries */
    double h;                /* mean edge length used in eps h^2 (1-D: mean width); for a
                                batch each mesh uses its own, and this is the union's */
    double min_insphere;     /* min over cells of 2 dim |tau| / |d tau| (CFL length) */
} wlseno_info;

typedef struct wlseno_ctx *wlseno_t;

/* Fill *out with the defaults described above (p=3, n_lo=12, n_hi=20,
 * advection with a = (1,0,0), gamma = 1.4). */
void wlseno_params_default(wlseno_params *out);

/* Create a context on HIP device `device` whose device work goes to
 * `hip_stream` (a hipStream_t; NULL = the device's null stream; see also
 * wlseno_set_stream).  device = -1 creates a host-only context (hip_stream must
 * be NULL): mesh upload, stencil build and the query functions work, device
 * calls return ESTATE. */
wlseno_status wlseno_create(int device, void *hip_stream, wlseno_t *out);

/* Free everything the context owns (host and device).  NULL is accepted. */
wlseno_status wlseno_destroy(wlseno_t ctx);

/* Text of the last error on this context ("" if none); valid until the next
 * call on the context.  ctx = NULL gives the last create() failure. */
const char *wlseno_last_error(wlseno_t ctx);

/* Enqueue all later device work on `hip_stream` (a hipStream_t; NULL = the
 * device's null stream). */
wlseno_status wlseno_set_stream(wlseno_t ctx, void *hip_stream);

/* enable != 0: wlseno_reconstruct, wlseno_rhs, wlseno_rhs_noalloc,
 * wlseno_step and wlseno_batch_step scan their input averages for NaN or
 * infinity before any work, and their outputs after it (a small kernel and a
 * stream synchronisation per scan), and return ENUMERIC naming the first such
 * entry (component and cell, user order) in wlseno_last_error.  A bad input
 * leaves the outputs untouched; a bad output is written as computed.  (The
 * solve does not pass a NaN average on: a NaN row makes the cell's rank 0 and
 * its polynomial zero, so the input scan is what catches it.)  Default: off.
 * A device context allocates 8 bytes of device memory the first time. */
wlseno_status wlseno_set_numeric_check(wlseno_t ctx, int enable);

/* Upload a simplex mesh (host arrays, copied).
 *   xyz   : double[n_vert * dim] vertex coordinates
 *   cells : int32[n_cell * (dim+1)] vertex ids; every cell must have positive
 *           measure (2-D counter-clockwise, 3-D positively oriented), else EINVAL
 *           naming the cell.
 *   flags : WLSENO_MESH_PERIODIC_1D, WLSENO_MESH_PERIODIC_2D or 0.  On a periodic
 *           mesh stencils, centroid offsets and facet neighbours wrap around.
 * Facets shared by more than two cells give EINVAL.  Invalidates any previous
 * stencil build.  (Sec. 3.3.1: cells, sibling half-facets, vertex-to-cell map.) */
wlseno_status wlseno_mesh_upload(wlseno_t ctx, int dim, int64_t n_vert, const double *xyz,
                                 int64_t n_cell, const int32_t *cells, uint32_t flags);

/* Build the per-cell stencils and all per-cell geometry for `params`, and
 * copy them to the device (device contexts).  Stencils follow the k-ring
 * neighbourhoods of Sec. 3.2 (1/2-ring increments in 2-D, 1/3-ring in 3-D):
 * levels grow until a stencil holds >= n_lo cells; stencils with more than
 * n_hi cells keep the centre and the n_hi-1 cells with the smallest squared
 * centroid distance (ties: lower user id).  Rows are ordered centre first,
 * then by (squared distance, user id).  The squared distance is
 * sum_d (c_jd - c_id)^2 accumulated in coordinate order with centroids
 * (sum_v x_v)/(dim+1) accumulated in vertex order, no fused multiply-add
 * (1-D periodic: nearest image).  A stencil with fewer than m cells gives
 * EINVAL naming the cell. */
wlseno_status wlseno_stencil_build(wlseno_t ctx, const wlseno_params *params);

/* Sizes of the current build (after stencil_build). */
wlseno_status wlseno_get_info(wlseno_t ctx, wlseno_info *out);

/* Copy the stencils to host arrays in user order and user ids:
 * row_ptr int32[n_cell+1], col int32[nnz]; rows as described above. */
wlseno_status wlseno_get_stencil(wlseno_t ctx, int32_t *row_ptr, int32_t *col);

/* Reconstruct every cell from u_dev (double[n_vars * n_cell]): gather the
 * stencil's averages (Sec. 3.1.1, 3.2), weight the rows by the
 * non-smoothness indicators (Sec. 3.1.2), solve the column-scaled weighted
 * least-squares system by QR with column pivoting (Sec. 3.3.2) and evaluate
 * the polynomial at the facet quadrature points (Sec. 1, 3.3.1).
 *   coef_dev     : nullable, double[n_vars * n_cell * m] Taylor coefficients
 *   facevals_dev : nullable, double[n_vars * n_cell * (dim+1) * Q] values of the
 *                  reconstruction at each cell's own facet points
 *   rank_dev     : nullable, int32[n_vars * n_cell] numerical ranks */
wlseno_status wlseno_reconstruct(wlseno_t ctx, const double *u_dev, double *coef_dev,
                                 double *facevals_dev, int32_t *rank_dev);

/* dudt_dev = L(u_dev): the semi-discrete right-hand side
 * -(1/|tau_i|) sum_f |f| sum_q w_q Fhat(u-, u+, n) (Sec. 1, the finite-volume
 * and Lax-Friedrichs flux equations), with the alpha that wlseno_params.lf_alpha
 * selects.  At boundary facets u+ is the outside state that wlseno_params.bc
 * selects.  dudt_dev must not alias u_dev. */
wlseno_status wlseno_rhs(wlseno_t ctx, const double *u_dev, double *dudt_dev);

/* Advance u_dev in place by n_steps steps of size dt of the third-order TVD
 * Runge-Kutta scheme (Sec. 4.2.1; three right-hand sides per step, each as
 * wlseno_rhs). */
wlseno_status wlseno_step(wlseno_t ctx, double *u_dev, double dt, int n_steps);

/* The global Lax-Friedrichs alpha of the last rhs stage: the largest normal
 * spectral radius over all facet points (Burgers/Euler; 0 for advection; for
 * a batch the largest over its meshes), also when lf_alpha = 1 selects local
 * values for the flux (it bounds the CFL time step).  Read back from the
 * device (synchronises the stream). */
wlseno_status wlseno_last_alpha(wlseno_t ctx, double *alpha);

/* wlseno_step and wlseno_batch_step replay runs of RK3 steps from HIP graphs
 * of 32, 16, 8, 4 and 2 steps (32 as often as it fits, then each shorter size
 * at most once) and launch an odd last step directly.  The five graphs are
 * captured together the first time a run of 2 or more steps needs them, once
 * per context and stencil build (time steps are read from device memory, so a
 * new dt needs no recapture).  enable = 0 launches every kernel directly; results
 * are identical either way.  The default is enabled. */
wlseno_status wlseno_set_graphs(wlseno_t ctx, int enable);

/* How wlseno_step and wlseno_batch_step launch their stages: 0 = two kernels
 * per stage, launched directly; 1 (the default) = the same kernels replayed
 * from HIP graphs as described for wlseno_set_graphs; 2 = all steps in one
 * cooperative launch of a persistent kernel whose workgroups (as many as fit
 * on the device at once) run every stage's reconstruction and update phases
 * with a device-wide barrier after each.  Results are identical in every
 * mode.  Mode 2 is compiled for 2-D p = 3 advection and Burgers with 2 lanes
 * per cell and no balanced refit (else the stepping call returns
 * EUNSUPPORTED); its barrier waits are bounded, and wlseno_step then waits for
 * the device and returns EDEVICE if a barrier timed out.  EINVAL for another
 * mode.  wlseno_set_graphs(ctx, e) is wlseno_set_step_mode(ctx, e ? 1 : 0). */
wlseno_status wlseno_set_step_mode(wlseno_t ctx, int mode);

/* Batches of independent meshes (many meshes stepped by one set of launches
 * per stage).  Each call appends one mesh (host arrays, copied; no flags) and
 * returns its index in *mesh_id (nullable); adding costs time in proportion
 * to the mesh alone (the batch is assembled by the next stencil build).  The
 * batch replaces any mesh given by wlseno_mesh_upload, and wlseno_mesh_upload
 * replaces the batch.  After wlseno_stencil_build every call works on the
 * concatenation in add order: cells of mesh 0 first, then mesh 1, ...; fields
 * are double[n_vars][sum of n_cell].  Stencils never cross meshes (they share
 * no vertex); each mesh uses its own eps h^2 and its own Lax-Friedrichs alpha
 * (Burgers, Euler).
 *
 * Meshes of different dims may share a batch: the meshes of each dim form a
 * group with its own stencils, order p and compiled kernels (parameters per
 * dim from wlseno_batch_params), and every stage runs the groups' kernels
 * concurrently on streams forked from the context's (joined back into it
 * before the call's work ends).  All groups need the same n_vars; the caller's
 * arrays stay in add order.  Such a batch supports stencil build, get_info
 * (per-dim sizes m, faces and points are 0 there; dim is 0), get_stencil,
 * rhs, rhs_noalloc, step, batch_step, last_alpha, batch_last_alpha,
 * set_graphs, set_step_mode and autotune (each group tuned; out describes the
 * first); reconstruct and time_kernel give EUNSUPPORTED, as do the adjoint
 * calls for any batch.
 *
 * Sizes: the total must fit 32-bit cell indices, as for a single mesh.  EINVAL
 * for a bad mesh. */
wlseno_status wlseno_batch_add_mesh(wlseno_t ctx, int dim, int64_t n_vert, const double *xyz, int64_t n_cell,
                                    const int32_t *cells, int32_t *mesh_id);

/* Parameters for the batch's meshes of one dim (1, 2 or 3): the next
 * wlseno_stencil_build uses *params for them instead of its own argument (for
 * instance p and the stencil sizes n_lo, n_hi differ between 2-D and 3-D
 * meshes).  params = NULL drops the setting.  EINVAL for another dim. */
wlseno_status wlseno_batch_params(wlseno_t ctx, int dim, const wlseno_params *params);

/* n_steps TVD RK3 steps of the whole batch in place, mesh k with time step
 * dt_per_mesh[k] (host array of n_mesh finite doubles).  wlseno_step on a
 * batch uses one dt for every mesh.  EINVAL for null pointers, n_steps < 0 or
 * a non-finite step. */
wlseno_status wlseno_batch_step(wlseno_t ctx, double *u_dev, const double *dt_per_mesh, int n_steps);

/* The Lax-Friedrichs alpha of each mesh in the last rhs stage (host array of
 * n_mesh doubles; 0 for advection).  Synchronises the stream. */
wlseno_status wlseno_batch_last_alpha(wlseno_t ctx, double *alpha_per_mesh);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * dudt_dev = L(u_dev) as wlseno_rhs, bit for bit, with every scratch buffer
 * (stage state and result in device order, facet values, Lax-Friedrichs alpha
 * slots) in one static array of 32 MiB per GPU inside the library, held until
 * the process ends.  The call allocates nothing and frees nothing; it enqueues
 * kernels only (the alpha slots are cleared by a kernel).  Limit: a mesh whose
 * scratch exceeds 32 MiB gives EINVAL (2-D p = 3 scalar: 64 B per cell, about
 * 520 k cells; 2-D Euler p = 4: 256 B per cell); the balanced refit gives
 * EUNSUPPORTED.  All contexts on one GPU share the array and each call
 * overwrites it: calls that overlap on one GPU (several host threads, or
 * streams not ordered with each other) race and must be serialised by the
 * caller.  wlseno_last_alpha does not see this call.  Arguments and errors as
 * wlseno_rhs. */
wlseno_status wlseno_rhs_noalloc(wlseno_t ctx, const double *u_dev, double *dudt_dev);

/* Adjoint (scalar linear advection on a single mesh; other cases return
 * EUNSUPPORTED).  The right-hand side L(u) is differentiated on its active
 * branch: stencils, pivot order, numerical rank and the facet neighbour that
 * gives the centre's smallest indicator are held at their values at u, while
 * the weights' dependence on u (eq. for beta and omega) is differentiated.
 *
 * out_dev = J(u)^T v_dev with J = dL/du at u_dev (all double[n_cell] on the
 * device, user order; out_dev must not alias an input).  Deterministic: each
 * cell's contributions are summed over the transposed stencil in a fixed
 * order, without atomics. */
wlseno_status wlseno_rhs_vjp(wlseno_t ctx, const double *u_dev, const double *v_dev, double *out_dev);

/* g0_dev = (d u(T) / d u0)^T gT_dev, where u(T) is n_steps TVD RK3 steps of
 * size dt from u0_dev: the gradient of any loss of u(T) with respect to u0
 * given its gradient gT with respect to u(T).  The forward trajectory is
 * stored every ckpt_every steps and recomputed in between (memory: n_steps /
 * ckpt_every + 3 ckpt_every states).  EINVAL for null pointers, a
 * non-finite dt, n_steps < 0 or ckpt_every < 1. */
wlseno_status wlseno_step_adjoint(wlseno_t ctx, const double *u0_dev, double dt, int n_steps, int ckpt_every,
                                  const double *gT_dev, double *g0_dev);

/* The same gradient in two calls, for callers that run the forward anyway
 * (training loops, torch.autograd): wlseno_step_record advances u_dev in
 * place by n_steps RK3 steps (as wlseno_step) and keeps the state every
 * ckpt_every steps; wlseno_step_adjoint_recorded then writes
 * g0_dev = (d u(T) / d u0)^T gT_dev for that trajectory without running the
 * forward again.  A rebuild, another record or wlseno_step_adjoint drops the
 * record (ESTATE until the next record).  Arguments as wlseno_step_adjoint. */
wlseno_status wlseno_step_record(wlseno_t ctx, double *u_dev, double dt, int n_steps, int ckpt_every);
wlseno_status wlseno_step_adjoint_recorded(wlseno_t ctx, const double *gT_dev, double *g0_dev);

/* Result of wlseno_autotune. */
typedef struct {
    int32_t n;          /* lane counts timed (at most 4) */
    int32_t lanes[4];   /* each lane count per cell timed */
    double us[4];       /* its average reconstruction launch, microseconds */
    int32_t chosen;     /* the fastest: the context uses it from now on */
    int32_t cached;     /* 1 when taken, without timing, from this process's earlier result for the
                           same device, kernel build and workload class */
} wlseno_tune;

/* Launch-shape autotuner of the reconstruction kernel: times every lane count
 * per cell compiled for the current stencil build (2-D p = 3: 2, 4, 8, 16; p = 4: 4, 8, 16;
 * p = 5 and 3-D p = 3: 8, 16; otherwise one) on this mesh, back-to-back launches
 * between HIP events (~20 ms each), and keeps the fastest for this context
 * (the automatic choice of wlseno_params.lanes = 0 unless another is faster
 * by 2% or more)
 * (captured step graphs are dropped and recaptured).  Fewer lanes per cell
 * hold more stencil rows per lane (more registers, fewer resident waves);
 * more lanes add exchanges per column.  The choice is cached in the process
 * per device, kernel build and workload class (dim, p, flux variant,
 * components, smallest and largest stencil, share of cells per stencil-size
 * bucket in tenths, cell count to the next power of two).  u_dev: the state
 * to time on (double[n_vars * n_cell], user order), or NULL for a smooth
 * synthetic state.  A rebuild (wlseno_stencil_build) returns to
 * wlseno_params.lanes.  Synchronises the stream. */
wlseno_status wlseno_autotune(wlseno_t ctx, const double *u_dev, wlseno_tune *out);

/* Kernel timing for measurement.  Reconstructs u_dev (user order, n_cell
 * doubles on the device, not modified) once, then records a HIP event on the
 * context's stream, launches one kernel of a right-hand-side stage `launches`
 * times back to back, records a second event and synchronises; *avg_ms is the
 * elapsed time divided by `launches`.  kernel 0 = reconstruction
 * (k_reconstruct: stencil gather, weights, QRCP solve, facet evaluation),
 * 1 = flux, divergence and update (k_update, writing L(u) to an internal
 * buffer).  Both launches are idempotent, so back-to-back runs measure the
 * kernel itself without event gaps between launches.  EINVAL for kernel not
 * 0/1, launches < 1 or a null pointer; ESTATE without a device stencil build. */
wlseno_status wlseno_time_kernel(wlseno_t ctx, int kernel, const double *u_dev, int launches, double *avg_ms);

#ifdef __cplusplus
}
#endif

#endif /* WLSENO_H */
