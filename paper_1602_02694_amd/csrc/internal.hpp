// Internal declarations of the WLS-ENO library (host setup, device data,
// kernel launchers).  Not part of the C-ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wlseno.h"

namespace wlseno {

struct Error {
    wlseno_status status;
    std::string msg;
};

// Number of Taylor coefficients C(p-1+dim, dim).
int num_coeffs(int dim, int p);

// Stencil-size buckets of the reconstruction kernel: bucket b holds the cells
// whose stencils have at most cap[b] rows; its variant keeps ceil(cap[b]/G)
// rows per lane with G lanes per cell.
constexpr int kMaxBuckets = 3;
// Ascending bucket capacities compiled for (dim, p); empty if none.  They
// match the rows-per-lane template arguments of the reconstruction kernels.
inline std::vector<int> stencil_capacities(int dim, int p)
{
    if (dim == 1 && p >= 2 && p <= 5) return {8};
    if (dim == 2 && p == 2) return {8};
    if (dim == 2 && p == 3) return {12, 16, 20};
    if (dim == 2 && p == 4) return {20, 28, 36};
    if (dim == 2 && p == 5) return {24, 32, 40};
    if (dim == 3 && p == 2) return {16};
    if (dim == 3 && p == 3) return {32, 40, 56};
    return {};
}
// Facet quadrature points per facet (1-D: 1; 2-D: ceil(p/2); 3-D: 3).
int points_per_face(int dim, int p);

// Mesh as uploaded (user order), with topology.
struct HostMesh {
    int dim = 0;
    int64_t nv = 0, nc = 0;
    bool periodic = false;
    double period = 0.0, period_y = 0.0;   // along x (1-D: the circle) and, 2-D, along y
    std::vector<double> xyz;         // nv*dim
    std::vector<int32_t> cells;      // nc*(dim+1), user vertex ids
    std::vector<int32_t> vid;        // nc*(dim+1), periodic images identified (one id per point)
    std::vector<double> vol;         // nc
    std::vector<double> cent;        // nc*dim
    std::vector<int32_t> sib;        // nc*(dim+1): (cell << 2 | lf) of the sibling half-facet, or -1
    std::vector<int32_t> v2c_ptr, v2c;   // vertex -> incident cells (CSR, ascending)
    std::vector<int32_t> e2c_ptr, e2c;   // 3-D: edge -> incident cells
    std::vector<int32_t> cell_edges;     // 3-D: nc*6 edge ids
    double h = 0.0;                  // mean edge length (1-D: mean width)
    // batches of independent meshes: mesh of each cell (user order; empty for
    // one mesh) and each mesh's own mean edge length
    int nmesh = 1;
    std::vector<int32_t> mesh_of;
    std::vector<double> mesh_h;
};

// Everything derived for one parameter set, in device cell order.
struct Build {
    wlseno_params prm{};
    int m = 0, nq = 0, nf = 0, nvars = 1, gs = 0;   // gs: geometry record stride (doubles)
    int min_stencil = 0, max_stencil = 0;
    double min_insphere = 0.0;
    // user order / user ids
    std::vector<int32_t> row_ptr, col;
    // perm[d] = user id of device cell d; iperm[u] = device id of user cell u
    std::vector<int32_t> perm, iperm;
    // stencil-size buckets: device cells [bucket_cell0[b], bucket_cell0[b+1])
    // have at most bucket_cap[b] stencil rows (nbuckets <= kMaxBuckets; 0 = unsupported)
    int nbuckets = 0;
    int bucket_cap[kMaxBuckets] = {0, 0, 0};
    int64_t bucket_cell0[kMaxBuckets + 1] = {0, 0, 0, 0};
    // device order records
    std::vector<double> geo;        // nc*gs: centroid, then moments nu(alpha)=mu(alpha)/alpha! for 2 <= |alpha| <= p-1
    std::vector<double> vrel;       // nc*(dim+1)*dim vertex offsets from the centroid
    std::vector<int32_t> sptr, scol;    // device-order CSR, device ids, centre first
    // padded stencil table for the reconstruction kernel: cells of bucket b
    // hold bucket_cap[b] entries each (device ids, centre first, -1 padding)
    // starting at spad_off[b]
    std::vector<int32_t> spad;
    int64_t spad_off[kMaxBuckets + 1] = {0, 0, 0, 0};
    // facet arrays are facet-major: [F][nc] (normals [F][nc][dim])
    std::vector<int32_t> dsib;      // [F][nc]: (device cell << 2 | lf) or -1
    std::vector<int32_t> qperm;     // [F][nc]: 2 bits per point q: sibling's point index of own point q
    std::vector<double> normal;     // [F][nc][dim] outward normals scaled by the facet measure (|f| n);
                                    // the sibling's is the exact negation
    std::vector<double> nsum;       // [F][nc] sum of the unit normal's components (Burgers bound)
    std::vector<double> area;       // [F][nc] facet measures (host only)
    std::vector<double> rvol;       // nc: 1/|tau|
    std::vector<int32_t> mid;       // batches: mesh of each device cell (empty for one mesh)
    // balanced-stencil refit: enlarged stencils, device order and ids, centre
    // first, pool_cap entries per cell (-1 padding)
    std::vector<int32_t> pool;
    int pool_cap = 0;
    // h_mode 1: eps h_i^2 per device cell, h_i the cell's mean edge length
    std::vector<double> eh2_cell;
};

void mesh_setup(HostMesh &mesh, int dim, int64_t nv, const double *xyz, int64_t nc,
                const int32_t *cells, uint32_t flags);
void build_setup(const HostMesh &mesh, const wlseno_params &prm, Build &b);

// ---------------------------------------------------------------- device
struct DevMesh {
    int dim = 0, p = 0, m = 0, nq = 0, nf = 0, nvars = 1, gs = 0;
    int flux = 0, weight_mode = 0, max_stencil = 0;
    int bc = 0;   // boundary facets: 0 outside state = inside state, 1 outside state = 0
    int characteristic = 0;   // Euler: reconstruct characteristic fields per facet
    int lf_alpha = 0;         // 1: local Lax-Friedrichs (Rusanov) alpha per facet point
    const double *eh2_cell = nullptr;   // h_mode 1: eps h_i^2 per cell
    double far[5] = {0, 0, 0, 0, 0};   // bc = 2: outside state
    // balanced-stencil refit: enlarged stencils, the refit list of each stage
    // parity (count at bal_count[parity * 16]) and the listed cells' gradients
    int balance = 0, pool_cap = 0;
    const int32_t *pool = nullptr;
    int32_t *bal_list = nullptr;
    unsigned long long *bal_count = nullptr;
    double *bal_grad = nullptr;
    unsigned long long *bal_alpha = nullptr;   // scratch alpha slots of the discarded first fits
    int lanes = 0;   // lanes per cell in the reconstruction: 0 = automatic, 4 or 8
    int64_t nc = 0;
    int64_t user_stride = 0;   // component stride of user-order arrays (0: nc)
    int nbuckets = 0;
    int bucket_cap[kMaxBuckets] = {0, 0, 0};
    int64_t bucket_cell0[kMaxBuckets + 1] = {0, 0, 0, 0};
    double eh2 = 0.0, alpha_w = 1.5, rank_tol = 1e-12, period = 0.0, period_y = 0.0, gamma = 1.4;
    double vel[3] = {0, 0, 0};
    const double *geo = nullptr, *vrel = nullptr, *normal = nullptr, *rvol = nullptr;   // normal = |f| n
    const double *nsum = nullptr;   // [F][nc] sum_d n_d of the unit normal
    const int32_t *sptr = nullptr, *scol = nullptr, *sib = nullptr, *qperm = nullptr, *perm = nullptr;
    const int32_t *spad = nullptr;
    int64_t spad_off[kMaxBuckets + 1] = {0, 0, 0, 0};
    double *fv = nullptr;                  // [nvars][F][nc][Q], device order
    // Lax-Friedrichs alpha maxima (u64 bits, one slot per 128 bytes): two
    // parities of nmesh x slots_per_mesh slots
    unsigned long long *alpha = nullptr;
    int nmesh = 1, slots_per_mesh = 64;
    const int32_t *mid = nullptr;          // batches: mesh of each device cell
    const double *eh2_tab = nullptr;       // batches: eps h^2 of each mesh
    double *dt_tab = nullptr;              // batches: time step of each mesh
    int64_t alpha_slots() const { return (int64_t)nmesh * slots_per_mesh; }
};

constexpr int kAlphaSlots = 64;       // slots of a single mesh
constexpr int kAlphaSlotsBatch = 8;   // slots per mesh of a batch

// Returns hipSuccess (0) or an error code; `supported` tells whether the
// (dim, p, stencil size) combination has a compiled variant.
bool reconstruct_supported(const DevMesh &dm);
// Lane counts per cell compiled for the reconstruction of this stencil build (the
// automatic choice first is not implied; the autotuner times them all).
std::vector<int> lane_choices(const DevMesh &dm);
// The automatic lane count (wlseno_params.lanes = 0).
int default_lanes(const DevMesh &dm);
int launch_permute(const DevMesh &dm, const double *in, double *out, bool to_device_order, void *stream);
// Transposed Jacobian of the advection right-hand side: per-cell
// contributions written into each receiving cell's segment of contrib
// (positions tpos), then each segment summed and combined as
// out = A x + B y + C z + D (J^T v) (null vectors count as zero).
bool adjoint_supported(const DevMesh &dm);
int launch_adjoint(const DevMesh &dm, const double *u, const double *v, const int32_t *tpos, double *contrib,
                   void *stream);
int launch_adjoint_gather(const DevMesh &dm, const int64_t *tptr, const double *contrib, const double *x,
                          const double *y, const double *z, double *out, double A, double B, double C, double D,
                          void *stream);
// Transposed stencil: segment tptr[j]..tptr[j+1] of cell j lists, in
// increasing source index, the contribution slots that read j (padded stencil
// slots first, then npad + lf nc + i for facet slots); tpos maps each slot to
// its place (-1: padding or a boundary facet).
void transpose_tables(const Build &b, int64_t nc, int nf, std::vector<int64_t> &tptr, std::vector<int32_t> &tpos);
int launch_clear_alpha(const DevMesh &dm, void *stream);
// Smallest index i < n with p[i] not finite into *first_host (all ones if
// none); first_dev: 8 bytes of device memory.  Synchronises the stream.
int first_nonfinite(const double *p, int64_t n, unsigned long long *first_dev, unsigned long long *first_host,
                    void *stream);
// n TVD RK3 steps of the device-order state u (stage buffer k) in one
// cooperative launch with device-wide barriers between phases; sync: 64
// unsigned words of device memory (arrival counter, failure flag at [32],
// nonzero after the launch if a barrier timed out).  Compiled for 2-D p = 3
// scalar fluxes with 2 lanes per cell.
bool steps_supported(const DevMesh &dm);
int launch_steps(const DevMesh &dm, double *u, double *k, double h, int nsteps, unsigned *sync, void *stream);
// Static scratch array of the allocation-free entry point: its size, and its
// device address on `device` (looked up once per device; hipSuccess or an error).
size_t scratch_capacity();
int scratch_address(int device, void **out);
int launch_reconstruct(const DevMesh &dm, const double *u, int parity, double *coef_user,
                       double *fv_user, int32_t *rank_user, void *stream);
// out = L (mode 0) or A*u0 + B*prev + Cdt*L (mode 1).
// Batches: Cdt is the stage coefficient, multiplied by each mesh's time step.
// One mesh with dt_one non-null: likewise, by dt_one[0] (device memory), so
// that captured graphs do not depend on the time step.
int launch_update(const DevMesh &dm, const double *u0, const double *prev, double *out, double A,
                  double B, double Cdt, int mode, int parity, void *stream, const double *dt_one = nullptr);

}  // namespace wlseno
