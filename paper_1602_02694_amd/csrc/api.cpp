// C-ABI entry points of the WLS-ENO library (declared in include/wlseno.h).
// Host orchestration only: every numerical step of the path runs in the HIP
// kernels of kernels.hip; this file validates arguments, owns device memory
// and enqueues the kernels on the context's stream.
#include <hip/hip_runtime_api.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace wlseno;

struct wlseno_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    unsigned char *scratch = nullptr;   // this device's static scratch array (wlseno_rhs_noalloc)
    bool check_numeric = false;         // wlseno_set_numeric_check
    unsigned long long *nf_first = nullptr;   // its device word (first non-finite entry)
    std::string err;
    bool have_mesh = false, have_build = false;
    HostMesh mesh;
    Build build;
    DevMesh dm;
    std::vector<void *> allocs;
    double *ubuf = nullptr, *kbuf = nullptr, *tbuf = nullptr;
    int last_parity = 0;
    // batch of independent meshes, concatenated in the order they were added
    struct Part {
        int64_t nv, nc;
    };
    int batch_dim = 0;
    std::vector<Part> parts;
    std::vector<double> batch_xyz;
    std::vector<int32_t> batch_cells;
    std::vector<double> batch_h;   // each mesh's mean edge length
    bool batch_pending = false;    // meshes added since the union was last set up
    // parameters given per dim for batches (wlseno_batch_params), index dim
    bool has_dim_prm[4] = {false, false, false, false};
    wlseno_params dim_prm[4];
    // a batch whose meshes have several dims: one group per dim (in order of
    // first appearance), each an internal single-dim batch context whose
    // permutation maps its device cells straight to the caller's cells
    struct Group {
        int dim = 0;
        wlseno_ctx *c = nullptr;
        std::vector<int32_t> meshes;   // batch mesh ids of the group, ascending
        hipStream_t st = nullptr;      // the group's stream (forked from ours)
        hipEvent_t done = nullptr;
    };
    std::vector<Group> groups;         // empty unless the batch has several dims
    std::vector<int32_t> mesh_group;   // group of each batch mesh
    hipEvent_t fork = nullptr;
    std::vector<double> dt_host;   // per-mesh time steps last sent to the device
    // RK3 steps replayed from captured HIP graphs of kGraphSteps[g] steps (an
    // even number: stage parities 0,1,0,1,... start and end alike), captured
    // on a private stream for one stage scale
    bool use_graphs = true;
    int step_mode = 1;            // 0 direct launches, 1 graph replay, 2 one persistent launch
    unsigned *sync = nullptr;     // persistent launch: barrier counter and failure flag
    hipStream_t cap = nullptr;
    hipGraphExec_t graph[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double graph_h[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    // adjoint: transposed stencil, contributions, cotangents, checkpoints
    bool adj_ready = false;
    int64_t *tptr = nullptr;
    int32_t *tpos = nullptr;
    double *contrib = nullptr, *ga = nullptr, *gb = nullptr, *gc = nullptr;
    double *ck = nullptr, *seg = nullptr;
    size_t ck_cap = 0, seg_cap = 0;   // doubles
    bool rec_valid = false;           // ck holds the checkpoints of a recorded trajectory
    double rec_dt = 0.0;
    int rec_n = 0, rec_ckpt = 1;
};

namespace {

thread_local std::string g_create_error;

void check_hip(hipError_t e, const char *what)
{
    if (e != hipSuccess) throw Error{WLSENO_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

void check_launch(int e, const char *what)
{
    if (e != 0) throw Error{WLSENO_EDEVICE, std::string(what) + ": " + hipGetErrorString((hipError_t)e)};
}

// Steps per graph: a ladder of powers of two, so that a run of n steps takes
// floor(n / 32) replays of the longest and at most one of each shorter size
// (each replay costs ~7 us of launch overhead on the 19,602-triangle
// benchmark, against 44 us per step), then one direct step if n is odd.
constexpr int kGraphLadder = 5;
constexpr int kGraphSteps[kGraphLadder] = {32, 16, 8, 4, 2};
// Cells up to which newly captured graphs get one replay ahead of use.
constexpr int64_t kPrereplayCells = int64_t(1) << 16;

void drop_graph(wlseno_ctx *c)
{
    for (int g = 0; g < kGraphLadder; ++g) {
        if (c->graph[g]) {
            (void)hipSetDevice(c->device);
            (void)hipGraphExecDestroy(c->graph[g]);
        }
        c->graph[g] = nullptr;
    }
}

void free_device(wlseno_ctx *c)
{
    drop_graph(c);
    if (c->device >= 0) {
        (void)hipSetDevice(c->device);
        for (void *p : c->allocs) (void)hipFree(p);
    }
    c->allocs.clear();
    c->dm = DevMesh{};
    c->ubuf = c->kbuf = c->tbuf = nullptr;
    c->sync = nullptr;
    c->adj_ready = false;
    c->tptr = nullptr;
    c->tpos = nullptr;
    c->contrib = c->ga = c->gb = c->gc = c->ck = c->seg = nullptr;
    c->ck_cap = c->seg_cap = 0;
    c->rec_valid = false;
}

void *dev_alloc(wlseno_ctx *c, size_t bytes)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 8);
    if (e != hipSuccess) throw Error{WLSENO_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    c->allocs.push_back(p);
    return p;
}

// A device buffer of at least n doubles held in *p (capacity *cap), grown
// after the stream has drained.
double *dev_grow(wlseno_ctx *c, double **p, size_t *cap, size_t n)
{
    if (*p && *cap >= n) return *p;
    if (*p) {
        check_hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        for (auto it = c->allocs.begin(); it != c->allocs.end(); ++it)
            if (*it == *p) {
                c->allocs.erase(it);
                break;
            }
        (void)hipFree(*p);
        *p = nullptr;
        *cap = 0;
    }
    *p = (double *)dev_alloc(c, n * sizeof(double));
    *cap = n;
    return *p;
}

template <class T>
T *upload(wlseno_ctx *c, const std::vector<T> &v)
{
    T *p = (T *)dev_alloc(c, v.size() * sizeof(T));
    if (!v.empty()) check_hip(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
    return p;
}

void need_device(wlseno_ctx *c)
{
    if (c->device < 0) throw Error{WLSENO_ESTATE, "host-only context has no device"};
    if (!c->have_build) throw Error{WLSENO_ESTATE, "call wlseno_stencil_build first"};
    check_hip(hipSetDevice(c->device), "hipSetDevice");
}

void upload_build(wlseno_ctx *c)
{
    free_device(c);
    const Build &b = c->build;
    const HostMesh &m = c->mesh;
    check_hip(hipSetDevice(c->device), "hipSetDevice");
    DevMesh dm;
    dm.dim = m.dim;
    dm.p = b.prm.p;
    dm.m = b.m;
    dm.nq = b.nq;
    dm.nf = b.nf;
    dm.nvars = b.nvars;
    dm.gs = b.gs;
    dm.flux = b.prm.flux;
    dm.weight_mode = b.prm.weight_mode;
    dm.lanes = b.prm.lanes;
    dm.max_stencil = b.max_stencil;
    dm.nc = m.nc;
    dm.nbuckets = b.nbuckets;
    for (int t = 0; t < kMaxBuckets; ++t) dm.bucket_cap[t] = b.bucket_cap[t];
    for (int t = 0; t <= kMaxBuckets; ++t) dm.bucket_cell0[t] = b.bucket_cell0[t];
    dm.eh2 = b.prm.eps * m.h * m.h;
    dm.nmesh = m.nmesh;
    dm.slots_per_mesh = m.nmesh > 1 ? kAlphaSlotsBatch : kAlphaSlots;
    if (m.nmesh > 1) {
        std::vector<double> eh2(m.nmesh);
        for (int k = 0; k < m.nmesh; ++k) eh2[k] = b.prm.eps * m.mesh_h[k] * m.mesh_h[k];
        dm.mid = upload(c, b.mid);
        dm.eh2_tab = upload(c, eh2);
    }
    // time step per mesh in device memory (one mesh: one entry), read by the
    // stepping kernels so that captured graphs hold no time step
    dm.dt_tab = (double *)dev_alloc(c, m.nmesh * sizeof(double));
    c->dt_host.assign(m.nmesh, NAN);
    dm.alpha_w = b.prm.alpha_w;
    dm.rank_tol = b.prm.rank_tol;
    dm.period = m.periodic ? m.period : 0.0;
    dm.period_y = m.periodic ? m.period_y : 0.0;
    dm.gamma = b.prm.gamma;
    dm.bc = b.prm.bc;
    dm.characteristic = b.prm.characteristic;
    dm.lf_alpha = b.prm.lf_alpha;
    if (b.prm.h_mode == 1) dm.eh2_cell = upload(c, b.eh2_cell);
    for (int v = 0; v < 5; ++v) dm.far[v] = b.prm.far_state[v];
    for (int d = 0; d < 3; ++d) dm.vel[d] = b.prm.velocity[d];
    if (b.prm.balance) {
        dm.balance = 1;
        dm.pool_cap = b.pool_cap;
        dm.pool = upload(c, b.pool);
        dm.bal_list = (int32_t *)dev_alloc(c, m.nc * sizeof(int32_t));
        dm.bal_grad = (double *)dev_alloc(c, m.nc * m.dim * sizeof(double));
        dm.bal_count = (unsigned long long *)dev_alloc(c, 32 * sizeof(unsigned long long));
        check_hip(hipMemset(dm.bal_count, 0, 32 * sizeof(unsigned long long)), "hipMemset");
        dm.bal_alpha = (unsigned long long *)dev_alloc(c, (size_t)dm.alpha_slots() * 16 * sizeof(unsigned long long));
        check_hip(hipMemset(dm.bal_alpha, 0, (size_t)dm.alpha_slots() * 16 * sizeof(unsigned long long)), "hipMemset");
    }
    dm.geo = upload(c, b.geo);
    dm.vrel = upload(c, b.vrel);
    dm.normal = upload(c, b.normal);
    dm.nsum = upload(c, b.nsum);
    dm.rvol = upload(c, b.rvol);
    dm.sptr = upload(c, b.sptr);
    dm.scol = upload(c, b.scol);
    dm.spad = upload(c, b.spad);
    for (int t = 0; t <= kMaxBuckets; ++t) dm.spad_off[t] = b.spad_off[t];
    dm.sib = upload(c, b.dsib);
    dm.qperm = upload(c, b.qperm);
    dm.perm = upload(c, b.perm);
    const size_t nfv = (size_t)b.nvars * m.nc * b.nf * b.nq;
    dm.fv = (double *)dev_alloc(c, nfv * sizeof(double));
    const size_t nslot = 2 * (size_t)dm.alpha_slots() * 16;
    dm.alpha = (unsigned long long *)dev_alloc(c, nslot * sizeof(unsigned long long));
    check_hip(hipMemset(dm.alpha, 0, nslot * sizeof(unsigned long long)), "hipMemset");
    const size_t nu = (size_t)b.nvars * m.nc;
    c->ubuf = (double *)dev_alloc(c, nu * sizeof(double));
    c->kbuf = (double *)dev_alloc(c, nu * sizeof(double));
    c->tbuf = (double *)dev_alloc(c, nu * sizeof(double));
    c->dm = dm;
    if (!reconstruct_supported(dm))
        throw Error{WLSENO_EUNSUPPORTED, "no compiled reconstruction variant for dim " + std::to_string(m.dim) +
                                             ", p " + std::to_string(dm.p) + ", stencils up to " +
                                             std::to_string(b.max_stencil) + " cells"};
}

// One right-hand-side stage: K1 then K2/K3 (flux, divergence, RK combination).
// dev_dt (one mesh): Cdt is the stage coefficient and the kernel multiplies it
// by the time step held in dm.dt_tab[0].
void stage(wlseno_ctx *c, const double *in, const double *u0, const double *prev, double *out, double A,
           double B, double Cdt, int mode, int parity, hipStream_t st, bool dev_dt = false)
{
    check_launch(launch_reconstruct(c->dm, in, parity, nullptr, nullptr, nullptr, st), "reconstruct");
    check_launch(launch_update(c->dm, u0, prev, out, A, B, Cdt, mode, parity, st, dev_dt ? c->dm.dt_tab : nullptr),
                 "update");
    c->last_parity = parity;
}

// One TVD RK3 step on the device-order state ubuf, starting at `par`:
// k1 = u + dt L(u); k2 = 3/4 u + 1/4 k1 + 1/4 dt L(k1); u = 1/3 u + 2/3 k2 + 2/3 dt L(k2)
// (h = dt, or h = 1 with the time step in device memory: batches, or dev_dt)
int rk3_step(wlseno_ctx *c, double h, int par, hipStream_t st, bool dev_dt = false)
{
    double *u = c->ubuf, *k = c->kbuf;
    stage(c, u, u, u, k, 1.0, 0.0, h, 1, par, st, dev_dt);
    par ^= 1;
    stage(c, k, u, k, k, 0.75, 0.25, 0.25 * h, 1, par, st, dev_dt);
    par ^= 1;
    stage(c, k, u, k, u, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0 * h, 1, par, st, dev_dt);
    return par ^ 1;
}

// The graph of kGraphSteps[g] steps for stage scale h (captured if missing).
hipGraphExec_t steps_graph(wlseno_ctx *c, double h, int g)
{
    if (c->graph[g] && std::memcmp(&c->graph_h[g], &h, sizeof h) == 0) return c->graph[g];
    if (c->graph[g]) {
        (void)hipGraphExecDestroy(c->graph[g]);
        c->graph[g] = nullptr;
    }
    if (!c->cap) check_hip(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    check_hip(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipGraph_t gr = nullptr;
    try {
        int par = 0;
        for (int t = 0; t < kGraphSteps[g]; ++t) par = rk3_step(c, h, par, c->cap, c->dm.nmesh == 1);
    } catch (...) {
        (void)hipStreamEndCapture(c->cap, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
    }
    check_hip(hipStreamEndCapture(c->cap, &gr), "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    check_hip(e, "hipGraphInstantiate");
    // set up its device-side resources now rather than at its first replay
    e = hipGraphUpload(ex, c->stream);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(ex);
        check_hip(e, "hipGraphUpload");
    }
    c->graph[g] = ex;
    c->graph_h[g] = h;
    return ex;
}

double time_launches(wlseno_ctx *ctx, int kernel, int launches);

// With the numeric check on: ENUMERIC if p[0, n) (an output in user order,
// `per` entries per component and cell, components of `stride` cells) holds a
// NaN or infinity, naming the first.
void numeric_check(wlseno_ctx *ctx, const double *p, int64_t n, int64_t stride, int per, const char *what)
{
    if (!ctx->check_numeric || !p || n <= 0) return;
    unsigned long long first = 0;
    check_launch(first_nonfinite(p, n, ctx->nf_first, &first, ctx->stream), "numeric check");
    if (first == ~0ull) return;
    const int64_t i = (int64_t)first, cell = (i / per) % stride, comp = (i / per) / stride;
    throw Error{WLSENO_ENUMERIC, std::string("non-finite ") + what + " at entry " + std::to_string(i) + " (component " +
                                     std::to_string(comp) + ", cell " + std::to_string(cell) + ")"};
}

// Cells and components of the caller's arrays: the whole batch for a mixed one.
int64_t user_cells(const wlseno_ctx *ctx)
{
    if (ctx->groups.empty()) return ctx->dm.nc;
    int64_t n = 0;
    for (const auto &pt : ctx->parts) n += pt.nc;
    return n;
}
int user_vars(const wlseno_ctx *ctx) { return ctx->groups.empty() ? ctx->dm.nvars : ctx->groups[0].c->dm.nvars; }

}  // namespace

// A roctx range around each call that enqueues device work, so that a
// marker trace shows the C-ABI calls above their kernels (no cost without a tool).
struct ApiRange {
    explicit ApiRange(const char *name) { roctxRangePushA(name); }
    ~ApiRange() { roctxRangePop(); }
    ApiRange(const ApiRange &) = delete;
    ApiRange &operator=(const ApiRange &) = delete;
};

#define API_BEGIN(ctx)                                                   \
    if (!(ctx)) return WLSENO_EINVAL;                                    \
    (ctx)->err.clear();                                                  \
    try {
#define API_END(ctx)                                                     \
    }                                                                    \
    catch (const Error &e) {                                             \
        (ctx)->err = e.msg;                                              \
        return e.status;                                                 \
    }                                                                    \
    catch (const std::bad_alloc &) {                                     \
        (ctx)->err = "host allocation failed";                           \
        return WLSENO_ENOMEM;                                            \
    }                                                                    \
    catch (const std::exception &e) {                                    \
        (ctx)->err = e.what();                                           \
        return WLSENO_EINVAL;                                            \
    }                                                                    \
    return WLSENO_OK;

namespace {

// ---------------------------------------------------------- batch groups

bool mixed(const wlseno_ctx *c) { return !c->groups.empty(); }

void check_child(wlseno_ctx *g, wlseno_status st, int dim)
{
    if (st != WLSENO_OK) throw Error{st, std::to_string(dim) + "-D meshes of the batch: " + g->err};
}

void drop_groups(wlseno_ctx *c)
{
    for (auto &g : c->groups) {
        if (g.c) (void)wlseno_destroy(g.c);
        if (g.st) (void)hipStreamDestroy(g.st);
        if (g.done) (void)hipEventDestroy(g.done);
    }
    c->groups.clear();
    c->mesh_group.clear();
    if (c->fork) (void)hipEventDestroy(c->fork);
    c->fork = nullptr;
}

// Append batch mesh `id` (host arrays) to the group of its dim, opening the
// group (an internal context on our device, with a stream of its own) if new.
void group_add(wlseno_ctx *c, int dim, int64_t nv, const double *xyz, int64_t nc, const int32_t *cells, int32_t id)
{
    size_t gi = 0;
    while (gi < c->groups.size() && c->groups[gi].dim != dim) ++gi;
    if (gi == c->groups.size()) {
        wlseno_ctx::Group g;
        g.dim = dim;
        if (wlseno_create(c->device, nullptr, &g.c) != WLSENO_OK)
            throw Error{WLSENO_EDEVICE, wlseno_last_error(nullptr)};
        c->groups.push_back(g);
        wlseno_ctx::Group &gr = c->groups.back();
        gr.c->step_mode = c->step_mode;
        gr.c->use_graphs = c->use_graphs;
        if (c->device >= 0) {
            check_hip(hipSetDevice(c->device), "hipSetDevice");
            check_hip(hipStreamCreateWithFlags(&gr.st, hipStreamNonBlocking), "hipStreamCreateWithFlags");
            check_hip(hipEventCreateWithFlags(&gr.done, hipEventDisableTiming), "hipEventCreateWithFlags");
            check_child(gr.c, wlseno_set_stream(gr.c, gr.st), dim);
        }
    }
    wlseno_ctx::Group &g = c->groups[gi];
    check_child(g.c, wlseno_batch_add_mesh(g.c, dim, nv, xyz, nc, cells, nullptr), dim);
    g.meshes.push_back(id);
    c->mesh_group.push_back((int32_t)gi);
}

// The meshes added so far (one dim) become the first group.
void enter_mixed(wlseno_ctx *c)
{
    const int d = c->batch_dim;
    int64_t nv0 = 0, nc0 = 0;
    for (size_t k = 0; k < c->parts.size(); ++k) {
        const auto &pt = c->parts[k];
        std::vector<int32_t> cl((size_t)pt.nc * (d + 1));
        for (size_t t = 0; t < cl.size(); ++t) cl[t] = c->batch_cells[(size_t)nc0 * (d + 1) + t] - (int32_t)nv0;
        group_add(c, d, pt.nv, c->batch_xyz.data() + (size_t)nv0 * d, pt.nc, cl.data(), (int32_t)k);
        nv0 += pt.nv;
        nc0 += pt.nc;
    }
    c->batch_xyz.clear();
    c->batch_cells.clear();
    c->batch_h.clear();
}

// First cell of each batch mesh in the caller's arrays (add order), and the total.
std::vector<int64_t> mesh_cell0(const wlseno_ctx *c)
{
    std::vector<int64_t> c0(c->parts.size() + 1, 0);
    for (size_t k = 0; k < c->parts.size(); ++k) c0[k + 1] = c0[k] + c->parts[k].nc;
    return c0;
}

// For group g: the caller's cell index of each of its user cells (its meshes
// concatenated in add order).
std::vector<int64_t> group_to_caller(const wlseno_ctx *c, const wlseno_ctx::Group &g)
{
    const std::vector<int64_t> c0 = mesh_cell0(c);
    std::vector<int64_t> out;
    for (int32_t k : g.meshes)
        for (int64_t i = c0[k]; i < c0[k + 1]; ++i) out.push_back(i);
    return out;
}

// Work of every group on its own stream, ordered after the caller's stream
// and joined back into it.
void fork_groups(wlseno_ctx *c)
{
    if (!c->fork) check_hip(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming), "hipEventCreateWithFlags");
    check_hip(hipEventRecord(c->fork, c->stream), "hipEventRecord");
    for (auto &g : c->groups) check_hip(hipStreamWaitEvent(g.st, c->fork, 0), "hipStreamWaitEvent");
}

void join_groups(wlseno_ctx *c)
{
    for (auto &g : c->groups) {
        check_hip(hipEventRecord(g.done, g.st), "hipEventRecord");
        check_hip(hipStreamWaitEvent(c->stream, g.done, 0), "hipStreamWaitEvent");
    }
}

// fork_groups on construction; join_groups on join() or, if a group's call
// threw first, on destruction, so that the caller's stream is always joined.
struct GroupRun {
    wlseno_ctx *c;
    bool joined = false;
    explicit GroupRun(wlseno_ctx *ctx) : c(ctx) { fork_groups(c); }
    void join()
    {
        joined = true;
        join_groups(c);
    }
    ~GroupRun()
    {
        if (!joined) {
            try {
                join_groups(c);
            } catch (...) {
            }
        }
    }
};

void need_single_dim(const wlseno_ctx *c, const char *what)
{
    if (mixed(c)) throw Error{WLSENO_EUNSUPPORTED, std::string(what) + " works on batches of one dim only"};
}

}  // namespace

extern "C" {

void wlseno_params_default(wlseno_params *out)
{
    if (!out) return;
    std::memset(out, 0, sizeof(*out));
    out->p = 3;
    out->n_lo = 12;
    out->n_hi = 20;
    out->flux = WLSENO_FLUX_ADVECTION;
    out->weight_mode = 0;
    out->eps = 1e-2;
    out->alpha_w = 1.5;
    out->rank_tol = 1e-12;
    out->velocity[0] = 1.0;
    out->gamma = 1.4;
    out->bc = 0;
    out->characteristic = 0;
    out->balance = 0;
    out->lf_alpha = 0;
    out->h_mode = 0;
    for (int v = 0; v < 5; ++v) out->far_state[v] = 0.0;
}

wlseno_status wlseno_create(int device, void *hip_stream, wlseno_t *out)
{
    if (!out) return WLSENO_EINVAL;
    *out = nullptr;
    g_create_error.clear();
    if (device == -1 && hip_stream) {
        g_create_error = "a host-only context takes no stream";
        return WLSENO_EINVAL;
    }
    if (device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || device >= n) {
            g_create_error = "no HIP device " + std::to_string(device);
            return WLSENO_EDEVICE;
        }
        e = hipSetDevice(device);
        if (e != hipSuccess) {
            g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
            return WLSENO_EDEVICE;
        }
    } else if (device != -1) {
        g_create_error = "device must be >= 0, or -1 for a host-only context";
        return WLSENO_EINVAL;
    }
    void *scr = nullptr;
    if (device >= 0) {
        const int e = scratch_address(device, &scr);
        if (e != 0) {
            g_create_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString((hipError_t)e);
            return WLSENO_EDEVICE;
        }
    }
    wlseno_ctx *c = new (std::nothrow) wlseno_ctx;
    if (!c) return WLSENO_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->scratch = (unsigned char *)scr;
    *out = c;
    return WLSENO_OK;
}

wlseno_status wlseno_destroy(wlseno_t ctx)
{
    if (!ctx) return WLSENO_OK;
    drop_groups(ctx);
    free_device(ctx);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    if (ctx->nf_first) (void)hipFree(ctx->nf_first);
    delete ctx;
    return WLSENO_OK;
}

wlseno_status wlseno_set_numeric_check(wlseno_t ctx, int enable)
{
    API_BEGIN(ctx)
    if (enable && ctx->device >= 0 && !ctx->nf_first) {
        check_hip(hipSetDevice(ctx->device), "hipSetDevice");
        void *p = nullptr;
        if (hipMalloc(&p, sizeof(unsigned long long)) != hipSuccess)
            throw Error{WLSENO_ENOMEM, "device allocation failed (numeric check word)"};
        ctx->nf_first = (unsigned long long *)p;
    }
    ctx->check_numeric = enable != 0;
    API_END(ctx)
}

wlseno_status wlseno_set_graphs(wlseno_t ctx, int enable)
{
    API_BEGIN(ctx)
    ctx->use_graphs = enable != 0;
    ctx->step_mode = enable ? 1 : 0;
    if (!ctx->use_graphs) drop_graph(ctx);
    for (auto &g : ctx->groups) check_child(g.c, wlseno_set_graphs(g.c, enable), g.dim);
    API_END(ctx)
}

wlseno_status wlseno_set_step_mode(wlseno_t ctx, int mode)
{
    API_BEGIN(ctx)
    if (mode < 0 || mode > 2) throw Error{WLSENO_EINVAL, "step mode must be 0, 1 or 2"};
    ctx->step_mode = mode;
    ctx->use_graphs = mode == 1;
    if (!ctx->use_graphs) drop_graph(ctx);
    for (auto &g : ctx->groups) check_child(g.c, wlseno_set_step_mode(g.c, mode), g.dim);
    API_END(ctx)
}

const char *wlseno_last_error(wlseno_t ctx)
{
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

wlseno_status wlseno_set_stream(wlseno_t ctx, void *hip_stream)
{
    API_BEGIN(ctx)
    if (ctx->device < 0) throw Error{WLSENO_ESTATE, "host-only context has no stream"};
    ctx->stream = (hipStream_t)hip_stream;
    API_END(ctx)
}

wlseno_status wlseno_mesh_upload(wlseno_t ctx, int dim, int64_t n_vert, const double *xyz, int64_t n_cell,
                                 const int32_t *cells, uint32_t flags)
{
    API_BEGIN(ctx)
    HostMesh m;
    mesh_setup(m, dim, n_vert, xyz, n_cell, cells, flags);
    drop_groups(ctx);
    free_device(ctx);
    ctx->mesh = std::move(m);
    ctx->have_mesh = true;
    ctx->have_build = false;
    ctx->build = Build{};
    ctx->parts.clear();
    ctx->batch_xyz.clear();
    ctx->batch_cells.clear();
    ctx->batch_h.clear();
    ctx->batch_pending = false;
    API_END(ctx)
}

wlseno_status wlseno_batch_add_mesh(wlseno_t ctx, int dim, int64_t n_vert, const double *xyz, int64_t n_cell,
                                    const int32_t *cells, int32_t *mesh_id)
{
    API_BEGIN(ctx)
    // validates the mesh on its own and gives its mean edge length
    HostMesh one;
    mesh_setup(one, dim, n_vert, xyz, n_cell, cells, 0);
    int64_t nv0 = 0, nc0 = 0;
    for (const auto &pt : ctx->parts) {
        nv0 += pt.nv;
        nc0 += pt.nc;
    }
    if (nc0 + n_cell > (int64_t)(INT32_MAX / 8) || nv0 + n_vert > (int64_t)INT32_MAX)
        throw Error{WLSENO_EINVAL, "batch too large for 32-bit indices"};
    if (!ctx->parts.empty() && dim != ctx->batch_dim && !mixed(ctx)) enter_mixed(ctx);
    if (mixed(ctx)) {
        group_add(ctx, dim, n_vert, xyz, n_cell, cells, (int32_t)ctx->parts.size());
        ctx->parts.push_back({n_vert, n_cell});
        free_device(ctx);
        ctx->mesh = HostMesh{};
        ctx->have_mesh = true;
        ctx->have_build = false;
        ctx->build = Build{};
        ctx->batch_pending = false;
        if (mesh_id) *mesh_id = (int32_t)ctx->parts.size() - 1;
        return WLSENO_OK;
    }
    ctx->batch_dim = dim;
    ctx->batch_xyz.insert(ctx->batch_xyz.end(), xyz, xyz + n_vert * dim);
    for (int64_t t = 0; t < n_cell * (dim + 1); ++t) ctx->batch_cells.push_back((int32_t)(cells[t] + nv0));
    ctx->parts.push_back({n_vert, n_cell});
    ctx->batch_h.push_back(one.h);
    // the union (disjoint meshes, so stencils stay within a mesh) is set up
    // once, by the next stencil build: adding n meshes stays linear in size
    free_device(ctx);
    ctx->mesh = HostMesh{};
    ctx->have_mesh = true;
    ctx->have_build = false;
    ctx->build = Build{};
    ctx->batch_pending = true;
    if (mesh_id) *mesh_id = (int32_t)ctx->parts.size() - 1;
    API_END(ctx)
}

wlseno_status wlseno_batch_params(wlseno_t ctx, int dim, const wlseno_params *params)
{
    API_BEGIN(ctx)
    if (dim < 1 || dim > 3) throw Error{WLSENO_EINVAL, "dim must be 1, 2 or 3"};
    ctx->has_dim_prm[dim] = params != nullptr;
    if (params) ctx->dim_prm[dim] = *params;
    ctx->have_build = false;
    API_END(ctx)
}

wlseno_status wlseno_stencil_build(wlseno_t ctx, const wlseno_params *params)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_stencil_build");
    if (!params) throw Error{WLSENO_EINVAL, "params is NULL"};
    if (!ctx->have_mesh) throw Error{WLSENO_ESTATE, "call wlseno_mesh_upload first"};
    if (mixed(ctx)) {
        ctx->have_build = false;
        int nvars = -1;
        for (auto &g : ctx->groups) {
            const wlseno_params &prm = ctx->has_dim_prm[g.dim] ? ctx->dim_prm[g.dim] : *params;
            check_child(g.c, wlseno_stencil_build(g.c, &prm), g.dim);
            if (nvars >= 0 && g.c->build.nvars != nvars)
                throw Error{WLSENO_EINVAL, "the meshes of a batch need the same number of field components"};
            nvars = g.c->build.nvars;
        }
        if (ctx->device >= 0) {
            // each group's device cells map straight to the caller's cells
            const int64_t total = mesh_cell0(ctx).back();
            for (auto &g : ctx->groups) {
                const std::vector<int64_t> to = group_to_caller(ctx, g);
                std::vector<int32_t> gp(g.c->build.perm.size());
                for (size_t d = 0; d < gp.size(); ++d) gp[d] = (int32_t)to[g.c->build.perm[d]];
                g.c->dm.perm = upload(g.c, gp);
                g.c->dm.user_stride = total;
            }
        }
        ctx->build = Build{};
        ctx->build.prm = *params;
        ctx->build.nvars = nvars;
        ctx->have_build = true;
        return WLSENO_OK;
    }
    const bool per_dim = !ctx->parts.empty() && ctx->has_dim_prm[ctx->batch_dim];
    if (per_dim) params = &ctx->dim_prm[ctx->batch_dim];
    if (ctx->batch_pending) {
        int64_t nv = 0, nc = 0;
        for (const auto &pt : ctx->parts) {
            nv += pt.nv;
            nc += pt.nc;
        }
        HostMesh m;
        mesh_setup(m, ctx->batch_dim, nv, ctx->batch_xyz.data(), nc, ctx->batch_cells.data(), 0);
        m.nmesh = (int)ctx->parts.size();
        if (m.nmesh > 1) {
            m.mesh_h = ctx->batch_h;
            m.mesh_of.resize(m.nc);
            int64_t at = 0;
            for (int k = 0; k < m.nmesh; ++k)
                for (int64_t i = 0; i < ctx->parts[k].nc; ++i) m.mesh_of[at++] = k;
        }
        ctx->mesh = std::move(m);
        ctx->batch_pending = false;
    }
    ctx->have_build = false;
    Build b;
    build_setup(ctx->mesh, *params, b);
    ctx->build = std::move(b);
    if (ctx->device >= 0) upload_build(ctx);
    ctx->have_build = true;
    API_END(ctx)
}

wlseno_status wlseno_get_info(wlseno_t ctx, wlseno_info *out)
{
    API_BEGIN(ctx)
    if (!out) throw Error{WLSENO_EINVAL, "out is NULL"};
    if (!ctx->have_build) throw Error{WLSENO_ESTATE, "call wlseno_stencil_build first"};
    std::memset(out, 0, sizeof(*out));
    if (mixed(ctx)) {
        // several dims: totals and extremes over the groups; per-dim sizes are 0
        out->min_stencil = INT32_MAX;
        out->min_insphere = INFINITY;
        for (auto &g : ctx->groups) {
            const Build &gb = g.c->build;
            out->n_vars = gb.nvars;
            out->min_stencil = std::min(out->min_stencil, gb.min_stencil);
            out->max_stencil = std::max(out->max_stencil, gb.max_stencil);
            out->n_cell += g.c->mesh.nc;
            out->nnz += (int64_t)gb.col.size();
            out->min_insphere = std::min(out->min_insphere, gb.min_insphere);
        }
        out->n_mesh = (int32_t)ctx->parts.size();
        return WLSENO_OK;
    }
    const Build &b = ctx->build;
    out->dim = ctx->mesh.dim;
    out->m = b.m;
    out->n_vars = b.nvars;
    out->faces_per_cell = b.nf;
    out->points_per_face = b.nq;
    out->min_stencil = b.min_stencil;
    out->max_stencil = b.max_stencil;
    out->n_mesh = ctx->mesh.nmesh;
    out->n_cell = ctx->mesh.nc;
    out->nnz = (int64_t)b.col.size();
    out->h = ctx->mesh.h;
    out->min_insphere = b.min_insphere;
    API_END(ctx)
}

wlseno_status wlseno_get_stencil(wlseno_t ctx, int32_t *row_ptr, int32_t *col)
{
    API_BEGIN(ctx)
    if (!row_ptr || !col) throw Error{WLSENO_EINVAL, "null output array"};
    if (!ctx->have_build) throw Error{WLSENO_ESTATE, "call wlseno_stencil_build first"};
    if (mixed(ctx)) {
        // the caller's cell order and ids: each mesh's rows from its group
        const std::vector<int64_t> c0 = mesh_cell0(ctx);
        std::vector<std::vector<int64_t>> to(ctx->groups.size());
        std::vector<std::vector<int64_t>> first(ctx->groups.size());   // group user index of each mesh's first cell
        for (size_t gi = 0; gi < ctx->groups.size(); ++gi) {
            to[gi] = group_to_caller(ctx, ctx->groups[gi]);
            int64_t at = 0;
            for (int32_t k : ctx->groups[gi].meshes) {
                first[gi].push_back(at);
                at += c0[k + 1] - c0[k];
            }
        }
        std::vector<int32_t> pos(ctx->parts.size());   // position of each mesh within its group
        for (size_t gi = 0; gi < ctx->groups.size(); ++gi)
            for (size_t t = 0; t < ctx->groups[gi].meshes.size(); ++t) pos[ctx->groups[gi].meshes[t]] = (int32_t)t;
        int64_t w = 0;
        row_ptr[0] = 0;
        for (size_t k = 0; k < ctx->parts.size(); ++k) {
            const int gi = ctx->mesh_group[k];
            const Build &gb = ctx->groups[gi].c->build;
            for (int64_t i = c0[k]; i < c0[k + 1]; ++i) {
                const int64_t ui = first[gi][pos[k]] + (i - c0[k]);
                for (int32_t t = gb.row_ptr[ui]; t < gb.row_ptr[ui + 1]; ++t) col[w++] = (int32_t)to[gi][gb.col[t]];
                row_ptr[i + 1] = (int32_t)w;
            }
        }
        return WLSENO_OK;
    }
    std::memcpy(row_ptr, ctx->build.row_ptr.data(), ctx->build.row_ptr.size() * sizeof(int32_t));
    std::memcpy(col, ctx->build.col.data(), ctx->build.col.size() * sizeof(int32_t));
    API_END(ctx)
}

wlseno_status wlseno_reconstruct(wlseno_t ctx, const double *u_dev, double *coef_dev, double *facevals_dev,
                                 int32_t *rank_dev)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_reconstruct");
    if (!u_dev) throw Error{WLSENO_EINVAL, "u_dev is NULL"};
    need_single_dim(ctx, "wlseno_reconstruct (per-dim coefficient and facet layouts)");
    if (coef_dev && ctx->have_build && ctx->build.prm.characteristic)
        throw Error{WLSENO_EINVAL, "no coefficient output with characteristic fields (one fit per facet)"};
    need_device(ctx);
    numeric_check(ctx, u_dev, (int64_t)ctx->dm.nvars * ctx->dm.nc, ctx->dm.nc, 1, "input average");
    check_launch(launch_permute(ctx->dm, u_dev, ctx->ubuf, true, ctx->stream), "permute");
    check_launch(launch_clear_alpha(ctx->dm, ctx->stream), "clear");
    check_launch(launch_reconstruct(ctx->dm, ctx->ubuf, 0, coef_dev, facevals_dev, rank_dev, ctx->stream),
                 "reconstruct");
    ctx->last_parity = 0;
    {
        const DevMesh &d = ctx->dm;
        const int per_f = d.nf * d.nq;
        numeric_check(ctx, facevals_dev, (int64_t)d.nvars * d.nc * per_f, d.nc, per_f, "facet value");
        numeric_check(ctx, coef_dev, (int64_t)d.nvars * d.nc * d.m, d.nc, d.m, "coefficient");
    }
    API_END(ctx)
}

wlseno_status wlseno_rhs(wlseno_t ctx, const double *u_dev, double *dudt_dev)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_rhs");
    if (!u_dev || !dudt_dev) throw Error{WLSENO_EINVAL, "null device pointer"};
    if (u_dev == dudt_dev) throw Error{WLSENO_EINVAL, "dudt_dev must not alias u_dev"};
    need_device(ctx);
    numeric_check(ctx, u_dev, user_vars(ctx) * user_cells(ctx), user_cells(ctx), 1, "input average");
    if (mixed(ctx)) {
        GroupRun run(ctx);
        for (auto &g : ctx->groups) check_child(g.c, wlseno_rhs(g.c, u_dev, dudt_dev), g.dim);
        run.join();
    } else {
        check_launch(launch_permute(ctx->dm, u_dev, ctx->ubuf, true, ctx->stream), "permute");
        check_launch(launch_clear_alpha(ctx->dm, ctx->stream), "clear");
        stage(ctx, ctx->ubuf, nullptr, nullptr, ctx->tbuf, 0.0, 0.0, 1.0, 0, 0, ctx->stream);
        check_launch(launch_permute(ctx->dm, ctx->tbuf, dudt_dev, false, ctx->stream), "permute");
    }
    numeric_check(ctx, dudt_dev, user_vars(ctx) * user_cells(ctx), user_cells(ctx), 1, "right-hand side");
    API_END(ctx)
}

wlseno_status wlseno_rhs_noalloc(wlseno_t ctx, const double *u_dev, double *dudt_dev)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_rhs_noalloc");
    if (!u_dev || !dudt_dev) throw Error{WLSENO_EINVAL, "null device pointer"};
    if (u_dev == dudt_dev) throw Error{WLSENO_EINVAL, "dudt_dev must not alias u_dev"};
    need_device(ctx);
    numeric_check(ctx, u_dev, user_vars(ctx) * user_cells(ctx), user_cells(ctx), 1, "input average");
    if (mixed(ctx)) {
        // the groups share this device's array: one after another, on our stream
        for (auto &g : ctx->groups) {
            check_child(g.c, wlseno_set_stream(g.c, ctx->stream), g.dim);
            const wlseno_status st = wlseno_rhs_noalloc(g.c, u_dev, dudt_dev);
            (void)wlseno_set_stream(g.c, g.st);
            check_child(g.c, st, g.dim);
        }
        numeric_check(ctx, dudt_dev, user_vars(ctx) * user_cells(ctx), user_cells(ctx), 1, "right-hand side");
        return WLSENO_OK;
    }
    if (ctx->dm.balance) throw Error{WLSENO_EUNSUPPORTED, "the balanced refit keeps buffers of its own"};
    if (!ctx->scratch) throw Error{WLSENO_ESTATE, "no scratch address on this device"};
    // scratch layout: alpha slots (two parities), state and result in device
    // order, facet values; each part 256-byte aligned
    const DevMesh &cm = ctx->dm;
    auto up256 = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t a_bytes = up256(2 * (size_t)cm.alpha_slots() * 16 * sizeof(unsigned long long));
    const size_t u_bytes = up256((size_t)cm.nvars * cm.nc * sizeof(double));
    const size_t f_bytes = up256((size_t)cm.nvars * cm.nc * cm.nf * cm.nq * sizeof(double));
    const size_t need = a_bytes + 2 * u_bytes + f_bytes;
    if (need > scratch_capacity())
        throw Error{WLSENO_EINVAL, "this mesh needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                       std::to_string(scratch_capacity()) + " of the allocation-free entry point"};
    DevMesh dm = cm;
    dm.alpha = (unsigned long long *)ctx->scratch;
    double *ub = (double *)(ctx->scratch + a_bytes);
    double *tb = (double *)(ctx->scratch + a_bytes + u_bytes);
    dm.fv = (double *)(ctx->scratch + a_bytes + 2 * u_bytes);
    check_launch(launch_permute(dm, u_dev, ub, true, ctx->stream), "permute");
    check_launch(launch_clear_alpha(dm, ctx->stream), "clear");
    check_launch(launch_reconstruct(dm, ub, 0, nullptr, nullptr, nullptr, ctx->stream), "reconstruct");
    check_launch(launch_update(dm, nullptr, nullptr, tb, 0.0, 0.0, 1.0, 0, 0, ctx->stream), "update");
    check_launch(launch_permute(dm, tb, dudt_dev, false, ctx->stream), "permute");
    numeric_check(ctx, dudt_dev, user_vars(ctx) * user_cells(ctx), user_cells(ctx), 1, "right-hand side");
    API_END(ctx)
}

namespace {

// Transposed-stencil tables and cotangent buffers, built on first use.
void adjoint_setup(wlseno_ctx *c)
{
    if (c->adj_ready) return;
    if (!adjoint_supported(c->dm))
        throw Error{WLSENO_EUNSUPPORTED, "the adjoint covers scalar linear advection on a single mesh"};
    std::vector<int64_t> tptr;
    std::vector<int32_t> tpos;
    transpose_tables(c->build, c->dm.nc, c->dm.nf, tptr, tpos);
    c->tptr = upload(c, tptr);
    c->tpos = upload(c, tpos);
    c->contrib = (double *)dev_alloc(c, (size_t)tptr.back() * sizeof(double));
    c->ga = (double *)dev_alloc(c, c->dm.nc * sizeof(double));
    c->gb = (double *)dev_alloc(c, c->dm.nc * sizeof(double));
    c->gc = (double *)dev_alloc(c, c->dm.nc * sizeof(double));
    c->adj_ready = true;
}

// out = A x + B y + C z + D J(u)^T v (device order; null vectors count as zero).
void vjp(wlseno_ctx *c, const double *u, const double *v, const double *x, const double *y, const double *z,
         double *out, double A, double B, double C, double D)
{
    check_launch(launch_adjoint(c->dm, u, v, c->tpos, c->contrib, c->stream), "adjoint");
    check_launch(launch_adjoint_gather(c->dm, c->tptr, c->contrib, x, y, z, out, A, B, C, D, c->stream),
                 "adjoint gather");
}

}  // namespace

wlseno_status wlseno_rhs_vjp(wlseno_t ctx, const double *u_dev, const double *v_dev, double *out_dev)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_rhs_vjp");
    if (!u_dev || !v_dev || !out_dev) throw Error{WLSENO_EINVAL, "null device pointer"};
    if (out_dev == u_dev || out_dev == v_dev) throw Error{WLSENO_EINVAL, "out_dev must not alias an input"};
    need_device(ctx);
    adjoint_setup(ctx);
    check_launch(launch_permute(ctx->dm, u_dev, ctx->ubuf, true, ctx->stream), "permute");
    check_launch(launch_permute(ctx->dm, v_dev, ctx->ga, true, ctx->stream), "permute");
    vjp(ctx, ctx->ubuf, ctx->ga, nullptr, nullptr, nullptr, ctx->gb, 0.0, 0.0, 0.0, 1.0);
    check_launch(launch_permute(ctx->dm, ctx->gb, out_dev, false, ctx->stream), "permute");
    API_END(ctx)
}

namespace {

// Forward sweep from the device-order state in ubuf: store the state at the
// start of every segment of ckpt_every steps, and advance to step n_steps
// (advance_last) or only to the start of the last segment.
void forward_checkpoints(wlseno_ctx *ctx, double dt, int n_steps, int ckpt_every, bool advance_last)
{
    const int64_t nc = ctx->dm.nc;
    const int nseg = n_steps == 0 ? 0 : (n_steps + ckpt_every - 1) / ckpt_every;
    const int E = n_steps < ckpt_every ? n_steps : ckpt_every;
    dev_grow(ctx, &ctx->ck, &ctx->ck_cap, (size_t)(nseg > 0 ? nseg : 1) * nc);
    dev_grow(ctx, &ctx->seg, &ctx->seg_cap, (size_t)(E > 0 ? E : 1) * 3 * nc);
    ctx->rec_valid = false;
    const size_t bytes = (size_t)nc * sizeof(double);
    for (int sg = 0; sg < nseg; ++sg) {
        check_hip(hipMemcpyAsync(ctx->ck + (size_t)sg * nc, ctx->ubuf, bytes, hipMemcpyDeviceToDevice, ctx->stream),
                  "hipMemcpyAsync");
        const int s_end = (sg + 1) * ckpt_every < n_steps ? (sg + 1) * ckpt_every : n_steps;
        if (sg + 1 < nseg || advance_last)
            for (int s = sg * ckpt_every; s < s_end; ++s) rk3_step(ctx, dt, 0, ctx->stream);
    }
}

// Reverse sweep over the stored checkpoints, segment by segment: recompute
// the segment's stage states, then transpose each RK3 step (g = cotangent of
// the step's output):
//   g2 = 2/3 g + 2/3 dt J(U2)^T g;  g1 = 1/4 g2 + 1/4 dt J(U1)^T g2;
//   g  = 1/3 g + 3/4 g2 + g1 + dt J(U)^T g1
void reverse_sweep(wlseno_ctx *ctx, double dt, int n_steps, int ckpt_every, const double *gT_dev, double *g0_dev)
{
    const int64_t nc = ctx->dm.nc;
    const int nseg = n_steps == 0 ? 0 : (n_steps + ckpt_every - 1) / ckpt_every;
    const size_t bytes = (size_t)nc * sizeof(double);
    double *u = ctx->ubuf;
    double *g = ctx->ga, *g2 = ctx->gb, *g1 = ctx->gc;
    check_launch(launch_permute(ctx->dm, gT_dev, g, true, ctx->stream), "permute");
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int s0 = sg * ckpt_every;
        const int ns = (s0 + ckpt_every < n_steps ? s0 + ckpt_every : n_steps) - s0;
        check_hip(hipMemcpyAsync(u, ctx->ck + (size_t)sg * nc, bytes, hipMemcpyDeviceToDevice, ctx->stream),
                  "hipMemcpyAsync");
        for (int t = 0; t < ns; ++t) {
            double *U = ctx->seg + (size_t)(3 * t) * nc, *U1 = U + nc, *U2 = U1 + nc;
            check_hip(hipMemcpyAsync(U, u, bytes, hipMemcpyDeviceToDevice, ctx->stream), "hipMemcpyAsync");
            stage(ctx, U, U, U, U1, 1.0, 0.0, dt, 1, 0, ctx->stream);
            stage(ctx, U1, U, U1, U2, 0.75, 0.25, 0.25 * dt, 1, 0, ctx->stream);
            if (t + 1 < ns) stage(ctx, U2, U, U2, u, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0 * dt, 1, 0, ctx->stream);
        }
        for (int t = ns - 1; t >= 0; --t) {
            const double *U = ctx->seg + (size_t)(3 * t) * nc, *U1 = U + nc, *U2 = U1 + nc;
            vjp(ctx, U2, g, g, nullptr, nullptr, g2, 2.0 / 3.0, 0.0, 0.0, 2.0 / 3.0 * dt);
            vjp(ctx, U1, g2, g2, nullptr, nullptr, g1, 0.25, 0.0, 0.0, 0.25 * dt);
            vjp(ctx, U, g1, g, g2, g1, g, 1.0 / 3.0, 0.75, 1.0, dt);
        }
    }
    check_launch(launch_permute(ctx->dm, g, g0_dev, false, ctx->stream), "permute");
}

void check_adjoint_args(double dt, int n_steps, int ckpt_every)
{
    if (!std::isfinite(dt) || n_steps < 0 || ckpt_every < 1)
        throw Error{WLSENO_EINVAL, "dt finite, n_steps >= 0 and ckpt_every >= 1 required"};
}

}  // namespace

wlseno_status wlseno_step_adjoint(wlseno_t ctx, const double *u0_dev, double dt, int n_steps, int ckpt_every,
                                  const double *gT_dev, double *g0_dev)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_step_adjoint");
    if (!u0_dev || !gT_dev || !g0_dev) throw Error{WLSENO_EINVAL, "null device pointer"};
    check_adjoint_args(dt, n_steps, ckpt_every);
    need_device(ctx);
    adjoint_setup(ctx);
    check_launch(launch_permute(ctx->dm, u0_dev, ctx->ubuf, true, ctx->stream), "permute");
    // the last segment's states are recomputed by the reverse sweep anyway
    forward_checkpoints(ctx, dt, n_steps, ckpt_every, false);
    reverse_sweep(ctx, dt, n_steps, ckpt_every, gT_dev, g0_dev);
    API_END(ctx)
}

wlseno_status wlseno_step_record(wlseno_t ctx, double *u_dev, double dt, int n_steps, int ckpt_every)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_step_record");
    if (!u_dev) throw Error{WLSENO_EINVAL, "u_dev is NULL"};
    check_adjoint_args(dt, n_steps, ckpt_every);
    need_device(ctx);
    adjoint_setup(ctx);
    check_launch(launch_permute(ctx->dm, u_dev, ctx->ubuf, true, ctx->stream), "permute");
    forward_checkpoints(ctx, dt, n_steps, ckpt_every, true);
    check_launch(launch_permute(ctx->dm, ctx->ubuf, u_dev, false, ctx->stream), "permute");
    ctx->rec_valid = true;
    ctx->rec_dt = dt;
    ctx->rec_n = n_steps;
    ctx->rec_ckpt = ckpt_every;
    API_END(ctx)
}

wlseno_status wlseno_step_adjoint_recorded(wlseno_t ctx, const double *gT_dev, double *g0_dev)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_step_adjoint_recorded");
    if (!gT_dev || !g0_dev) throw Error{WLSENO_EINVAL, "null device pointer"};
    need_device(ctx);
    if (!ctx->rec_valid) throw Error{WLSENO_ESTATE, "no recorded trajectory (wlseno_step_record first)"};
    reverse_sweep(ctx, ctx->rec_dt, ctx->rec_n, ctx->rec_ckpt, gT_dev, g0_dev);
    API_END(ctx)
}

namespace {

// n_steps of TVD RK3; dt_mesh (batches) holds one time step per mesh.
void run_steps(wlseno_ctx *ctx, double *u_dev, double dt, const double *dt_mesh, int n_steps)
{
    const bool batch = ctx->dm.nmesh > 1;
    // the time steps go to device memory (one per mesh), read there by the
    // stepping kernels so that captured graphs hold none; only the persistent
    // kernel on one mesh takes its time step as an argument
    if (batch || ctx->step_mode != 2) {
        bool changed = false;
        for (int k = 0; k < ctx->dm.nmesh; ++k) {
            const double v = dt_mesh ? dt_mesh[k] : dt;
            if (!std::isfinite(v)) throw Error{WLSENO_EINVAL, "time steps must be finite"};
            changed = changed || !(ctx->dt_host[k] == v);
            ctx->dt_host[k] = v;
        }
        if (changed)
            check_hip(hipMemcpyAsync(ctx->dm.dt_tab, ctx->dt_host.data(), ctx->dt_host.size() * sizeof(double),
                                     hipMemcpyHostToDevice, ctx->stream),
                      "hipMemcpyAsync");
    }
    // stage coefficients c (times dt in the kernel), or c dt for the persistent
    // kernel on one mesh
    const double h = (batch || ctx->step_mode != 2) ? 1.0 : dt;
    if (ctx->step_mode == 2 && !steps_supported(ctx->dm))
        throw Error{WLSENO_EUNSUPPORTED, "the persistent step kernel is compiled for 2-D p = 3 scalar fluxes with "
                                         "2 lanes per cell and no balanced refit"};
    if (ctx->use_graphs && ctx->step_mode != 2 && n_steps >= 2) {
        // the whole ladder is captured together the first time any graph is
        // needed for this h, so that later runs of other lengths capture
        // nothing.  On meshes small enough for launch overhead to matter,
        // each new graph is also replayed once here, on whatever the state
        // buffers hold (the state is copied in below): a graph's first replay
        // costs ~35 us more than later ones on the 19,602-triangle benchmark.
        bool fresh = false;
        for (int g = 0; g < kGraphLadder; ++g) {
            fresh = fresh || !ctx->graph[g] || std::memcmp(&ctx->graph_h[g], &h, sizeof h) != 0;
            (void)steps_graph(ctx, h, g);
        }
        if (fresh && ctx->dm.nc <= kPrereplayCells)
            for (int g = 0; g < kGraphLadder; ++g)
                check_hip(hipGraphLaunch(ctx->graph[g], ctx->stream), "hipGraphLaunch");
    }
    check_launch(launch_permute(ctx->dm, u_dev, ctx->ubuf, true, ctx->stream), "permute");
    check_launch(launch_clear_alpha(ctx->dm, ctx->stream), "clear");
    if (ctx->step_mode == 2) {
        if (!ctx->sync) ctx->sync = (unsigned *)dev_alloc(ctx, 64 * sizeof(unsigned));
        check_launch(launch_steps(ctx->dm, ctx->ubuf, ctx->kbuf, h, n_steps, ctx->sync, ctx->stream), "steps");
        check_launch(launch_permute(ctx->dm, ctx->ubuf, u_dev, false, ctx->stream), "permute");
        ctx->last_parity = (3 * n_steps - 1) & 1;
        unsigned failed = 0;
        check_hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        check_hip(hipMemcpy(&failed, ctx->sync + 32, sizeof failed, hipMemcpyDeviceToHost), "hipMemcpy");
        if (failed) throw Error{WLSENO_EDEVICE, "persistent step kernel: a device-wide barrier timed out"};
        return;
    }
    int s = 0;
    if (ctx->use_graphs && n_steps >= 2) {
        for (int g = 0; g < kGraphLadder; ++g) {
            const int k = kGraphSteps[g];
            for (; s + k <= n_steps; s += k) check_hip(hipGraphLaunch(ctx->graph[g], ctx->stream), "hipGraphLaunch");
        }
        ctx->last_parity = 1;
    }
    for (; s < n_steps; ++s) rk3_step(ctx, h, s & 1 ? 1 : 0, ctx->stream, !batch);
    check_launch(launch_permute(ctx->dm, ctx->ubuf, u_dev, false, ctx->stream), "permute");
}

}  // namespace

wlseno_status wlseno_step(wlseno_t ctx, double *u_dev, double dt, int n_steps)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_step");
    if (!u_dev) throw Error{WLSENO_EINVAL, "u_dev is NULL"};
    if (!std::isfinite(dt) || n_steps < 0) throw Error{WLSENO_EINVAL, "dt must be finite and n_steps >= 0"};
    need_device(ctx);
    if (n_steps == 0) return WLSENO_OK;
    numeric_check(ctx, u_dev, user_vars(ctx) * user_cells(ctx), user_cells(ctx), 1, "input average");
    if (mixed(ctx)) {
        GroupRun run(ctx);
        for (auto &g : ctx->groups) check_child(g.c, wlseno_step(g.c, u_dev, dt, n_steps), g.dim);
        run.join();
    } else {
        run_steps(ctx, u_dev, dt, nullptr, n_steps);
    }
    numeric_check(ctx, u_dev, user_vars(ctx) * user_cells(ctx), user_cells(ctx), 1, "state");
    API_END(ctx)
}

wlseno_status wlseno_batch_step(wlseno_t ctx, double *u_dev, const double *dt_per_mesh, int n_steps)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_batch_step");
    if (!u_dev || !dt_per_mesh) throw Error{WLSENO_EINVAL, "null pointer"};
    if (n_steps < 0) throw Error{WLSENO_EINVAL, "n_steps >= 0 required"};
    need_device(ctx);
    if (n_steps > 0) numeric_check(ctx, u_dev, user_vars(ctx) * user_cells(ctx), user_cells(ctx), 1, "input average");
    if (mixed(ctx)) {
        for (size_t k = 0; k < ctx->parts.size(); ++k)
            if (!std::isfinite(dt_per_mesh[k])) throw Error{WLSENO_EINVAL, "time steps must be finite"};
        if (n_steps == 0) return WLSENO_OK;
        GroupRun run(ctx);
        for (auto &g : ctx->groups) {
            std::vector<double> dts;
            for (int32_t k : g.meshes) dts.push_back(dt_per_mesh[k]);
            check_child(g.c, wlseno_batch_step(g.c, u_dev, dts.data(), n_steps), g.dim);
        }
        run.join();
    } else {
        for (int k = 0; k < ctx->mesh.nmesh; ++k)
            if (!std::isfinite(dt_per_mesh[k])) throw Error{WLSENO_EINVAL, "time steps must be finite"};
        if (n_steps == 0) return WLSENO_OK;
        if (ctx->dm.nmesh == 1)
            run_steps(ctx, u_dev, dt_per_mesh[0], nullptr, n_steps);
        else
            run_steps(ctx, u_dev, 0.0, dt_per_mesh, n_steps);
    }
    numeric_check(ctx, u_dev, user_vars(ctx) * user_cells(ctx), user_cells(ctx), 1, "state");
    API_END(ctx)
}

namespace {

// Per-mesh maxima of the alpha slots of the last stage's parity.
std::vector<double> read_alpha(wlseno_ctx *ctx)
{
    const DevMesh &dm = ctx->dm;
    const size_t n = (size_t)dm.alpha_slots();
    std::vector<unsigned long long> slots(n * 16);
    check_hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    check_hip(hipMemcpy(slots.data(), dm.alpha + (size_t)ctx->last_parity * n * 16,
                        slots.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost),
              "hipMemcpy");
    std::vector<double> out(dm.nmesh, 0.0);
    for (int k = 0; k < dm.nmesh; ++k)
        for (int t = 0; t < dm.slots_per_mesh; ++t) {
            double v;
            std::memcpy(&v, &slots[((size_t)k * dm.slots_per_mesh + t) * 16], sizeof(double));
            out[k] = v > out[k] ? v : out[k];
        }
    return out;
}

}  // namespace

wlseno_status wlseno_last_alpha(wlseno_t ctx, double *alpha)
{
    API_BEGIN(ctx)
    if (!alpha) throw Error{WLSENO_EINVAL, "alpha is NULL"};
    need_device(ctx);
    if (mixed(ctx)) {
        double a = 0.0;
        for (auto &g : ctx->groups) {
            double ag = 0.0;
            check_child(g.c, wlseno_last_alpha(g.c, &ag), g.dim);
            a = ag > a ? ag : a;
        }
        *alpha = a;
        return WLSENO_OK;
    }
    double a = 0.0;
    for (double v : read_alpha(ctx)) a = v > a ? v : a;
    *alpha = a;
    API_END(ctx)
}

wlseno_status wlseno_batch_last_alpha(wlseno_t ctx, double *alpha_per_mesh)
{
    API_BEGIN(ctx)
    if (!alpha_per_mesh) throw Error{WLSENO_EINVAL, "alpha_per_mesh is NULL"};
    need_device(ctx);
    if (mixed(ctx)) {
        for (auto &g : ctx->groups) {
            std::vector<double> ag(g.meshes.size());
            check_child(g.c, wlseno_batch_last_alpha(g.c, ag.data()), g.dim);
            for (size_t t = 0; t < ag.size(); ++t) alpha_per_mesh[g.meshes[t]] = ag[t];
        }
        return WLSENO_OK;
    }
    const std::vector<double> a = read_alpha(ctx);
    for (size_t k = 0; k < a.size(); ++k) alpha_per_mesh[k] = a[k];
    API_END(ctx)
}

wlseno_status wlseno_time_kernel(wlseno_t ctx, int kernel, const double *u_dev, int launches, double *avg_ms)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_time_kernel");
    if (!u_dev || !avg_ms) throw Error{WLSENO_EINVAL, "null pointer"};
    if (kernel != 0 && kernel != 1) throw Error{WLSENO_EINVAL, "kernel must be 0 or 1"};
    if (launches < 1) throw Error{WLSENO_EINVAL, "launches must be >= 1"};
    need_device(ctx);
    need_single_dim(ctx, "wlseno_time_kernel");
    // state in device order, facet values and alpha of one reconstruction
    check_launch(launch_permute(ctx->dm, u_dev, ctx->ubuf, true, ctx->stream), "permute");
    *avg_ms = time_launches(ctx, kernel, launches);
    API_END(ctx)
}

}  // extern "C"

namespace {

// Average duration of `launches` back-to-back launches of one stage kernel
// (0 reconstruction, 1 flux/update) on the device-order state in ubuf,
// between two HIP events on the context's stream, after one untimed
// reconstruction (facet values and alpha).
double time_launches(wlseno_ctx *ctx, int kernel, int launches)
{
    check_launch(launch_clear_alpha(ctx->dm, ctx->stream), "clear");
    check_launch(launch_reconstruct(ctx->dm, ctx->ubuf, 0, nullptr, nullptr, nullptr, ctx->stream), "reconstruct");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    check_hip(hipEventCreate(&e0), "hipEventCreate");
    hipError_t he = hipEventCreate(&e1);
    float ms = 0.0f;
    if (he == hipSuccess) he = hipEventRecord(e0, ctx->stream);
    int le = 0;
    for (int i = 0; he == hipSuccess && le == 0 && i < launches; ++i) {
        // both are idempotent here: the reconstruction rewrites the same facet
        // values and alpha maximum, the update writes L(u) to a buffer of its own
        if (kernel == 0)
            le = launch_reconstruct(ctx->dm, ctx->ubuf, 0, nullptr, nullptr, nullptr, ctx->stream);
        else
            le = launch_update(ctx->dm, nullptr, nullptr, ctx->tbuf, 0.0, 0.0, 1.0, 0, 0, ctx->stream);
    }
    if (he == hipSuccess && le == 0) he = hipEventRecord(e1, ctx->stream);
    if (he == hipSuccess && le == 0) he = hipEventSynchronize(e1);
    if (he == hipSuccess && le == 0) he = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    check_launch(le, kernel == 0 ? "reconstruct" : "update");
    check_hip(he, "kernel timing events");
    ctx->last_parity = 0;
    return (double)ms / launches;
}

// A smooth, physical state in device order for timing (the solve's cost does
// not depend on the values beyond rare pivot exchanges): scalars
// 0.5 + 0.25 sin(2 pi x) cos(2 pi y) + 0.1 z; Euler rho = 1 + 0.2 sin(2 pi x),
// velocity (0.3, -0.2), p = 1 + 0.1 cos(2 pi y).
void synthetic_state(wlseno_ctx *ctx)
{
    const Build &b = ctx->build;
    const int64_t nc = ctx->dm.nc;
    const int dim = ctx->dm.dim;
    const double tp = 6.283185307179586;
    std::vector<double> u((size_t)b.nvars * nc);
    for (int64_t i = 0; i < nc; ++i) {
        const double *c = &b.geo[(size_t)i * b.gs];
        const double x = c[0], y = dim > 1 ? c[1] : 0.0, z = dim > 2 ? c[2] : 0.0;
        if (b.nvars == 1) {
            u[i] = 0.5 + 0.25 * std::sin(tp * x) * std::cos(tp * y) + 0.1 * z;
        } else {
            const double rho = 1.0 + 0.2 * std::sin(tp * x), vx = 0.3, vy = -0.2, pr = 1.0 + 0.1 * std::cos(tp * y);
            u[i] = rho;
            u[nc + i] = rho * vx;
            u[2 * nc + i] = rho * vy;
            u[3 * nc + i] = pr / (b.prm.gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy);
        }
    }
    check_hip(hipMemcpyAsync(ctx->ubuf, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream),
              "hipMemcpyAsync");
    check_hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
}

#ifndef WLSENO_BUILD_ID
#define WLSENO_BUILD_ID "unversioned"
#endif

// Autotuning results of this process, per device, kernel build and workload
// class: dim, order, flux variant, components, stencil sizes and the share of
// cells per stencil-size bucket (tenths), cell count (power of two).
struct TuneEntry {
    wlseno_tune result;
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune_cache;

std::string tune_key(wlseno_ctx *ctx)
{
    hipDeviceProp_t prop;
    check_hip(hipGetDeviceProperties(&prop, ctx->device), "hipGetDeviceProperties");
    const DevMesh &dm = ctx->dm;
    std::string k = std::string(prop.gcnArchName) + "/" + std::to_string(prop.pciBusID) + "/" + WLSENO_BUILD_ID;
    k += "/d" + std::to_string(dm.dim) + "p" + std::to_string(dm.p) + "f" + std::to_string(dm.flux) + "c" +
         std::to_string(dm.characteristic) + "v" + std::to_string(dm.nvars) + "b" + std::to_string(dm.balance) +
         "s" + std::to_string(ctx->build.min_stencil) + "-" + std::to_string(dm.max_stencil);
    for (int t = 0; t < dm.nbuckets; ++t) {
        const double share = dm.nc ? (double)(dm.bucket_cell0[t + 1] - dm.bucket_cell0[t]) / dm.nc : 0.0;
        k += "/" + std::to_string((int)std::lround(10.0 * share));
    }
    int lg = 0;
    while ((int64_t(1) << lg) < dm.nc) ++lg;
    return k + "/n" + std::to_string(lg);
}

}  // namespace

extern "C" {

wlseno_status wlseno_autotune(wlseno_t ctx, const double *u_dev, wlseno_tune *out)
{
    API_BEGIN(ctx)
    ApiRange range_("wlseno_autotune");
    if (!out) throw Error{WLSENO_EINVAL, "out is NULL"};
    need_device(ctx);
    std::memset(out, 0, sizeof(*out));
    if (mixed(ctx)) {
        // every group on its own; out describes the first
        for (size_t gi = 0; gi < ctx->groups.size(); ++gi) {
            wlseno_tune t;
            auto &g = ctx->groups[gi];
            check_child(g.c, wlseno_autotune(g.c, u_dev, &t), g.dim);
            if (gi == 0) *out = t;
        }
        return WLSENO_OK;
    }
    const std::string key = tune_key(ctx);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *out = it->second.result;
            out->cached = 1;
            if (ctx->dm.lanes != out->chosen) drop_graph(ctx);
            ctx->dm.lanes = out->chosen;
            ctx->build.prm.lanes = out->chosen;
            return WLSENO_OK;
        }
    }
    if (u_dev)
        check_launch(launch_permute(ctx->dm, u_dev, ctx->ubuf, true, ctx->stream), "permute");
    else
        synthetic_state(ctx);
    const std::vector<int> cand = lane_choices(ctx->dm);
    const int keep = ctx->dm.lanes;
    int best = -1;
    double best_us = 0.0;
    try {
        for (int lanes : cand) {
            if (out->n >= 4) break;
            ctx->dm.lanes = lanes;
            // about 20 ms of launches, at least 3 and at most 200
            const double one = time_launches(ctx, 0, 1);
            int n = (int)(20.0 / (one > 1e-3 ? one : 1e-3));
            n = n < 3 ? 3 : (n > 200 ? 200 : n);
            const double us = 1e3 * time_launches(ctx, 0, n);
            out->lanes[out->n] = lanes;
            out->us[out->n] = us;
            out->n += 1;
            if (best < 0 || us < best_us) {
                best = lanes;
                best_us = us;
            }
        }
    } catch (...) {
        ctx->dm.lanes = keep;
        throw;
    }
    // the automatic choice stays unless another is faster by 2% or more:
    // differences below that are run-to-run noise
    const int dflt = default_lanes(ctx->dm);
    for (int t = 0; t < out->n; ++t)
        if (out->lanes[t] == dflt && !(best_us < 0.98 * out->us[t])) best = dflt;
    out->chosen = best;
    out->cached = 0;
    if (keep != best) drop_graph(ctx);
    ctx->dm.lanes = best;
    ctx->build.prm.lanes = best;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = TuneEntry{*out};
    API_END(ctx)
}

}  // extern "C"
