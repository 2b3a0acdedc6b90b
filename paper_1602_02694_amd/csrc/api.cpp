// C-ABI entry points of the WLS-ENO library (declared in include/wlseno.h).
// Host orchestration only: every numerical step of the path runs in the HIP
// kernels of kernels.hip; this file validates arguments, owns device memory
// and enqueues the kernels on the context's stream.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace wlseno;

struct wlseno_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    std::string err;
    bool have_mesh = false, have_build = false;
    HostMesh mesh;
    Build build;
    DevMesh dm;
    std::vector<void *> allocs;
    double *ubuf = nullptr, *kbuf = nullptr, *tbuf = nullptr;
    int last_parity = 0;
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

void free_device(wlseno_ctx *c)
{
    if (c->device >= 0) {
        (void)hipSetDevice(c->device);
        for (void *p : c->allocs) (void)hipFree(p);
    }
    c->allocs.clear();
    c->dm = DevMesh{};
    c->ubuf = c->kbuf = c->tbuf = nullptr;
}

void *dev_alloc(wlseno_ctx *c, size_t bytes)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 8);
    if (e != hipSuccess) throw Error{WLSENO_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    c->allocs.push_back(p);
    return p;
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
    dm.alpha_w = b.prm.alpha_w;
    dm.rank_tol = b.prm.rank_tol;
    dm.period = m.periodic ? m.period : 0.0;
    dm.gamma = b.prm.gamma;
    for (int d = 0; d < 3; ++d) dm.vel[d] = b.prm.velocity[d];
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
    dm.alpha = (unsigned long long *)dev_alloc(c, 2 * kAlphaSlots * 16 * sizeof(unsigned long long));
    check_hip(hipMemset(dm.alpha, 0, 2 * kAlphaSlots * 16 * sizeof(unsigned long long)), "hipMemset");
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
void stage(wlseno_ctx *c, const double *in, const double *u0, const double *prev, double *out, double A,
           double B, double Cdt, int mode, int parity)
{
    check_launch(launch_reconstruct(c->dm, in, parity, nullptr, nullptr, nullptr, c->stream), "reconstruct");
    check_launch(launch_update(c->dm, u0, prev, out, A, B, Cdt, mode, parity, c->stream), "update");
    c->last_parity = parity;
}

}  // namespace

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
}

wlseno_status wlseno_create(int device, wlseno_t *out)
{
    if (!out) return WLSENO_EINVAL;
    *out = nullptr;
    g_create_error.clear();
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
    wlseno_ctx *c = new (std::nothrow) wlseno_ctx;
    if (!c) return WLSENO_ENOMEM;
    c->device = device;
    *out = c;
    return WLSENO_OK;
}

wlseno_status wlseno_destroy(wlseno_t ctx)
{
    if (!ctx) return WLSENO_OK;
    free_device(ctx);
    delete ctx;
    return WLSENO_OK;
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
    free_device(ctx);
    ctx->mesh = std::move(m);
    ctx->have_mesh = true;
    ctx->have_build = false;
    ctx->build = Build{};
    API_END(ctx)
}

wlseno_status wlseno_stencil_build(wlseno_t ctx, const wlseno_params *params)
{
    API_BEGIN(ctx)
    if (!params) throw Error{WLSENO_EINVAL, "params is NULL"};
    if (!ctx->have_mesh) throw Error{WLSENO_ESTATE, "call wlseno_mesh_upload first"};
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
    const Build &b = ctx->build;
    out->dim = ctx->mesh.dim;
    out->m = b.m;
    out->n_vars = b.nvars;
    out->faces_per_cell = b.nf;
    out->points_per_face = b.nq;
    out->min_stencil = b.min_stencil;
    out->max_stencil = b.max_stencil;
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
    std::memcpy(row_ptr, ctx->build.row_ptr.data(), ctx->build.row_ptr.size() * sizeof(int32_t));
    std::memcpy(col, ctx->build.col.data(), ctx->build.col.size() * sizeof(int32_t));
    API_END(ctx)
}

wlseno_status wlseno_reconstruct(wlseno_t ctx, const double *u_dev, double *coef_dev, double *facevals_dev,
                                 int32_t *rank_dev)
{
    API_BEGIN(ctx)
    if (!u_dev) throw Error{WLSENO_EINVAL, "u_dev is NULL"};
    need_device(ctx);
    check_launch(launch_permute(ctx->dm, u_dev, ctx->ubuf, true, ctx->stream), "permute");
    check_launch(launch_clear_alpha(ctx->dm, ctx->stream), "clear");
    check_launch(launch_reconstruct(ctx->dm, ctx->ubuf, 0, coef_dev, facevals_dev, rank_dev, ctx->stream),
                 "reconstruct");
    ctx->last_parity = 0;
    API_END(ctx)
}

wlseno_status wlseno_rhs(wlseno_t ctx, const double *u_dev, double *dudt_dev)
{
    API_BEGIN(ctx)
    if (!u_dev || !dudt_dev) throw Error{WLSENO_EINVAL, "null device pointer"};
    if (u_dev == dudt_dev) throw Error{WLSENO_EINVAL, "dudt_dev must not alias u_dev"};
    need_device(ctx);
    check_launch(launch_permute(ctx->dm, u_dev, ctx->ubuf, true, ctx->stream), "permute");
    check_launch(launch_clear_alpha(ctx->dm, ctx->stream), "clear");
    stage(ctx, ctx->ubuf, nullptr, nullptr, ctx->tbuf, 0.0, 0.0, 1.0, 0, 0);
    check_launch(launch_permute(ctx->dm, ctx->tbuf, dudt_dev, false, ctx->stream), "permute");
    API_END(ctx)
}

wlseno_status wlseno_step(wlseno_t ctx, double *u_dev, double dt, int n_steps)
{
    API_BEGIN(ctx)
    if (!u_dev) throw Error{WLSENO_EINVAL, "u_dev is NULL"};
    if (!std::isfinite(dt) || n_steps < 0) throw Error{WLSENO_EINVAL, "dt must be finite and n_steps >= 0"};
    need_device(ctx);
    if (n_steps == 0) return WLSENO_OK;
    double *u = ctx->ubuf, *k = ctx->kbuf;
    check_launch(launch_permute(ctx->dm, u_dev, u, true, ctx->stream), "permute");
    check_launch(launch_clear_alpha(ctx->dm, ctx->stream), "clear");
    int par = 0;
    for (int s = 0; s < n_steps; ++s) {
        // k1 = u + dt L(u); k2 = 3/4 u + 1/4 k1 + 1/4 dt L(k1); u = 1/3 u + 2/3 k2 + 2/3 dt L(k2)
        stage(ctx, u, u, u, k, 1.0, 0.0, dt, 1, par);
        par ^= 1;
        stage(ctx, k, u, k, k, 0.75, 0.25, 0.25 * dt, 1, par);
        par ^= 1;
        stage(ctx, k, u, k, u, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0 * dt, 1, par);
        par ^= 1;
    }
    check_launch(launch_permute(ctx->dm, u, u_dev, false, ctx->stream), "permute");
    API_END(ctx)
}

wlseno_status wlseno_last_alpha(wlseno_t ctx, double *alpha)
{
    API_BEGIN(ctx)
    if (!alpha) throw Error{WLSENO_EINVAL, "alpha is NULL"};
    need_device(ctx);
    std::vector<unsigned long long> slots(kAlphaSlots * 16);
    check_hip(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    check_hip(hipMemcpy(slots.data(), ctx->dm.alpha + (size_t)ctx->last_parity * kAlphaSlots * 16,
                        slots.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost),
              "hipMemcpy");
    double a = 0.0;
    for (int s = 0; s < kAlphaSlots; ++s) {
        double v;
        std::memcpy(&v, &slots[s * 16], sizeof(double));
        a = v > a ? v : a;
    }
    *alpha = a;
    API_END(ctx)
}

wlseno_status wlseno_time_kernel(wlseno_t ctx, int kernel, const double *u_dev, int launches, double *avg_ms)
{
    API_BEGIN(ctx)
    if (!u_dev || !avg_ms) throw Error{WLSENO_EINVAL, "null pointer"};
    if (kernel != 0 && kernel != 1) throw Error{WLSENO_EINVAL, "kernel must be 0 or 1"};
    if (launches < 1) throw Error{WLSENO_EINVAL, "launches must be >= 1"};
    need_device(ctx);
    // state in device order, facet values and alpha of one reconstruction
    check_launch(launch_permute(ctx->dm, u_dev, ctx->ubuf, true, ctx->stream), "permute");
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
    *avg_ms = (double)ms / launches;
    API_END(ctx)
}

}  // extern "C"
