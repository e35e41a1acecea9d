// sme_lib.cpp -- host side of the SME library: the C ABI declared in include/sme.h.
//
// Binds the caller's two state buffers (ping-pong) to a context, owns the
// per-context tables (bathymetry in the internal cell order, triangle
// neighbours, normals and a reverse Cuthill-McKee cell order, the
// Gauss-Legendre points of the path integral) and the time-step slots, and
// queues the step kernels, capturing runs of steps in HIP graphs so a long
// run costs one graph launch per six steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/sme.h"
#include "sme_host.h"
#include "sme_mesh.h"
#include "sme_kernels.h"
#include "sme_lift.h"

using namespace sme;
using namespace sme::mesh;

namespace {

constexpr int kGraphSteps = 6;  // lcm of the ping-pong period (2) and the slot period (3)
constexpr int kLdsRunSteps = 2048;  // steps per launch of the multi-step kernel of small 1D grids
// The multi-step kernel runs on one compute unit, so past some number of
// 62-cell windows the per-step kernel, spread over the device, is faster; the
// arithmetic per window grows with the level.  Largest window counts per
// level, from measurements (us per step, multi-step against graphs): level 1,
// 2000 cells 4.3 / 5.1, 2900 cells 5.5 / 5.1; level 2, 1800 cells 4.8 / 5.3;
// level 4, 1200 cells 4.7 / 5.4; level 8, 390 cells 5.2 / 6.9, 900 cells
// 8.5 / 7.4; levels in between interpolated.
constexpr int kLdsRunMaxWindows[9] = {40, 40, 32, 26, 20, 16, 12, 10, 8};

struct GraphEntry {
    int cur, slot;
    double t_end;
    hipGraphExec_t exec;
};

}  // namespace

struct sme_ctx {
    int level = 0;
    int kind = 0;
    int nf = 0;
    int64_t ncells = 0;
    int64_t stride = 0;
    int64_t nx = 0, ny = 0;
    size_t lds_optin = 0;  // LDS a workgroup may request (multi-step kernel of small 1D grids)
    double dx = 0, dy = 0;
    int bc[4] = {0, 0, 0, 0};
    int rows = 16;
    sme_params p{};
    Quad quad{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    // device memory: the state buffers belong to the caller, the rest to the context
    double *q[2] = {nullptr, nullptr};
    double *b = nullptr;
    int32_t *nbr = nullptr;
    double *fsx = nullptr, *fsy = nullptr, *ivol = nullptr;
    double *cx = nullptr, *cy = nullptr;  // triangle centroids (3D lifting)
    int64_t *to_internal = nullptr;  // caller cell -> internal cell (triangles)
    int64_t *to_caller = nullptr;    // internal cell -> caller cell
    Slot *slots = nullptr;
    ErrWord *err = nullptr;
    double *quad_dev = nullptr;      // Gauss points [kMaxQuad] then weights [kMaxQuad]
    ClosureModel *closure = nullptr;  // learned closure attached to a level-1 context
    unsigned long long *oor = nullptr;  // cells that left the closure's training range
    float *rates = nullptr;             // closure rates of the current state (2 or 4 per cell)
    int closure_mode = 0;               // ClosurePrecision of the attached network
    double *ckpt = nullptr;             // state at the start of a closure chunk (sme_closure_run)
    bool order2 = false;                // the second-order scheme
    double *slopes = nullptr;           // its limited slopes (1D grids, and structured grids above
                                        // the levels of the fused band stages)
    double *t_host = nullptr;           // pinned: simulated time after the latest graph with an end time
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // completion of the last graphs of a run
    int cus = 256;                      // compute units of the device
    int cur = 0;   // which q[] holds the state
    int sa = 0;    // slot describing the current state
    bool has_state = false;
    std::vector<GraphEntry> graphs;
    std::string last;
};

namespace {

int fail(sme_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->last = buf;
    }
    return code;
}

#define HIPCHK(ctx, call)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail((ctx), SME_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));          \
    } while (0)


// field stride of a state: ncells rounded up to 256 elements (every field starts 2 KiB aligned)
int64_t stride_of(int64_t ncells) { return (ncells + 255) / 256 * 256; }

// A caller's state buffer must be device memory of the current device, at
// least `bytes` long from p, and 256-byte aligned.
int check_device_buffer(sme_ctx *c, const void *p, size_t bytes)
{
    if (((uintptr_t)p & 255u) != 0) return fail(c, SME_EINVAL, "state buffer %p is not 256-byte aligned", p);
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess || at.type != hipMemoryTypeDevice || at.device != c->device) {
        (void)hipGetLastError();
        return fail(c, SME_EINVAL, "state buffer %p is not device memory of device %d", p, c->device);
    }
    void *base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange((hipDeviceptr_t *)&base, &size, (hipDeviceptr_t)p) == hipSuccess && base) {
        if ((const char *)p + bytes > (const char *)base + size)
            return fail(c, SME_EINVAL, "state buffer %p holds fewer than %zu bytes", p, bytes);
    } else {
        (void)hipGetLastError();
    }
    return SME_OK;
}



template <typename T>
int dalloc(sme_ctx *c, T **p, size_t count)
{
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, e == hipErrorOutOfMemory ? SME_ENOMEM : SME_EHIP, "hipMalloc(%zu bytes): %s",
                    count * sizeof(T), hipGetErrorString(e));
    }
    return SME_OK;
}

StepArgs make_args(const sme_ctx *c)
{
    StepArgs a{};
    a.q = c->q[c->cur];
    a.qn = c->q[1 - c->cur];
    a.b = c->b;
    a.stride = c->stride;
    a.ncells = c->ncells;
    a.nx = (int)c->nx;
    a.ny = (int)c->ny;
    a.idx = c->dx > 0 ? 1.0 / c->dx : 0.0;
    a.idy = c->dy > 0 ? 1.0 / c->dy : 0.0;
    for (int s = 0; s < 4; ++s) a.bc[s] = c->bc[s];
    a.rows = c->rows;
    a.nbr = c->nbr;
    a.fsx = c->fsx;
    a.fsy = c->fsy;
    a.ivol = c->ivol;
    a.g = c->p.g;
    a.c_slip = c->p.c_slip;
    a.implicit = c->p.implicit_friction;
    a.nu = c->p.nu;
    a.cfl = c->p.cfl;
    a.quad = c->quad;
    a.slots = c->slots;
    a.sa = c->sa;
    a.sb = (c->sa + 1) % 3;
    a.sc = (c->sa + 2) % 3;
    a.err = c->err;
    a.closure = c->closure;
    a.oor = c->oor;
    a.rates = c->rates;
    return a;
}

// the second-order scheme keeps a slopes array on 1D grids and on structured
// grids above the levels of the fused band stages
bool needs_slopes(int kind, int level) { return kind != SME_MESH_2D_STRUCT || level > kStage2BandMaxLevel; }

hipError_t launch_one_step(sme_ctx *c, double dt_fixed, double t_end)
{
    StepArgs a = make_args(c);
    a.dt_fixed = dt_fixed;
    a.t_end = t_end;
    hipError_t e = hipSuccess;
    if (c->order2) {
        // second order: stage 1 into the other buffer, stage 2 back in place
        const int dim = c->kind == SME_MESH_1D ? 1 : 2;
        StepArgs a2 = a;
        a2.q = a.qn;
        a2.qn = const_cast<double *>(a.q);
        if (!c->slopes) {
            // structured grid: the reconstruction fused into the band stages
            e = launch_stage2_band(c->level, 1, a, c->stream);
            if (e == hipSuccess) e = launch_stage2_band(c->level, 2, a2, c->stream);
        } else {
            e = launch_recon2(c->level, dim, a, c->slopes, c->stream);
            if (e == hipSuccess) e = launch_flux2(c->level, dim, 1, a, c->slopes, c->stream);
            if (e == hipSuccess) e = launch_recon2(c->level, dim, a2, c->slopes, c->stream);
            if (e == hipSuccess) e = launch_flux2(c->level, dim, 2, a2, c->slopes, c->stream);
        }
        if (e == hipSuccess) c->sa = (c->sa + 1) % 3;
        return e;
    }
    if (c->closure) e = launch_closure_rates(a, c->kind == SME_MESH_1D ? 1 : 2, c->closure_mode, c->cus, c->stream);
    if (e != hipSuccess) return e;
    switch (c->kind) {
    case SME_MESH_1D: e = launch_step_1d(c->level, a, c->stream); break;
    case SME_MESH_2D_STRUCT: e = launch_step_2d(c->level, a, c->stream); break;
    default: e = launch_step_tri(c->level, a, c->stream); break;
    }
    if (e == hipSuccess) {
        c->cur = 1 - c->cur;
        c->sa = (c->sa + 1) % 3;
    }
    return e;
}

void drop_graphs(sme_ctx *c)
{
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

int get_graph(sme_ctx *c, double t_end, hipGraphExec_t *out)
{
    for (auto &g : c->graphs)
        if (g.cur == c->cur && g.slot == c->sa && g.t_end == t_end) {
            *out = g.exec;
            return SME_OK;
        }
    const int cur0 = c->cur, sa0 = c->sa;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (int k = 0; k < kGraphSteps && le == hipSuccess; ++k) le = launch_one_step(c, 0.0, t_end);
    // with an end time the graph also reports the simulated time to the host
    if (le == hipSuccess && t_end > 0.0)
        le = hipMemcpyAsync(c->t_host, &c->slots[sa0].t, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(c->stream, &graph);
    c->cur = cur0;
    c->sa = sa0;
    if (le != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(c, SME_EHIP, "graph capture failed: %s", hipGetErrorString(le != hipSuccess ? le : ee));
    }
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(c, SME_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
    c->graphs.push_back(GraphEntry{cur0, sa0, t_end, exec});
    *out = exec;
    return SME_OK;
}

int nonphys(sme_ctx *c, const ErrWord &e)
{
    if (e.first_step == 0) return fail(c, SME_ENONPHYS, "the loaded state is non-physical (h <= 0 or non-finite)");
    return fail(c, SME_ENONPHYS, "non-physical state (h <= 0 or non-finite) produced by step %llu",
                (unsigned long long)e.first_step);
}

int read_slot(sme_ctx *c, Slot *s, ErrWord *e)
{
    HIPCHK(c, hipMemcpyAsync(s, c->slots + c->sa, sizeof(Slot), hipMemcpyDeviceToHost, c->stream));
    if (e) HIPCHK(c, hipMemcpyAsync(e, c->err, sizeof(ErrWord), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SME_OK;
}

template <int N>
void copy_tensors(double *M, double *A, double *B, double *K)
{
    constexpr int n = N + 1;
    const auto &T = Basis<N>::T;
    for (int i = 0; i < n; ++i) {
        if (M) M[i] = T.M[i];
        for (int j = 0; j < n; ++j) {
            if (K) K[i * n + j] = T.K[i][j];
            for (int k = 0; k < n; ++k) {
                if (A) A[(i * n + j) * n + k] = T.A[i][j][k];
                if (B) B[(i * n + j) * n + k] = T.B[i][j][k];
            }
        }
    }
}
}  // namespace

extern "C" {

int sme_layout(int level, const sme_mesh *mesh, int *nfields, int64_t *ncells, int64_t *field_stride)
{
    int nf = 0;
    int64_t nc = 0;
    int r = check_mesh(mesh, level, &nf, &nc);
    if (r != SME_OK) return r;
    if (nfields) *nfields = nf;
    if (ncells) *ncells = nc;
    if (field_stride) *field_stride = stride_of(nc);
    return SME_OK;
}

int sme_workspace_size(int level, const sme_mesh *mesh, const sme_params *params, size_t *bytes)
{
    int nf = 0;
    int64_t nc = 0;
    int r = check_mesh(mesh, level, &nf, &nc);
    if (r != SME_OK) return r;
    if (!bytes) return SME_EINVAL;
    const size_t st = (size_t)stride_of(nc);
    size_t n = st * sizeof(double)                 // bathymetry (internal order)
               + 3 * sizeof(Slot) + sizeof(ErrWord) + 2 * kMaxQuad * sizeof(double);
    if (params && params->order == 2 && needs_slopes(mesh->kind, level))  // limited slopes of the second-order scheme
        n += (size_t)(mesh->kind == SME_MESH_1D ? 1 : 2) * (nf + 1) * st * sizeof(double);
    if (mesh->kind == SME_MESH_2D_TRI)
        n += 3 * st * (sizeof(int32_t) + 3 * sizeof(double))  // neighbours, normals, |e|/|V|
             + 2 * st * sizeof(double)                        // centroids
             + 2 * (size_t)nc * sizeof(int64_t);             // the two permutations
    *bytes = n;
    return SME_OK;
}

int sme_init(sme_ctx **out, int level, const sme_mesh *mesh, const sme_params *params, double *const q_dev[2],
             const double *b, int b_on_device, void *stream)
{
    if (!out || !params || !q_dev || !q_dev[0] || !q_dev[1] || q_dev[0] == q_dev[1]) return SME_EINVAL;
    *out = nullptr;
    int nf;
    int64_t nc;
    int r = check_mesh(mesh, level, &nf, &nc);
    if (r != SME_OK) return r;
    if (params->quad_points < 1 || params->quad_points > kMaxQuad || !(params->cfl > 0) || !(params->g > 0) ||
        params->c_slip < 0 || params->nu < 0 || (params->implicit_friction != 0 && params->implicit_friction != 1) ||
        (params->order != 1 && params->order != 2))
        return SME_EINVAL;
    if (params->order == 2 && mesh->kind == SME_MESH_2D_TRI) return SME_EINVAL;
    sme_ctx *c = new (std::nothrow) sme_ctx();
    if (!c) return SME_ENOMEM;
    c->level = level;
    c->kind = mesh->kind;
    c->nf = nf;
    c->ncells = nc;
    c->stride = stride_of(nc);
    c->p = *params;
    double qs[kMaxQuad] = {0}, qw[kMaxQuad] = {0};
    host::gauss_legendre01(params->quad_points, qs, qw);
    c->quad.n = params->quad_points;
    c->quad.s0 = qs[0];
    c->quad.s1 = qs[1];
    c->quad.s2 = qs[2];
    c->quad.w0 = qw[0];
    c->quad.w1 = qw[1];
    c->quad.w2 = qw[2];
    for (int s = 0; s < 4; ++s) c->bc[s] = mesh->bc[s];
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return SME_EHIP;
    }
    {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, c->device) != hipSuccess || v <= 0)
            v = 64 * 1024;
        c->lds_optin = (size_t)v;
    }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) {
            delete c;
            return SME_EHIP;
        }
        c->own_stream = true;
    }
    if (mesh->kind == SME_MESH_1D) {
        c->nx = mesh->nx;
        c->ny = 1;
        c->dx = (mesh->x1 - mesh->x0) / mesh->nx;
    } else if (mesh->kind == SME_MESH_2D_STRUCT) {
        c->nx = mesh->nx;
        c->ny = mesh->ny;
        c->dx = (mesh->x1 - mesh->x0) / mesh->nx;
        c->dy = (mesh->y1 - mesh->y0) / mesh->ny;
        const char *env = getenv("SME_ROWS");
        c->rows = env ? std::max(1, atoi(env)) : host::pick_rows(c->level, c->nx, c->ny, host::device_cus());
    }
    int rc = SME_OK;
    for (int k = 0; k < 2 && !rc; ++k) {
        c->q[k] = q_dev[k];
        rc = check_device_buffer(c, q_dev[k], (size_t)nf * c->stride * sizeof(double));
    }
    rc = rc ? rc : dalloc(c, &c->b, (size_t)c->stride);
    c->order2 = params->order == 2;
    if (c->order2 && needs_slopes(mesh->kind, level))
        rc = rc ? rc : dalloc(c, &c->slopes, (size_t)(mesh->kind == SME_MESH_1D ? 1 : 2) * (nf + 1) * c->stride);
    rc = rc ? rc : dalloc(c, &c->slots, 3);
    rc = rc ? rc : dalloc(c, &c->err, 1);
    rc = rc ? rc : dalloc(c, &c->quad_dev, 2 * kMaxQuad);
    if (!rc) {
        double buf[2 * kMaxQuad];
        memcpy(buf, qs, sizeof qs);
        memcpy(buf + kMaxQuad, qw, sizeof qw);
        if (hipMemcpy(c->quad_dev, buf, sizeof buf, hipMemcpyHostToDevice) != hipSuccess)
            rc = fail(c, SME_EHIP, "quadrature upload failed");
        c->quad.s = c->quad_dev;
        c->quad.w = c->quad_dev + kMaxQuad;
    }
    std::vector<int64_t> order;  // internal position -> caller cell
    if (!rc && mesh->kind == SME_MESH_2D_TRI) {
        TriGeom g;
        std::string why;
        rc = build_tri(mesh, g, why);
        if (rc) rc = fail(c, rc, "%s", why.c_str());
        if (!rc) {
            order = rcm_order(g.nbr, nc);
            std::vector<int64_t> inv(nc);
            for (int64_t k = 0; k < nc; ++k) inv[order[k]] = k;
            std::vector<int32_t> nb(3 * c->stride, -1);
            std::vector<double> fx(3 * c->stride, 0.0), fy(3 * c->stride, 0.0), iv(c->stride, 0.0);
            std::vector<double> ccx(c->stride, 0.0), ccy(c->stride, 0.0);
            for (int64_t k = 0; k < nc; ++k) {
                int64_t t = order[k];
                for (int s = 0; s < 3; ++s) {
                    ccx[k] += mesh->vert_xy[2 * mesh->tri[3 * t + s]] / 3.0;
                    ccy[k] += mesh->vert_xy[2 * mesh->tri[3 * t + s] + 1] / 3.0;
                }
                iv[k] = g.ivol[t];
                for (int s = 0; s < 3; ++s) {
                    int32_t v = g.nbr[3 * t + s];
                    nb[s * c->stride + k] = v >= 0 ? (int32_t)inv[v] : -1;
                    fx[s * c->stride + k] = g.sx[3 * t + s];
                    fy[s * c->stride + k] = g.sy[3 * t + s];
                }
            }
            rc = rc ? rc : dalloc(c, &c->nbr, 3 * c->stride);
            rc = rc ? rc : dalloc(c, &c->fsx, 3 * c->stride);
            rc = rc ? rc : dalloc(c, &c->fsy, 3 * c->stride);
            rc = rc ? rc : dalloc(c, &c->ivol, c->stride);
            rc = rc ? rc : dalloc(c, &c->to_internal, nc);
            rc = rc ? rc : dalloc(c, &c->to_caller, nc);
            rc = rc ? rc : dalloc(c, &c->cx, c->stride);
            rc = rc ? rc : dalloc(c, &c->cy, c->stride);
            if (!rc) {
                hipError_t e = hipSuccess;
                if (e == hipSuccess) e = hipMemcpy(c->nbr, nb.data(), nb.size() * sizeof(int32_t), hipMemcpyHostToDevice);
                if (e == hipSuccess) e = hipMemcpy(c->fsx, fx.data(), fx.size() * sizeof(double), hipMemcpyHostToDevice);
                if (e == hipSuccess) e = hipMemcpy(c->fsy, fy.data(), fy.size() * sizeof(double), hipMemcpyHostToDevice);
                if (e == hipSuccess) e = hipMemcpy(c->ivol, iv.data(), iv.size() * sizeof(double), hipMemcpyHostToDevice);
                if (e == hipSuccess) e = hipMemcpy(c->to_internal, inv.data(), nc * sizeof(int64_t), hipMemcpyHostToDevice);
                if (e == hipSuccess) e = hipMemcpy(c->to_caller, order.data(), nc * sizeof(int64_t), hipMemcpyHostToDevice);
                if (e == hipSuccess) e = hipMemcpy(c->cx, ccx.data(), ccx.size() * sizeof(double), hipMemcpyHostToDevice);
                if (e == hipSuccess) e = hipMemcpy(c->cy, ccy.data(), ccy.size() * sizeof(double), hipMemcpyHostToDevice);
                if (e != hipSuccess) rc = fail(c, SME_EHIP, "geometry upload: %s", hipGetErrorString(e));
            }
        }
    }
    // bathymetry (caller order -> internal order)
    if (!rc) {
        hipError_t e = hipMemsetAsync(c->b, 0, c->stride * sizeof(double), c->stream);
        if (e == hipSuccess && b) {
            if (c->to_internal) {
                double *tmp = c->q[1];
                e = hipMemcpyAsync(tmp, b, nc * sizeof(double), b_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                   c->stream);
                if (e == hipSuccess) e = launch_permute(tmp, nc, c->b, c->stride, c->to_internal, nc, 1, c->stream);
            } else {
                e = hipMemcpyAsync(c->b, b, nc * sizeof(double), b_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                   c->stream);
            }
        }
        if (e == hipSuccess) e = launch_slots_reset(c->slots, c->err, 0, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = fail(c, SME_EHIP, "init upload: %s", hipGetErrorString(e));
    }
    if (rc) {
        sme_destroy(c);
        return rc;
    }
    *out = c;
    return SME_OK;
}

int sme_set_state(sme_ctx *c, const double *q, int on_device)
{
    if (!c || !q) return SME_EINVAL;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const size_t row = c->ncells * sizeof(double);
    if (c->to_internal) {
        double *tmp = c->q[1 - c->cur];
        HIPCHK(c, hipMemcpy2DAsync(tmp, c->stride * sizeof(double), q, row, row, c->nf, kind, c->stream));
        HIPCHK(c, launch_permute(tmp, c->stride, c->q[c->cur], c->stride, c->to_internal, c->ncells, c->nf, c->stream));
    } else if (q == c->q[c->cur] || q == c->q[1 - c->cur]) {
        // the caller wrote the state into one of its bound buffers in place
        // (field stride of the context): adopt that buffer
        if (!on_device) return fail(c, SME_EINVAL, "a bound state buffer is device memory");
        c->cur = q == c->q[c->cur] ? c->cur : 1 - c->cur;
        drop_graphs(c);
    } else {
        HIPCHK(c, hipMemcpy2DAsync(c->q[c->cur], c->stride * sizeof(double), q, row, row, c->nf, kind, c->stream));
    }
    // fresh clock and CFL ratio of the loaded state
    c->sa = 0;
    if (c->oor) HIPCHK(c, hipMemsetAsync(c->oor, 0, sizeof(unsigned long long), c->stream));
    HIPCHK(c, launch_slots_reset(c->slots, c->err, 0, c->stream));
    StepArgs a = make_args(c);
    HIPCHK(c, launch_eig(c->kind == SME_MESH_1D ? 1 : 2, c->kind, c->level, a, c->stream));
    c->has_state = true;
    if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
    return SME_OK;
}

int sme_get_state(sme_ctx *c, double *q, int on_device)
{
    if (!c || !q) return SME_EINVAL;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t row = c->ncells * sizeof(double);
    const double *src = c->q[c->cur];
    if (c->to_caller) {
        double *tmp = c->q[1 - c->cur];
        HIPCHK(c, launch_permute(src, c->stride, tmp, c->stride, c->to_caller, c->ncells, c->nf, c->stream));
        src = tmp;
    }
    HIPCHK(c, hipMemcpy2DAsync(q, row, src, c->stride * sizeof(double), row, c->nf, kind, c->stream));
    if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
    return SME_OK;
}

int sme_eigmax(sme_ctx *c, double *lam_max, double *dt)
{
    if (!c) return SME_EINVAL;
    if (!c->has_state) return fail(c, SME_EINVAL, "no state loaded");
    // clear the ratio words and the speed of the current slot (they precede t)
    HIPCHK(c, hipMemsetAsync(c->slots + c->sa, 0, offsetof(Slot, t), c->stream));
    StepArgs a = make_args(c);
    HIPCHK(c, launch_eig(0, c->kind, c->level, a, c->stream));
    Slot s;
    int r = read_slot(c, &s, nullptr);
    if (r) return r;
    double rr, ll;
    rr = slot_ratio(s);
    memcpy(&ll, &s.lbits, sizeof ll);
    if (lam_max) *lam_max = ll;
    if (dt) *dt = rr > 0 ? c->p.cfl / rr : 0.0;
    return SME_OK;
}

int sme_step(sme_ctx *c, double dt, double *dt_used)
{
    if (!c) return SME_EINVAL;
    if (!c->has_state) return fail(c, SME_EINVAL, "no state loaded");
    if (std::isnan(dt)) return SME_EINVAL;
    HIPCHK(c, launch_one_step(c, dt > 0 ? dt : 0.0, 0.0));
    if (dt_used) {
        Slot s;
        int r = read_slot(c, &s, nullptr);
        if (r) return r;
        *dt_used = s.dt;
    }
    return SME_OK;
}

int sme_run(sme_ctx *c, int64_t n_steps, double t_end, double *t_out, int64_t *steps_done)
{
    if (!c || n_steps < 0 || std::isnan(t_end)) return SME_EINVAL;
    if (!c->has_state) return fail(c, SME_EINVAL, "no state loaded");
    const double te = t_end > 0 ? t_end : 0.0;
    int64_t left = n_steps;
    const bool use_graphs = getenv("SME_NO_GRAPH") == nullptr;
    // With an end time every graph copies the device clock to pinned host
    // memory.  After queueing graph k the host waits for graph k - 2 and stops
    // once its clock has reached t_end: the device always has queued work, and
    // at most two graphs of no-op steps (dt = 0, a plain copy) follow the end.
    if (use_graphs && te > 0.0 && left >= kGraphSteps && !c->t_host) {
        HIPCHK(c, hipHostMalloc((void **)&c->t_host, sizeof(double), hipHostMallocDefault));
        for (auto &e : c->ev) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    // a small 1D grid without a closure: one workgroup takes the steps with the
    // state in LDS, up to kLdsRunSteps per launch (checking the clock between
    // launches when there is an end time)
    if (c->kind == SME_MESH_1D && !c->closure && !c->order2 && getenv("SME_NO_LDS_RUN") == nullptr &&
        (c->nx + 61) / 62 <= kLdsRunMaxWindows[c->level] &&
        run_1d_lds_bytes(c->level, (int)c->nx) + 1024 <= c->lds_optin) {
        while (left > 0) {
            const int k = (int)std::min<int64_t>(left, kLdsRunSteps);
            StepArgs a = make_args(c);
            a.dt_fixed = 0.0;
            a.t_end = te;
            HIPCHK(c, launch_run_1d_lds(c->level, a, k, c->q[(c->cur + k) % 2], c->stream));
            c->cur = (c->cur + k) % 2;
            c->sa = (c->sa + k) % 3;
            left -= k;
            if (te > 0.0 && left > 0) {
                Slot s;
                int rr = read_slot(c, &s, nullptr);
                if (rr) return rr;
                if (s.t >= te) break;
            }
        }
    }
    int64_t k = 0;
    while (use_graphs && left >= kGraphSteps) {
        hipGraphExec_t ex;
        int r = get_graph(c, te, &ex);
        if (r) return r;
        HIPCHK(c, hipGraphLaunch(ex, c->stream));
        left -= kGraphSteps;  // after six steps cur and slot are back where they started
        if (te > 0.0) {
            HIPCHK(c, hipEventRecord(c->ev[k % 3], c->stream));
            if (k >= 2) {
                // stream order: every earlier copy to t_host has landed, later ones only raise it
                HIPCHK(c, hipEventSynchronize(c->ev[(k - 2) % 3]));
                if (*(volatile double *)c->t_host >= te) {
                    left = 0;
                    break;
                }
            }
            ++k;
        }
    }
    // single launches (the remainder, or every step without graphs): with an
    // end time, look at the device clock after every kGraphSteps steps
    for (int64_t k = 1; left > 0; ++k, --left) {
        HIPCHK(c, launch_one_step(c, 0.0, te));
        if (te > 0.0 && left > 1 && k % kGraphSteps == 0) {
            Slot s;
            int rr = read_slot(c, &s, nullptr);
            if (rr) return rr;
            if (s.t >= te) break;
        }
    }
    if (t_out || steps_done) {
        Slot s;
        ErrWord e;
        int r = read_slot(c, &s, &e);
        if (r) return r;
        if (t_out) *t_out = s.t;
        if (steps_done) *steps_done = s.step;
        if (e.flag) return nonphys(c, e);
    }
    return SME_OK;
}

int sme_time(sme_ctx *c, double *t, int64_t *steps)
{
    if (!c) return SME_EINVAL;
    Slot s;
    ErrWord e;
    int r = read_slot(c, &s, &e);
    if (r) return r;
    if (t) *t = s.t;
    if (steps) *steps = s.step;
    if (e.flag) return nonphys(c, e);
    return SME_OK;
}

int sme_interpolate_3d(sme_ctx *c, int nz, const double *zeta, double rho, double *out)
{
    if (!c || !zeta || !out || nz < 1 || nz > kLiftMaxLevels || !(rho > 0) || !std::isfinite(rho)) return SME_EINVAL;
    if (!c->has_state) return fail(c, SME_EINVAL, "no state loaded");
    LiftArgs a{};
    for (int l = 0; l < nz; ++l) {
        if (!(zeta[l] >= 0.0 && zeta[l] <= 1.0)) return fail(c, SME_EINVAL, "sigma level %d outside [0, 1]", l);
        a.zeta[l] = zeta[l];
    }
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, out) != hipSuccess || at.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(c, SME_EINVAL, "output %p is not device memory", (void *)out);
    }
    a.q = c->q[c->cur];
    a.b = c->b;
    a.stride = c->stride;
    a.ncells = c->ncells;
    a.nx = (int)c->nx;
    a.ny = (int)c->ny;
    a.inv_dx = c->dx > 0 ? 1.0 / c->dx : 0.0;
    a.inv_dy = c->dy > 0 ? 1.0 / c->dy : 0.0;
    for (int s = 0; s < 4; ++s) a.bc[s] = c->bc[s];
    a.nbr = c->nbr;
    a.cx = c->cx;
    a.cy = c->cy;
    a.to_caller = c->to_caller;
    a.nz = nz;
    a.rho_g = rho * c->p.g;
    a.out = out;
    const int kind = c->kind == SME_MESH_1D ? 1 : (c->kind == SME_MESH_2D_STRUCT ? 2 : 3);
    HIPCHK(c, launch_lift(c->level, kind, a, c->stream));
    return SME_OK;
}

int sme_current(const sme_ctx *c) { return c ? c->cur : SME_EINVAL; }
int sme_nfields(const sme_ctx *c) { return c ? c->nf : SME_EINVAL; }
int64_t sme_ncells(const sme_ctx *c) { return c ? c->ncells : SME_EINVAL; }
int sme_level(const sme_ctx *c) { return c ? c->level : SME_EINVAL; }
const double *sme_state_device(const sme_ctx *c) { return c ? c->q[c->cur] : nullptr; }
int64_t sme_field_stride(const sme_ctx *c) { return c ? c->stride : SME_EINVAL; }

int sme_basis_tensors(int level, double *M, double *A, double *B, double *K)
{
    switch (level) {
    case 0: copy_tensors<0>(M, A, B, K); return SME_OK;
    case 1: copy_tensors<1>(M, A, B, K); return SME_OK;
    case 2: copy_tensors<2>(M, A, B, K); return SME_OK;
    case 3: copy_tensors<3>(M, A, B, K); return SME_OK;
    case 4: copy_tensors<4>(M, A, B, K); return SME_OK;
    case 5: copy_tensors<5>(M, A, B, K); return SME_OK;
    case 6: copy_tensors<6>(M, A, B, K); return SME_OK;
    case 7: copy_tensors<7>(M, A, B, K); return SME_OK;
    case 8: copy_tensors<8>(M, A, B, K); return SME_OK;
    default: return SME_EINVAL;
    }
}

// ---- hooks for the closure front end (sme_closure.cpp) ----
__attribute__((visibility("hidden"))) int sme_internal_attach(sme_ctx *c, const ClosureModel *m_host)
{
    if (!c) return SME_EINVAL;
    if (!m_host) {
        (void)hipFree(c->closure);
        (void)hipFree(c->rates);
        c->closure = nullptr;
        c->rates = nullptr;
        drop_graphs(c);
        return SME_OK;
    }
    if (c->level != 1 || c->kind == SME_MESH_2D_TRI || c->order2)
        return fail(c, SME_EINVAL, "the learned closure acts on level-1 1D and structured 2D grids, first order");
    if (!c->closure) {
        if (dalloc(c, &c->closure, 1)) return SME_ENOMEM;
    }
    if (!c->rates) {
        const int64_t per = c->kind == SME_MESH_1D ? 2 : 4;
        if (dalloc(c, &c->rates, per * c->stride)) return SME_ENOMEM;
    }
    if (!c->oor) {
        if (dalloc(c, &c->oor, 1)) return SME_ENOMEM;
        HIPCHK(c, hipMemset(c->oor, 0, sizeof(unsigned long long)));
    }
    if (m_host->precision != kClosureFp32 && m_host->precision != kClosureFp16Mfma)
        return fail(c, SME_EINVAL, "unknown closure precision %d", m_host->precision);
    HIPCHK(c, hipMemcpyAsync(c->closure, m_host, sizeof(ClosureModel), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->closure_mode = m_host->precision;
    c->cus = host::device_cus();
    drop_graphs(c);
    return SME_OK;
}

__attribute__((visibility("hidden"))) int sme_internal_oor(sme_ctx *c, int64_t *count)
{
    if (!c) return SME_EINVAL;
    unsigned long long v = 0;
    if (c->oor) {
        HIPCHK(c, hipMemcpyAsync(&v, c->oor, sizeof v, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    *count = (int64_t)v;
    return SME_OK;
}

__attribute__((visibility("hidden"))) hipStream_t sme_internal_stream(sme_ctx *c) { return c ? c->stream : nullptr; }

int sme_closure_run(sme_ctx *c1, sme_ctx *c8, double t_end, int64_t chunk, int64_t max_steps,
                    double max_out_of_range, double *t_out, int64_t *steps_done, double *fallback_at)
{
    if (!c1 || !c8 || !(t_end > 0) || chunk < 1 || max_steps < 1 || !(max_out_of_range >= 0)) return SME_EINVAL;
    if (!c1->closure) return fail(c1, SME_EINVAL, "no closure attached");
    if (!c1->has_state) return fail(c1, SME_EINVAL, "no state loaded");
    if (c8->kind != c1->kind || c8->nx != c1->nx || c8->ny != c1->ny || c8->level < 2)
        return fail(c1, SME_EINVAL, "the fallback context must be a higher level on the same grid");
    if (!c1->ckpt && dalloc(c1, &c1->ckpt, (size_t)c1->nf * c1->stride)) return SME_ENOMEM;
    const size_t bytes = (size_t)c1->nf * c1->stride * sizeof(double);
    if (fallback_at) *fallback_at = -1.0;
    Slot s;
    int r = read_slot(c1, &s, nullptr);
    if (r) return r;
    double t = s.t;
    int64_t steps = s.step;
    int64_t oor = 0;
    r = sme_internal_oor(c1, &oor);
    if (r) return r;
    const int64_t step0 = steps;
    while (t < t_end && steps - step0 < max_steps) {
        // checkpoint of the chunk's start (device to device)
        HIPCHK(c1, hipMemcpyAsync(c1->ckpt, c1->q[c1->cur], bytes, hipMemcpyDeviceToDevice, c1->stream));
        double t1;
        int64_t n1;
        r = sme_run(c1, std::min(chunk, max_steps - (steps - step0)), t_end, &t1, &n1);
        if (r) return r;
        int64_t oor1 = 0;
        r = sme_internal_oor(c1, &oor1);
        if (r) return r;
        const int64_t n = n1 - steps;
        if ((double)(oor1 - oor) > max_out_of_range * (double)c1->ncells * (double)std::max<int64_t>(1, n)) {
            // the network left its training range in this chunk: redo it, and
            // the rest of the run, with the fallback level from the chunk's
            // start, lifted (the higher moments start at zero)
            if (fallback_at) *fallback_at = t;
            double *dst = c8->q[c8->cur];
            const int nb = c1->kind == SME_MESH_1D ? 1 : 2;  // moment blocks
            const int n1m = 2, n8m = c8->level + 1;             // moments per block
            HIPCHK(c1, hipStreamSynchronize(c1->stream));
            HIPCHK(c8, hipMemsetAsync(dst, 0, (size_t)c8->nf * c8->stride * sizeof(double), c8->stream));
            HIPCHK(c8, hipMemcpyAsync(dst, c1->ckpt, (size_t)c1->stride * sizeof(double), hipMemcpyDeviceToDevice,
                                      c8->stream));
            for (int blk = 0; blk < nb; ++blk)
                HIPCHK(c8, hipMemcpyAsync(dst + (1 + (int64_t)blk * n8m) * c8->stride,
                                          c1->ckpt + (1 + (int64_t)blk * n1m) * c1->stride,
                                          (size_t)n1m * c1->stride * sizeof(double), hipMemcpyDeviceToDevice,
                                          c8->stream));
            r = sme_set_state(c8, dst, 1);
            if (r) return r;
            double t8;
            int64_t n8;
            r = sme_run(c8, max_steps - (steps - step0), t_end - t, &t8, &n8);
            if (r) return r;
            if (t_out) *t_out = t + t8;
            if (steps_done) *steps_done = steps + n8;
            return SME_OK;
        }
        oor = oor1;
        steps = n1;
        if (n == 0) break;
        t = t1;
    }
    if (t_out) *t_out = t;
    if (steps_done) *steps_done = steps;
    return SME_OK;
}

const char *sme_strerror(int code)
{
    switch (code) {
    case SME_OK: return "ok";
    case SME_EINVAL: return "invalid argument";
    case SME_ENOMEM: return "out of memory";
    case SME_EHIP: return "HIP runtime error";
    case SME_ENONPHYS: return "non-physical state";
    case SME_EMESH: return "invalid mesh";
    default: return "unknown error";
    }
}

const char *sme_last_error(const sme_ctx *c) { return c ? c->last.c_str() : "no context"; }

void sme_destroy(sme_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    (void)hipFree(c->b);
    (void)hipFree(c->nbr);
    (void)hipFree(c->fsx);
    (void)hipFree(c->fsy);
    (void)hipFree(c->ivol);
    (void)hipFree(c->cx);
    (void)hipFree(c->cy);
    (void)hipFree(c->to_internal);
    (void)hipFree(c->to_caller);
    (void)hipFree(c->slots);
    (void)hipFree(c->err);
    (void)hipFree(c->quad_dev);
    (void)hipFree(c->closure);
    (void)hipFree(c->oor);
    (void)hipFree(c->rates);
    (void)hipFree(c->ckpt);
    (void)hipFree(c->slopes);
    if (c->t_host) (void)hipHostFree(c->t_host);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
