// sme_static.cpp -- sme_step_static: one SME step on caller buffers without any
// allocation (for code under HIP graph capture, tight serving loops and other
// callers that cannot call hipMalloc).
//
// The step kernels need a little device scratch besides the state: the three
// rotating time-step slots (CFL-ratio words, time, step count), the
// non-physical-state word and, for rules other than 3-point Gauss, the
// Gauss-Legendre points.  Here that scratch is one static device array per
// GPU, `scratch`, of kScratchBytes.  Its device address is taken once per
// device (hipGetSymbolAddress with that device current) and kept; host code
// never uses the array's name itself.  A small fill kernel (no memset, so the
// call can be captured into a graph) clears the slots and writes the Gauss
// points at the start of every call.  Every call on a device shares that
// device's array: calls that overlap on one GPU (different streams, or
// different host threads) race on it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "../../include/sme.h"
#include "sme_host.h"
#include "sme_kernels.h"

using namespace sme;

namespace {

constexpr size_t kScratchBytes = 8192;
constexpr int kMaxDevices = 64;

struct StaticScratch {
    Slot slots[3];
    ErrWord err;
    double quad[2 * kMaxQuad];  // Gauss points, then weights
};
static_assert(sizeof(StaticScratch) <= kScratchBytes, "scratch layout exceeds the static array");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceEntry {
    StaticScratch *ptr = nullptr;  // device address of `scratch` on that device
    int cus = 0;
};
DeviceEntry g_dev[kMaxDevices];
std::mutex g_mu;

struct QuadInit {
    double v[2 * kMaxQuad];
};

// clear the slots and the error word, write the Gauss points (one wave)
__global__ void k_static_init(StaticScratch *s, QuadInit q)
{
    const int t = threadIdx.x;
    if (t < 2 * kMaxQuad) s->quad[t] = q.v[t];
    if (t < 3) {
        for (int w = 0; w < kRatioWords; ++w) s->slots[t].r[w].bits = 0ull;
        s->slots[t].lbits = 0ull;
        s->slots[t].t = 0.0;
        s->slots[t].dt = 0.0;
        s->slots[t].step = 0;
    }
    if (t == 0) {
        s->err.flag = 0u;
        s->err.first_step = ~0ull;
    }
}

// Device address of this device's scratch array, taken on first use.
hipError_t scratch_of(int dev, DeviceEntry *out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceEntry &e = g_dev[dev];
    if (!e.ptr) {
        void *p = nullptr;
        hipError_t r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (r != hipSuccess) return r;
        if (!p) return hipErrorInvalidSymbol;
        e.cus = host::device_cus();
        e.ptr = (StaticScratch *)p;
    }
    *out = e;
    return hipSuccess;
}

bool aligned256(const void *p) { return ((uintptr_t)p & 255u) == 0; }

}  // namespace

extern "C" int sme_step_static(int level, const sme_mesh *mesh, const sme_params *params, const double *q,
                               double *q_next, int64_t field_stride, const double *b, double dt, double *dt_used,
                               void *stream)
{
    int nf = 0;
    int64_t nc = 0;
    if (!mesh || !params || !q || !q_next || !b || q == q_next || std::isnan(dt)) return SME_EINVAL;
    if (mesh->kind != SME_MESH_1D && mesh->kind != SME_MESH_2D_STRUCT) return SME_EINVAL;
    int r = sme_layout(level, mesh, &nf, &nc, nullptr);
    if (r) return r;
    if (params->quad_points < 1 || params->quad_points > kMaxQuad || !(params->cfl > 0) || !(params->g > 0) ||
        params->c_slip < 0 || params->nu < 0 || (params->implicit_friction != 0 && params->implicit_friction != 1) ||
        params->order != 1)
        return SME_EINVAL;
    if (field_stride < nc || field_stride % 256 != 0 || !aligned256(q) || !aligned256(q_next) || !aligned256(b))
        return SME_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SME_EHIP;
    DeviceEntry ent;
    if (scratch_of(dev, &ent) != hipSuccess) return SME_EHIP;
    StaticScratch *S = ent.ptr;
    const hipStream_t st = (hipStream_t)stream;

    QuadInit qi{};
    double qs[kMaxQuad] = {0}, qw[kMaxQuad] = {0};
    host::gauss_legendre01(params->quad_points, qs, qw);
    std::memcpy(qi.v, qs, sizeof qs);
    std::memcpy(qi.v + kMaxQuad, qw, sizeof qw);

    StepArgs a{};
    a.q = q;
    a.qn = q_next;
    a.b = b;
    a.stride = field_stride;
    a.ncells = nc;
    a.nx = (int)mesh->nx;
    a.ny = mesh->kind == SME_MESH_1D ? 1 : (int)mesh->ny;
    // the same spacing arithmetic as sme_init: dx = (x1 - x0) / nx, then 1 / dx
    a.idx = 1.0 / ((mesh->x1 - mesh->x0) / mesh->nx);
    a.idy = mesh->kind == SME_MESH_2D_STRUCT ? 1.0 / ((mesh->y1 - mesh->y0) / mesh->ny) : 0.0;
    for (int s = 0; s < 4; ++s) a.bc[s] = mesh->bc[s];
    a.rows = mesh->kind == SME_MESH_2D_STRUCT ? host::pick_rows(level, mesh->nx, mesh->ny, ent.cus) : 16;
    a.g = params->g;
    a.c_slip = params->c_slip;
    a.implicit = params->implicit_friction;
    a.nu = params->nu;
    a.cfl = params->cfl;
    a.quad.n = params->quad_points;
    a.quad.s0 = qs[0];
    a.quad.s1 = qs[1];
    a.quad.s2 = qs[2];
    a.quad.w0 = qw[0];
    a.quad.w1 = qw[1];
    a.quad.w2 = qw[2];
    a.quad.s = S->quad;
    a.quad.w = S->quad + kMaxQuad;
    a.dt_fixed = dt > 0 ? dt : 0.0;
    a.t_end = 0.0;
    a.slots = S->slots;
    a.sa = 0;
    a.sb = 1;
    a.sc = 2;
    a.err = &S->err;

    hipLaunchKernelGGL(k_static_init, dim3(1), dim3(64), 0, st, S, qi);
    hipError_t e = hipGetLastError();
    const int kind = mesh->kind == SME_MESH_1D ? 1 : 2;
    // the CFL step of q (the eigenvalue-bound reduction into slot 0)
    if (e == hipSuccess && !(dt > 0)) e = launch_eig(kind, kind, level, a, st);
    if (e == hipSuccess) e = kind == 1 ? launch_step_1d(level, a, st) : launch_step_2d(level, a, st);
    if (e != hipSuccess) return SME_EHIP;
    if (dt_used) {
        double used = 0.0;
        ErrWord ew{};
        e = hipMemcpyAsync(&used, &S->slots[1].dt, sizeof used, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&ew, &S->err, sizeof ew, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return SME_EHIP;
        *dt_used = used;
        if (ew.flag) return SME_ENONPHYS;
    }
    return SME_OK;
}
