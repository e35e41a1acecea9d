// sme_vam.cpp -- host side of the non-hydrostatic VAM channel (C ABI in
// include/sme.h, kernels in k_vam.hip).
//
// Binds the caller's two state buffers, owns the bathymetry, the pressure,
// the block-tridiagonal system of the corrector with its reduction levels and
// their factors, and the time slots, and queues the kernels of a step on the
// caller's stream: predictor; assembly, reduction levels, back substitution
// and pressure update; the residual at that pressure, the same levels for
// the right-hand side alone, back substitution and pressure increment; then
// the correction.  The step size is computed on the device from the CFL
// ratio of the previous state, as in the SME step.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/sme.h"
#include "sme_host.h"
#include "sme_vam.h"

using namespace sme;

struct sme_vam {
    int64_t nx = 0, stride = 0;
    int nb = 0;
    double dx = 0.0, g = 9.81, cfl = 0.45;
    Quad quad{};
    double *quad_dev = nullptr;
    double *q[2] = {nullptr, nullptr};  // caller-owned
    int cur = 0;
    double *b = nullptr, *p = nullptr, *sys = nullptr;
    std::vector<VamSystem> lev;   // reduction levels: lev[0] the assembled system
    std::vector<int> nlev;        // equations per level
    std::vector<double *> xlev;   // unknowns per level [4][n_l]
    int l0 = 0;                   // first level of the one-workgroup tail
    VamTail *tail = nullptr;      // its description, in device memory
    Slot *slots = nullptr;
    ErrWord *err = nullptr;
    int sa = 0;
    bool has_state = false;
    hipStream_t stream = nullptr;
    int device = 0;
    std::string last;
};

namespace {

constexpr int kMaxQuadVam = 8;
constexpr int kNewtonSolves = 2;  // linear solves per corrector

int vfail(sme_vam *c, int code, const char *fmt, ...)
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

#define VCHK(ctx, call)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return vfail((ctx), SME_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

int64_t vam_stride(int64_t nx) { return (nx + 255) / 256 * 256; }

template <typename T>
int valloc(sme_vam *c, T **p, size_t count)
{
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return vfail(c, e == hipErrorOutOfMemory ? SME_ENOMEM : SME_EHIP, "hipMalloc(%zu bytes): %s",
                     count * sizeof(T), hipGetErrorString(e));
    }
    return SME_OK;
}

// equations of the reduction levels: nb, nb / 2, ... down to one
std::vector<int> level_sizes(int nb)
{
    std::vector<int> n{nb};
    while (n.back() > 1) n.push_back(n.back() / 2);
    return n;
}

// doubles of the block systems (A, B, C: 16 each, d: 4 per equation), of
// the unknowns (4 per equation) and of the even equations' factors (52 per
// even equation) of every level
size_t system_doubles(int nb)
{
    size_t t = 0;
    for (int n : level_sizes(nb)) t += (size_t)56 * n + (size_t)52 * ((n + 1) / 2);
    return t;
}

VamArgs make_args(const sme_vam *c, double t_end, double dt_fixed)
{
    VamArgs a{};
    a.q = c->q[c->cur];
    a.qs = c->q[1 - c->cur];
    a.b = c->b;
    a.p = c->p;
    a.stride = c->stride;
    a.nx = (int)c->nx;
    a.nb = c->nb;
    a.dx = c->dx;
    a.g = c->g;
    a.cfl = c->cfl;
    a.quad = c->quad;
    a.t_end = t_end;
    a.dt_fixed = dt_fixed;
    a.slots = c->slots;
    a.sa = c->sa;
    a.sb = (c->sa + 1) % 3;
    a.sc = (c->sa + 2) % 3;
    a.err = c->err;
    return a;
}

// a caller's state buffer: device memory of the current device, 256-byte aligned, long enough
int check_buffer(sme_vam *c, const void *p, size_t bytes)
{
    if (((uintptr_t)p & 255u) != 0) return vfail(c, SME_EINVAL, "state buffer %p is not 256-byte aligned", p);
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess || at.type != hipMemoryTypeDevice || at.device != c->device) {
        (void)hipGetLastError();
        return vfail(c, SME_EINVAL, "state buffer %p is not device memory of device %d", p, c->device);
    }
    void *base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange((hipDeviceptr_t *)&base, &size, (hipDeviceptr_t)p) == hipSuccess && base) {
        if ((const char *)p + bytes > (const char *)base + size)
            return vfail(c, SME_EINVAL, "state buffer %p holds fewer than %zu bytes", p, bytes);
    } else {
        (void)hipGetLastError();
    }
    return SME_OK;
}

// queue one step: predictor, corrector, CFL ratio of the new state
int queue_step(sme_vam *c, double t_end, double dt_fixed)
{
    VamArgs a = make_args(c, t_end, dt_fixed);
    VCHK(c, launch_vam_predict(a, c->stream));
    // Newton on the affine constraints: the first solve from P = 0, then one
    // more with the residual at the pressure found (see k_vam.hip)
    // levels [0, l0) by one launch each, levels [l0, L) by one wave in LDS
    const int l0 = c->l0;
    for (int it = 0; it < kNewtonSolves; ++it) {
        // the matrix does not depend on P: factored by the first solve, reused after
        const bool rhs = it > 0;
        VCHK(c, rhs ? launch_vam_residual(a, c->lev[0], c->stream) : launch_vam_assemble(a, c->lev[0], c->stream));
        for (int l = 0; l < l0; ++l)
            VCHK(c, launch_vam_reduce(c->nlev[l], c->lev[l], c->lev[l + 1], rhs, c->stream));
        VCHK(c, launch_vam_tail(c->tail, rhs, c->stream));
        for (int l = l0 - 1; l >= 0; --l)
            VCHK(c, launch_vam_back(c->nlev[l], c->lev[l], c->xlev[l + 1], c->xlev[l], c->stream));
        VCHK(c, launch_vam_scatter(a, c->xlev[0], it, c->stream));
    }
    VCHK(c, launch_vam_correct(a, c->stream));
    c->cur = 1 - c->cur;
    c->sa = (c->sa + 1) % 3;
    return SME_OK;
}

int check_err(sme_vam *c)
{
    ErrWord e{};
    VCHK(c, hipMemcpyAsync(&e, c->err, sizeof e, hipMemcpyDeviceToHost, c->stream));
    VCHK(c, hipStreamSynchronize(c->stream));
    if (e.flag) return vfail(c, SME_ENONPHYS, "non-physical state (h <= 0 or non-finite) at step %llu", e.first_step);
    return SME_OK;
}

}  // namespace

extern "C" {

int sme_vam_layout(int64_t nx, int64_t *field_stride)
{
    if (nx < 1 || nx > ((int64_t)1 << 30) || !field_stride) return SME_EINVAL;
    *field_stride = vam_stride(nx);
    return SME_OK;
}

int sme_vam_workspace_size(int64_t nx, size_t *bytes)
{
    if (nx < 1 || nx > ((int64_t)1 << 30) || !bytes) return SME_EINVAL;
    const int64_t st = vam_stride(nx);
    const int nb = (int)((nx + 1) / 2);
    *bytes = sizeof(double) * (size_t)(st + 2 * st + system_doubles(nb) + 2 * kMaxQuadVam) + sizeof(VamTail) +
             3 * sizeof(Slot) + sizeof(ErrWord);
    return SME_OK;
}

int sme_vam_init(sme_vam **out, int64_t nx, double x0, double x1, double g, double cfl, int quad_points,
                 double *const q_dev[2], const double *b, int b_on_device, void *stream)
{
    if (!out) return SME_EINVAL;
    *out = nullptr;
    if (nx < 1 || nx > ((int64_t)1 << 30) || !(x1 > x0) || !(g > 0) || !(cfl > 0) || quad_points < 1 ||
        quad_points > kMaxQuadVam || !q_dev || !q_dev[0] || !q_dev[1] || q_dev[0] == q_dev[1])
        return SME_EINVAL;
    sme_vam *c = new (std::nothrow) sme_vam();
    if (!c) return SME_ENOMEM;
    c->nx = nx;
    c->stride = vam_stride(nx);
    c->nb = (int)((nx + 1) / 2);
    c->dx = (x1 - x0) / (double)nx;
    c->g = g;
    c->cfl = cfl;
    c->stream = (hipStream_t)stream;
    int rc = hipGetDevice(&c->device) == hipSuccess ? SME_OK : vfail(c, SME_EHIP, "hipGetDevice failed");
    for (int k = 0; k < 2 && !rc; ++k) rc = check_buffer(c, q_dev[k], (size_t)5 * c->stride * sizeof(double));
    c->q[0] = q_dev[0];
    c->q[1] = q_dev[1];
    double qs[kMaxQuadVam] = {0}, qw[kMaxQuadVam] = {0};
    host::gauss_legendre01(quad_points, qs, qw);
    c->quad.n = quad_points;
    c->quad.s0 = qs[0];
    c->quad.s1 = qs[1];
    c->quad.s2 = qs[2];
    c->quad.w0 = qw[0];
    c->quad.w1 = qw[1];
    c->quad.w2 = qw[2];
    rc = rc ? rc : valloc(c, &c->quad_dev, 2 * kMaxQuadVam);
    rc = rc ? rc : valloc(c, &c->b, c->stride);
    rc = rc ? rc : valloc(c, &c->p, 2 * c->stride);
    rc = rc ? rc : valloc(c, &c->sys, system_doubles(c->nb));
    rc = rc ? rc : valloc(c, &c->tail, 1);
    rc = rc ? rc : valloc(c, &c->slots, 3);
    rc = rc ? rc : valloc(c, &c->err, 1);
    if (!rc) {
        double buf[2 * kMaxQuadVam];
        memcpy(buf, qs, sizeof qs);
        memcpy(buf + kMaxQuadVam, qw, sizeof qw);
        if (hipMemcpy(c->quad_dev, buf, sizeof buf, hipMemcpyHostToDevice) != hipSuccess)
            rc = vfail(c, SME_EHIP, "quadrature upload failed");
        c->quad.s = c->quad_dev;
        c->quad.w = c->quad_dev + kMaxQuadVam;
        c->nlev = level_sizes(c->nb);
        double *base = c->sys;
        for (int n : c->nlev) {
            VamSystem m;
            m.A = base;
            m.B = base + 16 * (size_t)n;
            m.C = base + 32 * (size_t)n;
            m.d = base + 48 * (size_t)n;
            m.fac = base + 56 * (size_t)n;
            c->lev.push_back(m);
            c->xlev.push_back(base + 52 * (size_t)n);
            base += 56 * (size_t)n + 52 * (size_t)((n + 1) / 2);
        }
        const int L = (int)c->nlev.size();
        while (c->nlev[c->l0] > kTailMax) ++c->l0;
        VamTail tail{};
        tail.count = L - c->l0;
        for (int l = c->l0; l < L; ++l) {
            tail.m[l - c->l0] = c->lev[l];
            tail.x[l - c->l0] = c->xlev[l];
            tail.n[l - c->l0] = c->nlev[l];
        }
        if (!rc && hipMemcpy(c->tail, &tail, sizeof tail, hipMemcpyHostToDevice) != hipSuccess)
            rc = vfail(c, SME_EHIP, "reduction tail upload failed");
    }
    if (!rc) {
        hipError_t e = hipMemsetAsync(c->b, 0, c->stride * sizeof(double), c->stream);
        if (e == hipSuccess && b)
            e = hipMemcpyAsync(c->b, b, nx * sizeof(double), b_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                               c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->p, 0, 2 * c->stride * sizeof(double), c->stream);
        if (e == hipSuccess) e = launch_slots_reset(c->slots, c->err, 0, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = vfail(c, SME_EHIP, "initialisation: %s", hipGetErrorString(e));
    }
    if (rc) {
        sme_vam_destroy(c);
        return rc;
    }
    *out = c;
    return SME_OK;
}

int sme_vam_set_state(sme_vam *c, const double *q, int on_device)
{
    if (!c || !q) return SME_EINVAL;
    const size_t row = c->nx * sizeof(double);
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (q == c->q[0] || q == c->q[1]) {
        if (!on_device) return vfail(c, SME_EINVAL, "a bound state buffer is device memory");
        c->cur = q == c->q[0] ? 0 : 1;
    } else {
        VCHK(c, hipMemcpy2DAsync(c->q[c->cur], c->stride * sizeof(double), q, row, row, 5, kind, c->stream));
    }
    c->sa = 0;
    VCHK(c, launch_slots_reset(c->slots, c->err, 0, c->stream));
    VamArgs a = make_args(c, 0.0, 0.0);
    VCHK(c, launch_vam_eig(a, c->stream));
    c->has_state = true;
    VCHK(c, hipStreamSynchronize(c->stream));
    return check_err(c);
}

int sme_vam_get_state(sme_vam *c, double *q, int on_device)
{
    if (!c || !q) return SME_EINVAL;
    const size_t row = c->nx * sizeof(double);
    VCHK(c, hipMemcpy2DAsync(q, row, c->q[c->cur], c->stride * sizeof(double), row, 5,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    VCHK(c, hipStreamSynchronize(c->stream));
    return SME_OK;
}

int sme_vam_pressure(sme_vam *c, double *p, int on_device)
{
    if (!c || !p) return SME_EINVAL;
    const size_t row = c->nx * sizeof(double);
    VCHK(c, hipMemcpy2DAsync(p, row, c->p, c->stride * sizeof(double), row, 2,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    VCHK(c, hipStreamSynchronize(c->stream));
    return SME_OK;
}

int sme_vam_step(sme_vam *c, double dt, double *dt_used)
{
    if (!c) return SME_EINVAL;
    if (!c->has_state) return vfail(c, SME_EINVAL, "no state loaded");
    int rc = queue_step(c, 0.0, dt > 0.0 ? dt : 0.0);
    if (rc) return rc;
    if (dt_used) {
        Slot s{};
        VCHK(c, hipMemcpyAsync(&s, c->slots + c->sa, sizeof s, hipMemcpyDeviceToHost, c->stream));
        VCHK(c, hipStreamSynchronize(c->stream));
        *dt_used = s.dt;
    }
    return check_err(c);
}

int sme_vam_run(sme_vam *c, int64_t n_steps, double t_end, double *t_out, int64_t *steps_done)
{
    if (!c || n_steps < 0) return SME_EINVAL;
    if (!c->has_state) return vfail(c, SME_EINVAL, "no state loaded");
    for (int64_t k = 0; k < n_steps; ++k) {
        int rc = queue_step(c, t_end > 0.0 ? t_end : 0.0, 0.0);
        if (rc) return rc;
    }
    int rc = check_err(c);
    if (rc) return rc;
    if (t_out || steps_done) {
        Slot s{};
        VCHK(c, hipMemcpy(&s, c->slots + c->sa, sizeof s, hipMemcpyDeviceToHost));
        if (t_out) *t_out = s.t;
        if (steps_done) *steps_done = s.step;
    }
    return SME_OK;
}

int sme_vam_time(sme_vam *c, double *t, int64_t *steps)
{
    if (!c) return SME_EINVAL;
    Slot s{};
    VCHK(c, hipMemcpyAsync(&s, c->slots + c->sa, sizeof s, hipMemcpyDeviceToHost, c->stream));
    VCHK(c, hipStreamSynchronize(c->stream));
    if (t) *t = s.t;
    if (steps) *steps = s.step;
    return SME_OK;
}

int sme_vam_current(const sme_vam *c) { return c ? c->cur : SME_EINVAL; }

int64_t sme_vam_field_stride(const sme_vam *c) { return c ? c->stride : SME_EINVAL; }

const char *sme_vam_last_error(const sme_vam *c) { return c ? c->last.c_str() : ""; }

void sme_vam_destroy(sme_vam *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->quad_dev);
    (void)hipFree(c->b);
    (void)hipFree(c->p);
    (void)hipFree(c->sys);
    (void)hipFree(c->tail);
    (void)hipFree(c->slots);
    (void)hipFree(c->err);
    delete c;
}

}  // extern "C"
