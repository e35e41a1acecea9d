// sme_batch.cpp -- host side of the batched ensemble (sme_batch_* in include/sme.h).
//
// All grids live in two packed state arenas (ping-pong) and one bathymetry
// arena.  The work list holds one item per (grid, strip, band); in one
// persistent launch per step the resident waves take the items in list order
// from a device counter.  Runs of six steps are captured as HIP graphs (six = lcm of the
// arena ping-pong period 2 and the time-slot period 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/sme.h"
#include "sme_host.h"
#include "sme_kernels.h"

using namespace sme;

namespace {
constexpr int kBatchGraphSteps = 6;
constexpr int kArenaAlign = 256;  // elements
}  // namespace

struct sme_batch {
    int n = 0;
    sme_params p{};
    Quad quad{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<int> level, nx, ny, nf;
    std::vector<int64_t> offset, stride, boff;
    std::vector<double> dx, dy;
    std::vector<std::array<int, 4>> bc;
    int rows[kBatchMaxLevel + 1] = {8, 8, 8, 8, 8};
    int64_t cells = 0;
    double *q[2] = {nullptr, nullptr};
    double *b = nullptr;
    double *quad_dev = nullptr;
    BatchInst *inst = nullptr;
    BatchItem *items = nullptr;
    int nitems = 0;
    int items_cap = 0;
    Slot *slots = nullptr;
    unsigned *work = nullptr;  // the work counters of the three time slots
    ErrWord *err = nullptr;
    int cur = 0, sa = 0;
    int grid = 0;
    hipGraphExec_t graph[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    std::string last;
};

namespace {

int bfail(sme_batch *b, int code, const char *fmt, ...)
{
    if (b) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        b->last = buf;
    }
    return code;
}

#define BCHK(bt, call)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return bfail((bt), SME_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

void drop_graphs(sme_batch *b)
{
    for (auto &row : b->graph)
        for (auto &g : row) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

int nsx_of(int nx) { return (nx + 61) / 62; }

// one item per (grid, strip, band), costliest level first
int build_items(sme_batch *b)
{
    std::vector<BatchItem> it;
    std::vector<int> order(b->n);
    for (int i = 0; i < b->n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->level[x] > b->level[y]; });
    for (int i : order) {
        const int r = b->rows[b->level[i]];
        const int sx = nsx_of(b->nx[i]), sy = (b->ny[i] + r - 1) / r;
        for (int y = 0; y < sy; ++y)
            for (int x = 0; x < sx; ++x) it.push_back(BatchItem{i, x, y, 0});
    }
    if ((int)it.size() > b->items_cap) {
        if (b->items) (void)hipFree(b->items);
        b->items = nullptr;
        BCHK(b, hipMalloc((void **)&b->items, it.size() * sizeof(BatchItem)));
        b->items_cap = (int)it.size();
    }
    BCHK(b, hipMemcpy(b->items, it.data(), it.size() * sizeof(BatchItem), hipMemcpyHostToDevice));
    b->nitems = (int)it.size();
    std::vector<BatchInst> tab(b->n);
    for (int i = 0; i < b->n; ++i) {
        BatchInst &t = tab[i];
        t.level = b->level[i];
        t.nx = b->nx[i];
        t.ny = b->ny[i];
        t.rows = b->rows[t.level];
        for (int s = 0; s < 4; ++s) t.bc[s] = b->bc[i][s];
        t.offset = b->offset[i];
        t.stride = b->stride[i];
        t.boff = b->boff[i];
        t.idx = 1.0 / b->dx[i];
        t.idy = 1.0 / b->dy[i];
    }
    BCHK(b, hipMemcpy(b->inst, tab.data(), tab.size() * sizeof(BatchInst), hipMemcpyHostToDevice));
    // persistent grid: every resident wave slot of the device, at most one wave per item
    const int per_simd = batch_waves_per_simd();
    const int full = host::device_cus() * per_simd;  // blocks of 4 waves
    b->grid = std::max(1, std::min(full, (b->nitems + 3) / 4));
    drop_graphs(b);
    return SME_OK;
}

BatchArgs make_args(const sme_batch *b)
{
    BatchArgs a{};
    a.q = b->q[b->cur];
    a.qn = b->q[1 - b->cur];
    a.b = b->b;
    a.inst = b->inst;
    a.items = b->items;
    a.nitems = b->nitems;
    a.slots = b->slots;
    a.sa = b->sa;
    a.sb = (b->sa + 1) % 3;
    a.sc = (b->sa + 2) % 3;
    a.work = b->work;
    a.err = b->err;
    a.g = b->p.g;
    a.c_slip = b->p.c_slip;
    a.implicit = b->p.implicit_friction;
    a.nu = b->p.nu;
    a.cfl = b->p.cfl;
    a.quad = b->quad;
    return a;
}

hipError_t one_step(sme_batch *b)
{
    hipError_t e = launch_batch_step(make_args(b), b->grid, b->stream);
    if (e == hipSuccess) {
        b->cur = 1 - b->cur;
        b->sa = (b->sa + 1) % 3;
    }
    return e;
}

// single-grid view of grid i for the stand-alone reduction kernel
StepArgs inst_args(const sme_batch *b, int i)
{
    StepArgs a{};
    a.q = b->q[b->cur] + b->offset[i];
    a.qn = b->q[1 - b->cur] + b->offset[i];
    a.b = b->b + b->boff[i];
    a.stride = b->stride[i];
    a.ncells = (int64_t)b->nx[i] * b->ny[i];
    a.nx = b->nx[i];
    a.ny = b->ny[i];
    a.idx = 1.0 / b->dx[i];
    a.idy = 1.0 / b->dy[i];
    for (int s = 0; s < 4; ++s) a.bc[s] = b->bc[i][s];
    a.g = b->p.g;
    a.cfl = b->p.cfl;
    a.slots = b->slots + 3 * i;
    a.sa = b->sa;
    a.sb = (b->sa + 1) % 3;
    a.sc = (b->sa + 2) % 3;
    a.err = b->err;
    return a;
}

int load_state(sme_batch *b, int i, const double *q, hipMemcpyKind kind)
{
    const size_t row = (size_t)b->nx[i] * b->ny[i] * sizeof(double);
    BCHK(b, hipMemcpy2DAsync(b->q[b->cur] + b->offset[i], b->stride[i] * sizeof(double), q, row, row, b->nf[i], kind,
                             b->stream));
    // fresh clock for this grid, CFL ratio of its new state
    BCHK(b, launch_slots_reset(b->slots + 3 * i, nullptr, 0, b->stream));  // all three slots of grid i
    BCHK(b, launch_eig(2, SME_MESH_2D_STRUCT, b->level[i], inst_args(b, i), b->stream));
    return SME_OK;
}

}  // namespace

extern "C" {

int sme_batch_init(sme_batch **out, int n, const int *levels, const sme_mesh *meshes, const double *const *bath,
                   const sme_params *params, void *stream)
{
    if (!out || n < 1 || !levels || !meshes || !params) return SME_EINVAL;
    *out = nullptr;
    if (params->quad_points < 1 || params->quad_points > kMaxQuad || !(params->cfl > 0) || !(params->g > 0) ||
        params->c_slip < 0 || params->nu < 0 || (params->implicit_friction != 0 && params->implicit_friction != 1) ||
        params->order != 1)
        return SME_EINVAL;
    for (int i = 0; i < n; ++i) {
        const sme_mesh &m = meshes[i];
        if (levels[i] < 0 || levels[i] > kBatchMaxLevel || m.kind != SME_MESH_2D_STRUCT) return SME_EINVAL;
        if (m.nx < 1 || m.ny < 1 || m.nx > (1 << 20) || m.ny > (1 << 20) || !(m.x1 > m.x0) || !(m.y1 > m.y0))
            return SME_EINVAL;
        for (int s = 0; s < 4; ++s)
            if (m.bc[s] < 0 || m.bc[s] > 2) return SME_EINVAL;
        if ((m.bc[0] == SME_BC_PERIODIC) != (m.bc[1] == SME_BC_PERIODIC) ||
            (m.bc[2] == SME_BC_PERIODIC) != (m.bc[3] == SME_BC_PERIODIC))
            return SME_EINVAL;
    }
    sme_batch *b = new (std::nothrow) sme_batch();
    if (!b) return SME_ENOMEM;
    b->n = n;
    b->p = *params;
    double qs[kMaxQuad] = {0}, qw[kMaxQuad] = {0};
    host::gauss_legendre01(params->quad_points, qs, qw);
    b->quad.n = params->quad_points;
    b->quad.s0 = qs[0];
    b->quad.s1 = qs[1];
    b->quad.s2 = qs[2];
    b->quad.w0 = qw[0];
    b->quad.w1 = qw[1];
    b->quad.w2 = qw[2];
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else if (hipStreamCreate(&b->stream) == hipSuccess) {
        b->own_stream = true;
    } else {
        delete b;
        return SME_EHIP;
    }
    int64_t off = 0, boff = 0;
    for (int i = 0; i < n; ++i) {
        const sme_mesh &m = meshes[i];
        b->level.push_back(levels[i]);
        b->nx.push_back((int)m.nx);
        b->ny.push_back((int)m.ny);
        b->nf.push_back(2 * levels[i] + 3);
        const int64_t nc = m.nx * m.ny;
        const int64_t st = (nc + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
        b->stride.push_back(st);
        b->offset.push_back(off);
        b->boff.push_back(boff);
        off += st * (2 * levels[i] + 3);
        boff += st;
        b->dx.push_back((m.x1 - m.x0) / m.nx);
        b->dy.push_back((m.y1 - m.y0) / m.ny);
        b->bc.push_back({m.bc[0], m.bc[1], m.bc[2], m.bc[3]});
        b->cells += nc;
    }
    int rc = SME_OK;
    auto alloc = [&](void **p, size_t bytes) {
        if (rc) return;
        hipError_t e = hipMalloc(p, bytes ? bytes : 8);
        if (e != hipSuccess) rc = bfail(b, e == hipErrorOutOfMemory ? SME_ENOMEM : SME_EHIP, "hipMalloc(%zu): %s",
                                        bytes, hipGetErrorString(e));
    };
    alloc((void **)&b->q[0], off * sizeof(double));
    alloc((void **)&b->q[1], off * sizeof(double));
    alloc((void **)&b->b, boff * sizeof(double));
    alloc((void **)&b->inst, n * sizeof(BatchInst));
    alloc((void **)&b->slots, 3 * (size_t)n * sizeof(Slot));
    alloc((void **)&b->work, 3 * kWorkStride * sizeof(unsigned));
    alloc((void **)&b->err, sizeof(ErrWord));
    alloc((void **)&b->quad_dev, 2 * kMaxQuad * sizeof(double));
    if (!rc) {
        double buf[2 * kMaxQuad];
        memcpy(buf, qs, sizeof qs);
        memcpy(buf + kMaxQuad, qw, sizeof qw);
        if (hipMemcpy(b->quad_dev, buf, sizeof buf, hipMemcpyHostToDevice) != hipSuccess)
            rc = bfail(b, SME_EHIP, "quadrature upload failed");
        b->quad.s = b->quad_dev;
        b->quad.w = b->quad_dev + kMaxQuad;
    }
    if (!rc) {
        hipError_t e = hipMemsetAsync(b->q[0], 0, off * sizeof(double), b->stream);
        if (e == hipSuccess) e = hipMemsetAsync(b->q[1], 0, off * sizeof(double), b->stream);
        if (e == hipSuccess) e = hipMemsetAsync(b->b, 0, boff * sizeof(double), b->stream);
        for (int i = 0; i < n && e == hipSuccess; ++i)
            if (bath && bath[i])
                e = hipMemcpyAsync(b->b + b->boff[i], bath[i], (size_t)b->nx[i] * b->ny[i] * sizeof(double),
                                   hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipMemsetAsync(b->slots, 0, 3 * (size_t)n * sizeof(Slot), b->stream);
        if (e == hipSuccess) e = hipMemsetAsync(b->work, 0, 3 * kWorkStride * sizeof(unsigned), b->stream);
        if (e == hipSuccess) e = launch_slots_reset(b->slots, b->err, 0, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) rc = bfail(b, SME_EHIP, "batch upload: %s", hipGetErrorString(e));
    }
    if (!rc) rc = build_items(b);
    if (rc) {
        sme_batch_destroy(b);
        return rc;
    }
    *out = b;
    return SME_OK;
}

int sme_batch_set_state(sme_batch *b, int i, const double *q, int on_device)
{
    if (!b || !q || i < 0 || i >= b->n) return SME_EINVAL;
    int r = load_state(b, i, q, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (r) return r;
    if (!on_device) BCHK(b, hipStreamSynchronize(b->stream));
    return SME_OK;
}

int sme_batch_get_state(sme_batch *b, int i, double *q, int on_device)
{
    if (!b || !q || i < 0 || i >= b->n) return SME_EINVAL;
    const size_t row = (size_t)b->nx[i] * b->ny[i] * sizeof(double);
    BCHK(b, hipMemcpy2DAsync(q, row, b->q[b->cur] + b->offset[i], b->stride[i] * sizeof(double), row, b->nf[i],
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream));
    if (!on_device) BCHK(b, hipStreamSynchronize(b->stream));
    return SME_OK;
}

int sme_batch_run(sme_batch *b, int64_t n_steps)
{
    if (!b || n_steps < 0) return SME_EINVAL;
    int64_t left = n_steps;
    const bool use_graphs = getenv("SME_NO_GRAPH") == nullptr;
    while (use_graphs && left >= kBatchGraphSteps) {
        hipGraphExec_t &ex = b->graph[b->cur][b->sa];
        if (!ex) {
            const int cur0 = b->cur, sa0 = b->sa;
            BCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            hipError_t le = hipSuccess;
            for (int k = 0; k < kBatchGraphSteps && le == hipSuccess; ++k) le = one_step(b);
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(b->stream, &g);
            b->cur = cur0;
            b->sa = sa0;
            if (le != hipSuccess || ee != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return bfail(b, SME_EHIP, "graph capture failed: %s", hipGetErrorString(le != hipSuccess ? le : ee));
            }
            hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) return bfail(b, SME_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
        }
        BCHK(b, hipGraphLaunch(ex, b->stream));
        left -= kBatchGraphSteps;
    }
    while (left-- > 0) BCHK(b, one_step(b));
    ErrWord e;
    BCHK(b, hipMemcpyAsync(&e, b->err, sizeof e, hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    if (e.flag)
        return bfail(b, SME_ENONPHYS, "non-physical state (h <= 0 or non-finite) in a grid of the batch, step %llu",
                     (unsigned long long)e.first_step);
    return SME_OK;
}

int sme_batch_time(sme_batch *b, int i, double *t, int64_t *steps)
{
    if (!b || i < 0 || i >= b->n) return SME_EINVAL;
    Slot s;
    BCHK(b, hipMemcpyAsync(&s, b->slots + 3 * i + b->sa, sizeof s, hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    if (t) *t = s.t;
    if (steps) *steps = s.step;
    return SME_OK;
}

int64_t sme_batch_cells(const sme_batch *b) { return b ? b->cells : SME_EINVAL; }

int sme_batch_rows(const sme_batch *b, int level)
{
    if (!b || level < 0 || level > kBatchMaxLevel) return SME_EINVAL;
    return b->rows[level];
}

int sme_batch_set_rows(sme_batch *b, int level, int rows)
{
    if (!b || level < 0 || level > kBatchMaxLevel || rows < 1 || rows > 1024) return SME_EINVAL;
    b->rows[level] = rows;
    return build_items(b);
}

int sme_batch_autotune(sme_batch *b, const char *cache_path)
{
    if (!b) return SME_EINVAL;
    // the mix of grids is part of the key: the best band height depends on it
    int count[kBatchMaxLevel + 1] = {0};
    for (int i = 0; i < b->n; ++i) count[b->level[i]]++;
    char dev_name[256] = "unknown";
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            snprintf(dev_name, sizeof dev_name, "%s", prop.gcnArchName);
        for (char *p = dev_name; *p; ++p)
            if (*p == ' ' || *p == ':') *p = '_';
    }
    std::ostringstream mix;
    mix << "n" << b->n << "_cells" << b->cells;
    for (int l = 0; l <= kBatchMaxLevel; ++l) mix << "_L" << l << "x" << count[l];
    const std::string key_base = std::string(dev_name) + " " + std::to_string(host::device_cus()) + " " + mix.str();
    // cached answers
    std::vector<std::string> cache_lines;
    bool have[kBatchMaxLevel + 1] = {false};
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            cache_lines.push_back(line);
            std::istringstream ls(line);
            std::string dn, cu, mx;
            int lvl, rws;
            if (ls >> dn >> cu >> mx >> lvl >> rws)
                if (dn + " " + cu + " " + mx == key_base && lvl >= 0 && lvl <= kBatchMaxLevel && rws > 0) {
                    b->rows[lvl] = rws;
                    have[lvl] = true;
                }
        }
    }
    // lake at rest everywhere: the timing does not depend on the values
    for (int i = 0; i < b->n; ++i) {
        std::vector<double> st((size_t)b->nf[i] * b->nx[i] * b->ny[i], 0.0);
        std::fill(st.begin(), st.begin() + (size_t)b->nx[i] * b->ny[i], 1.0);
        int r = load_state(b, i, st.data(), hipMemcpyHostToDevice);
        if (r) return r;
        BCHK(b, hipStreamSynchronize(b->stream));
    }
    int r = build_items(b);
    if (r) return r;
    // The GPU's clocks ramp up over the first tens of milliseconds of load:
    // time no candidate before about 0.2 s of steps (the lake at rest does not
    // change under them).
    {
        const auto t0 = std::chrono::steady_clock::now();
        do {
            BCHK(b, one_step(b));
            BCHK(b, hipStreamSynchronize(b->stream));
        } while (std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(200));
    }
    static const int cand[] = {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
    hipEvent_t e0, e1;
    BCHK(b, hipEventCreate(&e0));
    BCHK(b, hipEventCreate(&e1));
    bool tuned_any = false;
    for (int lvl = kBatchMaxLevel; lvl >= 0; --lvl) {
        if (!count[lvl] || have[lvl]) continue;
        float best = 1e30f;
        int best_rows = b->rows[lvl];
        for (int c : cand) {
            b->rows[lvl] = c;
            if ((r = build_items(b))) return r;
            BCHK(b, one_step(b));  // warm-up
            float t = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                BCHK(b, hipEventRecord(e0, b->stream));
                BCHK(b, one_step(b));
                BCHK(b, hipEventRecord(e1, b->stream));
                BCHK(b, hipEventSynchronize(e1));
                float ms = 0;
                BCHK(b, hipEventElapsedTime(&ms, e0, e1));
                t = std::min(t, ms);
            }
            if (t < best) {
                best = t;
                best_rows = c;
            }
        }
        b->rows[lvl] = best_rows;
        tuned_any = true;
        if (cache_path) cache_lines.push_back(key_base + " " + std::to_string(lvl) + " " + std::to_string(best_rows));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if ((r = build_items(b))) return r;
    // leave a clean batch: zero states, fresh clocks, no error
    for (int k = 0; k < 2; ++k) {
        size_t total = 0;
        for (int i = 0; i < b->n; ++i) total = std::max(total, (size_t)(b->offset[i] + b->stride[i] * b->nf[i]));
        BCHK(b, hipMemsetAsync(b->q[k], 0, total * sizeof(double), b->stream));
    }
    b->cur = 0;
    b->sa = 0;
    BCHK(b, hipMemsetAsync(b->slots, 0, 3 * (size_t)b->n * sizeof(Slot), b->stream));
    // every step finds its counter at zero: steps clear the counter of the step after next
    BCHK(b, hipMemsetAsync(b->work, 0, 3 * kWorkStride * sizeof(unsigned), b->stream));
    BCHK(b, launch_slots_reset(b->slots, b->err, 0, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    drop_graphs(b);
    if (cache_path && tuned_any) {
        std::ofstream o(cache_path);
        for (auto &l : cache_lines) o << l << "\n";
    }
    return SME_OK;
}

const char *sme_batch_last_error(const sme_batch *b) { return b ? b->last.c_str() : "no batch"; }

void sme_batch_destroy(sme_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    (void)hipFree(b->q[0]);
    (void)hipFree(b->q[1]);
    (void)hipFree(b->b);
    (void)hipFree(b->quad_dev);
    (void)hipFree(b->inst);
    (void)hipFree(b->items);
    (void)hipFree(b->slots);
    (void)hipFree(b->work);
    (void)hipFree(b->err);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"
