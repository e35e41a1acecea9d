// sme_closure.cpp -- host side of the learned closure (sme_mlp_*, sme_closure_*).
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
#include "sme_kernels.h"

using namespace sme;

// hooks into the single-grid context (sme_lib.cpp, hidden symbols)
extern "C" {
int sme_internal_attach(sme_ctx *c, const ClosureModel *m_host);
int sme_internal_oor(sme_ctx *c, int64_t *count);
hipStream_t sme_internal_stream(sme_ctx *c);
}

struct sme_mlp {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    ClosureModel host{};       // parameters are mirrored here only on demand
    float *p = nullptr;        // device parameters [kMlpParams]
    float *m = nullptr, *v = nullptr, *g = nullptr, *loss = nullptr;
    float *partial = nullptr, *partial_loss = nullptr;
    int partial_blocks = 0;
    double *stat_partial = nullptr, *stat_out = nullptr, *stat_mean = nullptr;  // feature statistics
    int64_t t = 0;             // Adam step count
    std::string last;
};

namespace {

int mfail(sme_mlp *m, int code, const char *fmt, ...)
{
    if (m) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        m->last = buf;
    }
    return code;
}

#define MCHK(mm, call)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return mfail((mm), SME_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

int ensure_partials(sme_mlp *m, int64_t batch)
{
    const int nblk = mlp_grad_blocks(batch);
    if (nblk <= m->partial_blocks) return SME_OK;
    (void)hipFree(m->partial);
    (void)hipFree(m->partial_loss);
    m->partial = nullptr;
    m->partial_loss = nullptr;
    m->partial_blocks = 0;
    MCHK(m, hipMalloc((void **)&m->partial, (size_t)nblk * kMlpParams * sizeof(float)));
    MCHK(m, hipMalloc((void **)&m->partial_loss, (size_t)nblk * sizeof(float)));
    m->partial_blocks = nblk;
    return SME_OK;
}

// Operands of the FP16 matrix-core inference (see ClosureFp16): kappa =
// 2 log2(e) folded into the first two layers, columns of the second and third
// layer in the lane order of the previous result; one rounding each.
// False if a folded weight does not fit FP16.
bool fold_fp16(ClosureModel &cm)
{
    const double kappa = 2.0 / std::log(2.0);
    const float *P = cm.params;
    ClosureFp16 &H = cm.h;
    std::memset(&H, 0, sizeof H);
    double wmax = 0.0;
    auto put = [&wmax](_Float16 &dst, double v) {
        wmax = std::fmax(wmax, std::fabs(v));
        dst = (_Float16)(float)v;
    };
    for (int j = 0; j < kMlpHid; ++j) {
        for (int i = 0; i < kMlpIn; ++i) put(H.w1[j][i], kappa * P[kOffW1 + j * kMlpIn + i]);
        H.c1[j] = (float)(kappa * P[kOffB1 + j]);
        for (int p = 0; p < kMlpHid; ++p) put(H.w2[j][p], kappa * P[kOffW2 + j * kMlpHid + kFoldPerm(p)]);
        H.c2[j] = (float)(kappa * P[kOffB2 + j]);
    }
    for (int o = 0; o < kMlpOut; ++o) {
        for (int p = 0; p < kMlpHid; ++p) put(H.w3[o][p], P[kOffW3 + o * kMlpHid + kFoldPerm(p)]);
        H.c3[o] = P[kOffB3 + o];
    }
    return wmax <= 65504.0;
}

// splitmix64: a counter-based 64-bit generator (Steele, Lea and Flood, 2014)
struct SplitMix64 {
    uint64_t x;
    uint64_t next()
    {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }  // [0, 1)
    uint64_t below(uint64_t k) { return (uint64_t)(((unsigned __int128)next() * k) >> 64); }  // [0, k)
};

MlpScale scale_of(const sme_mlp *m)
{
    MlpScale sc{};
    for (int i = 0; i < kMlpIn; ++i) {
        sc.mu[i] = m->host.mu[i];
        sc.inv_sigma[i] = m->host.inv_sigma[i];
    }
    for (int o = 0; o < kMlpOut; ++o) sc.out_scale[o] = m->host.out_scale[o];
    return sc;
}

}  // namespace

extern "C" {

int sme_mlp_create(sme_mlp **out, void *stream)
{
    if (!out) return SME_EINVAL;
    *out = nullptr;
    sme_mlp *m = new (std::nothrow) sme_mlp();
    if (!m) return SME_ENOMEM;
    if (stream) {
        m->stream = (hipStream_t)stream;
    } else if (hipStreamCreate(&m->stream) == hipSuccess) {
        m->own_stream = true;
    } else {
        delete m;
        return SME_EHIP;
    }
    for (int i = 0; i < kMlpIn; ++i) {
        m->host.mu[i] = 0.0f;
        m->host.inv_sigma[i] = 1.0f;
        m->host.box_lo[i] = -INFINITY;
        m->host.box_hi[i] = INFINITY;
    }
    for (int o = 0; o < kMlpOut; ++o) m->host.out_scale[o] = 1.0f;
    hipError_t e = hipMalloc((void **)&m->p, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&m->m, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&m->v, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&m->g, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&m->loss, sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->p, 0, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->m, 0, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->v, 0, kMlpParams * sizeof(float));
    if (e != hipSuccess) {
        sme_mlp_destroy(m);
        return e == hipErrorOutOfMemory ? SME_ENOMEM : SME_EHIP;
    }
    *out = m;
    return SME_OK;
}

int sme_mlp_set_params(sme_mlp *m, const float *params, int on_device)
{
    if (!m || !params) return SME_EINVAL;
    MCHK(m, hipMemcpyAsync(m->p, params, kMlpParams * sizeof(float),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, m->stream));
    if (!on_device) MCHK(m, hipStreamSynchronize(m->stream));
    return SME_OK;
}

int sme_mlp_get_params(sme_mlp *m, float *params, int on_device)
{
    if (!m || !params) return SME_EINVAL;
    MCHK(m, hipMemcpyAsync(params, m->p, kMlpParams * sizeof(float),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, m->stream));
    if (!on_device) MCHK(m, hipStreamSynchronize(m->stream));
    return SME_OK;
}

int sme_mlp_set_scaling(sme_mlp *m, const float *mu, const float *sigma, const float *out_scale,
                        const double *box_lo, const double *box_hi)
{
    if (!m) return SME_EINVAL;
    for (int i = 0; i < kMlpIn; ++i) {
        if (sigma && !(sigma[i] > 0.0f)) return mfail(m, SME_EINVAL, "sigma must be positive");
        if (mu) m->host.mu[i] = mu[i];
        if (sigma) m->host.inv_sigma[i] = 1.0f / sigma[i];
        if (box_lo) m->host.box_lo[i] = box_lo[i];
        if (box_hi) m->host.box_hi[i] = box_hi[i];
    }
    if (out_scale)
        for (int o = 0; o < kMlpOut; ++o) m->host.out_scale[o] = out_scale[o];
    return SME_OK;
}

int sme_mlp_get_scaling(const sme_mlp *m, float *mu, float *sigma, float *out_scale, double *box_lo,
                        double *box_hi)
{
    if (!m) return SME_EINVAL;
    for (int i = 0; i < kMlpIn; ++i) {
        if (mu) mu[i] = m->host.mu[i];
        if (sigma) sigma[i] = 1.0f / m->host.inv_sigma[i];
        if (box_lo) box_lo[i] = m->host.box_lo[i];
        if (box_hi) box_hi[i] = m->host.box_hi[i];
    }
    if (out_scale)
        for (int o = 0; o < kMlpOut; ++o) out_scale[o] = m->host.out_scale[o];
    return SME_OK;
}

int sme_mlp_fit_scaling(sme_mlp *m, const float *feat, const float *targ, int64_t n, double margin)
{
    if (!m || !feat || !targ || n < 2 || !(margin >= 0.0)) return SME_EINVAL;
    const int w = mlp_stat_width();
    if (!m->stat_partial) {
        MCHK(m, hipMalloc((void **)&m->stat_partial, (size_t)mlp_stat_blocks() * w * sizeof(double)));
        MCHK(m, hipMalloc((void **)&m->stat_out, w * sizeof(double)));
        MCHK(m, hipMalloc((void **)&m->stat_mean, w * sizeof(double)));
    }
    std::vector<double> first(w), second(w), mean(w, 0.0);
    // pass 1: sums, minima, maxima; pass 2: squared deviations from the mean
    MCHK(m, launch_mlp_stats(feat, targ, n, nullptr, m->stat_partial, m->stat_out, m->stream));
    MCHK(m, hipMemcpyAsync(first.data(), m->stat_out, w * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    MCHK(m, hipStreamSynchronize(m->stream));
    constexpr int cols = kMlpIn + kMlpOut;
    for (int c = 0; c < cols; ++c) mean[c] = first[c] / (double)n;
    MCHK(m, hipMemcpyAsync(m->stat_mean, mean.data(), w * sizeof(double), hipMemcpyHostToDevice, m->stream));
    MCHK(m, launch_mlp_stats(feat, targ, n, m->stat_mean, m->stat_partial, m->stat_out, m->stream));
    MCHK(m, hipMemcpyAsync(second.data(), m->stat_out, w * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    MCHK(m, hipStreamSynchronize(m->stream));
    for (int c = 0; c < cols; ++c) {
        const double sd = std::sqrt(second[c] / (double)(n - 1));  // sample standard deviation
        if (c < kMlpIn) {
            const float sigma = std::max((float)sd, 1e-6f);
            const double lo = first[cols + c], hi = first[cols + kMlpIn + c], span = hi - lo;
            m->host.mu[c] = (float)mean[c];
            m->host.inv_sigma[c] = 1.0f / sigma;
            m->host.box_lo[c] = lo - margin * span;
            m->host.box_hi[c] = hi + margin * span;
        } else {
            m->host.out_scale[c - kMlpIn] = std::max((float)sd, 1e-12f);
        }
    }
    return SME_OK;
}

int sme_mlp_forward(sme_mlp *m, const float *x, int64_t batch, float *y)
{
    if (!m || !x || !y || batch < 0) return SME_EINVAL;
    MCHK(m, launch_mlp_forward(m->p, x, batch, scale_of(m), y, m->stream));
    return SME_OK;
}

int sme_mlp_loss_grad(sme_mlp *m, const float *x, const float *t, const int64_t *idx, int64_t batch, float *loss,
                      float *grad)
{
    if (!m || !x || !t || batch < 1) return SME_EINVAL;
    int r = ensure_partials(m, batch);
    if (r) return r;
    MCHK(m, launch_mlp_grad(m->p, x, t, idx, batch, scale_of(m), m->partial, m->partial_loss, m->g, m->loss,
                            m->stream));
    if (grad) MCHK(m, hipMemcpyAsync(grad, m->g, kMlpParams * sizeof(float), hipMemcpyDeviceToDevice, m->stream));
    if (loss) {
        MCHK(m, hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MCHK(m, hipStreamSynchronize(m->stream));
    }
    return SME_OK;
}

int sme_mlp_train_step(sme_mlp *m, const float *x, const float *t, const int64_t *idx, int64_t batch, float lr,
                       float *loss)
{
    if (!m || !x || !t || batch < 1 || !(lr > 0)) return SME_EINVAL;
    int r = ensure_partials(m, batch);
    if (r) return r;
    MCHK(m, launch_mlp_grad(m->p, x, t, idx, batch, scale_of(m), m->partial, m->partial_loss, m->g, m->loss,
                            m->stream));
    m->t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)m->t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)m->t)));
    MCHK(m, launch_mlp_adam(m->p, m->g, m->m, m->v, lr, (float)b1, (float)b2, 1e-8f, c1, c2, m->stream));
    if (loss) {
        MCHK(m, hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
        MCHK(m, hipStreamSynchronize(m->stream));
    }
    return SME_OK;
}

int sme_mlp_reset_optimizer(sme_mlp *m)
{
    if (!m) return SME_EINVAL;
    m->t = 0;
    MCHK(m, hipMemsetAsync(m->m, 0, kMlpParams * sizeof(float), m->stream));
    MCHK(m, hipMemsetAsync(m->v, 0, kMlpParams * sizeof(float), m->stream));
    return SME_OK;
}

const char *sme_mlp_last_error(const sme_mlp *m) { return m ? m->last.c_str() : "no network"; }

void sme_mlp_destroy(sme_mlp *m)
{
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    (void)hipFree(m->p);
    (void)hipFree(m->m);
    (void)hipFree(m->v);
    (void)hipFree(m->g);
    (void)hipFree(m->loss);
    (void)hipFree(m->partial);
    (void)hipFree(m->partial_loss);
    (void)hipFree(m->stat_partial);
    (void)hipFree(m->stat_out);
    (void)hipFree(m->stat_mean);
    if (m->own_stream) (void)hipStreamDestroy(m->stream);
    delete m;
}

int sme_closure_samples(const double *q8, int64_t stride8, const double *q8_next, int64_t stride8n,
                        const double *q1_step, int64_t stride1, int64_t ncells, double dt, const int64_t *cells,
                        int64_t nsamples, float *feat, float *targ, void *stream)
{
    if (!q8 || !q8_next || !q1_step || !cells || !feat || !targ || ncells < 3 || nsamples < 0 || !(dt > 0))
        return SME_EINVAL;
    if (stride8 < ncells || stride8n < ncells || stride1 < ncells) return SME_EINVAL;
    hipError_t e = launch_closure_samples(q8, stride8, q8_next, stride8n, q1_step, stride1, ncells, dt, cells, nsamples,
                                          feat, targ, (hipStream_t)stream);
    return e == hipSuccess ? SME_OK : SME_EHIP;
}

int sme_mlp_init(sme_mlp *m, uint64_t seed)
{
    if (!m) return SME_EINVAL;
    std::vector<float> p(kMlpParams, 0.0f);
    SplitMix64 g{seed};
    // Glorot-uniform weights U(-a, a), a = sqrt(6 / (fan_in + fan_out)); zero biases
    auto fill = [&](int off, int fan_out, int fan_in) {
        const double a = std::sqrt(6.0 / (fan_in + fan_out));
        for (int k = 0; k < fan_out * fan_in; ++k) p[off + k] = (float)((2.0 * g.uniform() - 1.0) * a);
    };
    fill(kOffW1, kMlpHid, kMlpIn);
    fill(kOffW2, kMlpHid, kMlpHid);
    fill(kOffW3, kMlpOut, kMlpHid);
    int r = sme_mlp_set_params(m, p.data(), 0);
    return r ? r : sme_mlp_reset_optimizer(m);
}

int sme_closure_train(sme_mlp *m, const float *feat, const float *targ, int64_t n, int epochs, int64_t batch,
                      float lr, float lr_end, uint64_t seed, double margin, float *loss_hist)
{
    if (!m || !feat || !targ || n < 2 || epochs < 1 || batch < 1 || !(lr > 0) || !(lr_end > 0)) return SME_EINVAL;
    int r = sme_mlp_fit_scaling(m, feat, targ, n, margin);
    if (!r) r = sme_mlp_reset_optimizer(m);
    if (r) return r;
    const int64_t bs = std::min(batch, n);
    const int64_t nb = std::max<int64_t>(1, n / bs);
    const int64_t total = (int64_t)epochs * nb;
    std::vector<int64_t> perm(n);
    int64_t *dperm = nullptr;
    MCHK(m, hipMalloc((void **)&dperm, (size_t)n * sizeof(int64_t)));
    SplitMix64 g{seed};
    int64_t step = 0;
    for (int ep = 0; ep < epochs && !r; ++ep) {
        for (int64_t i = 0; i < n; ++i) perm[i] = i;
        for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[(int64_t)g.below((uint64_t)i + 1)]);
        hipError_t e = hipMemcpyAsync(dperm, perm.data(), (size_t)n * sizeof(int64_t), hipMemcpyHostToDevice, m->stream);
        if (e != hipSuccess) {
            r = mfail(m, SME_EHIP, "permutation upload: %s", hipGetErrorString(e));
            break;
        }
        float loss = 0.0f;
        for (int64_t b = 0; b < nb && !r; ++b, ++step) {
            const double frac = (double)step / (double)std::max<int64_t>(1, total - 1);
            const float rate = (float)(lr * std::pow((double)lr_end / lr, frac));
            r = sme_mlp_train_step(m, feat, targ, dperm + b * bs, bs, rate, b == nb - 1 ? &loss : nullptr);
        }
        if (!r && loss_hist) loss_hist[ep] = loss;
    }
    // the host permutation must not change while a copy may still read it
    (void)hipStreamSynchronize(m->stream);
    (void)hipFree(dperm);
    return r;
}

int sme_closure_attach_ex(sme_ctx *ctx, const sme_mlp *m, int precision)
{
    if (!ctx) return SME_EINVAL;
    if (!m) return sme_internal_attach(ctx, nullptr);
    if (precision != SME_CLOSURE_FP32 && precision != SME_CLOSURE_FP16_MFMA) return SME_EINVAL;
    ClosureModel *cm = new (std::nothrow) ClosureModel(m->host);
    if (!cm) return SME_ENOMEM;
    // the parameters come from the device copy
    sme_mlp *mm = const_cast<sme_mlp *>(m);
    mm->last.clear();
    hipError_t e = hipMemcpyAsync(cm->params, m->p, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    int rc = e == hipSuccess ? SME_OK : mfail(mm, SME_EHIP, "parameter copy failed: %s", hipGetErrorString(e));
    cm->precision = precision == SME_CLOSURE_FP16_MFMA ? kClosureFp16Mfma : kClosureFp32;
    if (rc == SME_OK && precision == SME_CLOSURE_FP16_MFMA && !fold_fp16(*cm))
        rc = mfail(mm, SME_EINVAL, "folded weights exceed the FP16 range");
    if (rc == SME_OK) rc = sme_internal_attach(ctx, cm);
    delete cm;
    return rc;
}

int sme_closure_attach(sme_ctx *ctx, const sme_mlp *m) { return sme_closure_attach_ex(ctx, m, SME_CLOSURE_FP32); }

int sme_closure_out_of_range(sme_ctx *ctx, int64_t *cells)
{
    if (!ctx || !cells) return SME_EINVAL;
    return sme_internal_oor(ctx, cells);
}

}  // extern "C"
