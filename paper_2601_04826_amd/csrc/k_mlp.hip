// k_mlp.hip -- FP32 training kernels of the closure network, and the kernel
// that turns level-8 snapshots into training samples.
//
// Every kernel reads raw features and targets and normalises them with the
// network's scaling, x~ = (x - mu) * (1/sigma) and t~ = t / s_out (the same
// FP32 arithmetic as inference); training kernels take their batch rows
// through an index list (NULL: rows 0..B-1).
//
// Training step for a batch of B samples (normalised inputs x~, targets t~):
//   k_mlp_grad     one 64-lane wave per 64 samples: forward, reverse-mode
//                  backward, and that block's partial sums of every parameter
//                  gradient of L = (1/B) sum_b |y~_b - t~_b|^2 (activations in
//                  LDS, the per-parameter sums over the block's samples read
//                  them back); partial loss too
//   k_mlp_reduce   sums the block partials per parameter in a fixed order
//                  (deterministic), FP64 accumulation
//   k_mlp_adam     Adam update with bias correction (Kingma & Ba)
// Feature statistics (for the scaling and the training box):
//   k_mlp_stats    per block, FP64 column sums (or sums of squared deviations
//                  from a given mean) of 9 features and 2 targets, and the
//                  feature minima and maxima
//   k_mlp_stats_reduce  fixed-order sum over the blocks (deterministic)
#include <hip/hip_runtime.h>

#include "sme_kernels.h"
#include "sme_mlp.h"

namespace sme {

namespace {

constexpr int kGradBlock = 64;  // samples (= lanes) per gradient block
constexpr int kLdsPad = kMlpHid + 1;

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ params, const float *__restrict__ x,
                                                     int64_t B, MlpScale sc, float *__restrict__ y)
{
    __shared__ float P[kMlpParams];
    mlp_stage(params, P);
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float xi[kMlpIn], a1[kMlpHid], a2[kMlpHid], yo[kMlpOut];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) xi[i] = (x[b * kMlpIn + i] - sc.mu[i]) * sc.inv_sigma[i];
    mlp_forward(P, xi, a1, a2, yo);
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) y[b * kMlpOut + o] = yo[o];
}

__global__ __launch_bounds__(kGradBlock) void k_mlp_grad(const float *__restrict__ params, const float *__restrict__ x,
                                                         const float *__restrict__ t, const int64_t *__restrict__ idx,
                                                         int64_t B, float inv_b, MlpScale sc,
                                                         float *__restrict__ partial, float *__restrict__ partial_loss)
{
    __shared__ float P[kMlpParams];
    __shared__ float A1[kGradBlock][kLdsPad];
    __shared__ float A2[kGradBlock][kLdsPad];
    __shared__ float DZ1[kGradBlock][kLdsPad];
    __shared__ float DZ2[kGradBlock][kLdsPad];
    __shared__ float X[kGradBlock][kMlpIn + 1];
    __shared__ float DY[kGradBlock][kMlpOut];
    mlp_stage(params, P);
    const int tid = threadIdx.x;
    const int64_t b = (int64_t)blockIdx.x * kGradBlock + tid;
    const bool live = b < B;
    const int64_t row = live ? (idx ? idx[b] : b) : 0;
    float xi[kMlpIn], a1[kMlpHid], a2[kMlpHid], y[kMlpOut];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) xi[i] = live ? (x[row * kMlpIn + i] - sc.mu[i]) * sc.inv_sigma[i] : 0.0f;
    mlp_forward(P, xi, a1, a2, y);
    // backward of one sample; samples beyond B contribute nothing
    float dy[kMlpOut];
    float loss = 0.0f;
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) {
        const float r = live ? y[o] - t[row * kMlpOut + o] / sc.out_scale[o] : 0.0f;
        loss = fmaf(r, r, loss);
        dy[o] = 2.0f * r * inv_b;
    }
    float dz2[kMlpHid];
#pragma unroll
    for (int j = 0; j < kMlpHid; ++j) {
        float d = P[kOffW3 + j] * dy[0];
        d = fmaf(P[kOffW3 + kMlpHid + j], dy[1], d);
        dz2[j] = d * (1.0f - a2[j] * a2[j]);
    }
#pragma unroll
    for (int i = 0; i < kMlpHid; ++i) {
        float d = 0.0f;
#pragma unroll
        for (int j = 0; j < kMlpHid; ++j) d = fmaf(P[kOffW2 + j * kMlpHid + i], dz2[j], d);
        DZ1[tid][i] = d * (1.0f - a1[i] * a1[i]);
        A1[tid][i] = a1[i];
        A2[tid][i] = a2[i];
        DZ2[tid][i] = dz2[i];
    }
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) X[tid][i] = xi[i];
    DY[tid][0] = dy[0];
    DY[tid][1] = dy[1];
    __syncthreads();
    // parameter gradients: lane j sums row j of every weight matrix over the block's samples
    const int j = tid;
    float* out = partial + (int64_t)blockIdx.x * kMlpParams;
    {
        float gw2[kMlpHid];
#pragma unroll
        for (int i = 0; i < kMlpHid; ++i) gw2[i] = 0.0f;
        float gb2 = 0.0f, gb1 = 0.0f;
        float gw1[kMlpIn];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) gw1[i] = 0.0f;
        float gw30 = 0.0f, gw31 = 0.0f;
        for (int s = 0; s < kGradBlock; ++s) {
            const float d2 = DZ2[s][j];
            const float d1 = DZ1[s][j];
#pragma unroll
            for (int i = 0; i < kMlpHid; ++i) gw2[i] = fmaf(d2, A1[s][i], gw2[i]);
#pragma unroll
            for (int i = 0; i < kMlpIn; ++i) gw1[i] = fmaf(d1, X[s][i], gw1[i]);
            gb2 += d2;
            gb1 += d1;
            gw30 = fmaf(DY[s][0], A2[s][j], gw30);
            gw31 = fmaf(DY[s][1], A2[s][j], gw31);
        }
#pragma unroll
        for (int i = 0; i < kMlpHid; ++i) out[kOffW2 + j * kMlpHid + i] = gw2[i];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) out[kOffW1 + j * kMlpIn + i] = gw1[i];
        out[kOffB2 + j] = gb2;
        out[kOffB1 + j] = gb1;
        out[kOffW3 + j] = gw30;
        out[kOffW3 + kMlpHid + j] = gw31;
    }
    if (j < kMlpOut) {
        float g = 0.0f;
        for (int s = 0; s < kGradBlock; ++s) g += DY[s][j];
        out[kOffB3 + j] = g;
    }
    // block loss (one wave): lane sum
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
    if (tid == 0) partial_loss[blockIdx.x] = loss;
}

// grad[k] = sum over blocks of partial[block][k] (fixed order), loss likewise
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ partial,
                                                    const float *__restrict__ partial_loss, int nblk, float inv_b,
                                                    float *__restrict__ grad, float *__restrict__ loss)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kMlpParams) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += (double)partial[(int64_t)b * kMlpParams + k];
        grad[k] = (float)s;
    }
    if (k == 0) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += (double)partial_loss[b];
        *loss = (float)(s * (double)inv_b);
    }
}

__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ p, const float *__restrict__ g,
                                                  float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                                                  float b2, float eps, float c1, float c2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kMlpParams) return;
    const float gk = g[k];
    const float mk = fmaf(b1, m[k], (1.0f - b1) * gk);
    const float vk = fmaf(b2, v[k], (1.0f - b2) * gk * gk);
    m[k] = mk;
    v[k] = vk;
    // c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
    p[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
}

constexpr int kStatCols = kMlpIn + kMlpOut;  // 9 features, 2 targets
constexpr int kStatBlocks = 256;
constexpr int kStatWidth = kStatCols + 2 * kMlpIn;  // sums, feature minima, feature maxima

// value of column c of row r (features first, then targets)
__device__ __forceinline__ double stat_col(const float *feat, const float *targ, int64_t r, int c)
{
    return c < kMlpIn ? (double)feat[r * kMlpIn + c] : (double)targ[r * kMlpOut + c - kMlpIn];
}

// mean == nullptr: column sums, minima and maxima; else sums of squared
// deviations from mean.  One row per thread and stride; tree sums in LDS.
__global__ __launch_bounds__(256) void k_mlp_stats(const float *__restrict__ feat, const float *__restrict__ targ,
                                                   int64_t n, const double *__restrict__ mean,
                                                   double *__restrict__ partial)
{
    __shared__ double S[256][kStatWidth + 1];
    double acc[kStatWidth];
#pragma unroll
    for (int c = 0; c < kStatCols; ++c) acc[c] = 0.0;
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) {
        acc[kStatCols + c] = INFINITY;
        acc[kStatCols + kMlpIn + c] = -INFINITY;
    }
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < kStatCols; ++c) {
            const double v = stat_col(feat, targ, r, c);
            if (mean) {
                const double d = v - mean[c];
                acc[c] = fma(d, d, acc[c]);
            } else {
                acc[c] += v;
                if (c < kMlpIn) {
                    acc[kStatCols + c] = fmin(acc[kStatCols + c], v);
                    acc[kStatCols + kMlpIn + c] = fmax(acc[kStatCols + kMlpIn + c], v);
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kStatWidth; ++c) S[threadIdx.x][c] = acc[c];
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) {
            for (int c = 0; c < kStatWidth; ++c) {
                const double o = S[threadIdx.x + half][c];
                double &v = S[threadIdx.x][c];
                v = c < kStatCols ? v + o : (c < kStatCols + kMlpIn ? fmin(v, o) : fmax(v, o));
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < kStatWidth) partial[(int64_t)blockIdx.x * kStatWidth + threadIdx.x] = S[0][threadIdx.x];
}

__global__ void k_mlp_stats_reduce(const double *__restrict__ partial, int nblk, double *__restrict__ out)
{
    const int c = threadIdx.x;
    if (c >= kStatWidth) return;
    double v = partial[c];
    for (int b = 1; b < nblk; ++b) {
        const double o = partial[(int64_t)b * kStatWidth + c];
        v = c < kStatCols ? v + o : (c < kStatCols + kMlpIn ? fmin(v, o) : fmax(v, o));
    }
    out[c] = v;
}

// Training samples from two consecutive level-8 states and the level-1 step of
// the first (all on a periodic 1D row, SoA with the given strides).  Sample s
// is cell cells[s]: raw features (FP64 differences, stored FP32) and target
// (q_k of P(Q8^{n+1}) - q_k of Step_L1(P(Q8^n))) / dt for k = 0, 1.
__global__ __launch_bounds__(256) void k_closure_samples(const double *__restrict__ q8, int64_t s8,
                                                         const double *__restrict__ q8n, int64_t s8n,
                                                         const double *__restrict__ q1, int64_t s1, int64_t n,
                                                         double dt, const int64_t *__restrict__ cells, int64_t ns,
                                                         float *__restrict__ feat, float *__restrict__ targ)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const int64_t i = cells[s];
    const int64_t ip = i + 1 == n ? 0 : i + 1;
    const int64_t im = i == 0 ? n - 1 : i - 1;
    const double h = q8[i], a = q8[s8 + i], c = q8[2 * s8 + i];
    const double hp = q8[ip], ap = q8[s8 + ip], cp = q8[2 * s8 + ip];
    const double hm = q8[im], am = q8[s8 + im], cm = q8[2 * s8 + im];
    float *f = feat + s * kMlpIn;
    f[0] = (float)h;
    f[1] = (float)a;
    f[2] = (float)c;
    f[3] = (float)(hp - h);
    f[4] = (float)(ap - a);
    f[5] = (float)(cp - c);
    f[6] = (float)(h - hm);
    f[7] = (float)(a - am);
    f[8] = (float)(c - cm);
    targ[s * kMlpOut + 0] = (float)((q8n[s8n + i] - q1[s1 + i]) / dt);
    targ[s * kMlpOut + 1] = (float)((q8n[2 * s8n + i] - q1[2 * s1 + i]) / dt);
}

}  // namespace

hipError_t launch_mlp_forward(const float *params, const float *x, int64_t B, const MlpScale &sc, float *y,
                              hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, params, x, B, sc, y);
    return hipGetLastError();
}

int mlp_stat_width() { return kStatWidth; }
int mlp_stat_blocks() { return kStatBlocks; }

hipError_t launch_mlp_stats(const float *feat, const float *targ, int64_t n, const double *mean, double *partial,
                            double *out, hipStream_t s)
{
    if (n <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_stats, dim3(kStatBlocks), dim3(256), 0, s, feat, targ, n, mean, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_stats_reduce, dim3(1), dim3(64), 0, s, partial, kStatBlocks, out);
    return hipGetLastError();
}

int mlp_grad_blocks(int64_t B) { return (int)((B + kGradBlock - 1) / kGradBlock); }

hipError_t launch_mlp_grad(const float *params, const float *x, const float *t, const int64_t *idx, int64_t B,
                           const MlpScale &sc, float *partial, float *partial_loss, float *grad, float *loss,
                           hipStream_t s)
{
    if (B <= 0) return hipErrorInvalidValue;
    const int nblk = mlp_grad_blocks(B);
    const float inv_b = 1.0f / (float)B;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(kGradBlock), 0, s, params, x, t, idx, B, inv_b, sc, partial,
                       partial_loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, partial, partial_loss, nblk,
                       inv_b, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                           float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, p, g, m, v, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

hipError_t launch_closure_samples(const double *q8, int64_t s8, const double *q8n, int64_t s8n, const double *q1,
                                  int64_t s1, int64_t n, double dt, const int64_t *cells, int64_t ns, float *feat,
                                  float *targ, hipStream_t s)
{
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_closure_samples, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, q8, s8, q8n, s8n, q1,
                       s1, n, dt, cells, ns, feat, targ);
    return hipGetLastError();
}

}  // namespace sme
