// sme_mlp.h -- the closure network (9 -> 64 -> 64 -> 2, tanh, FP32), device side.
//
// The learned closure maps per-cell features of a level-1 state to correction
// rates of its momentum moments (q_0, q_1), so that level 1 stands in for
// level 8.  Parameters are one flat FP32 array:
//   W1[64][9], b1[64], W2[64][64], b2[64], W3[2][64], b3[2]   (4,930 floats)
// The network works on normalised inputs x~ = (x - mu) / sigma and outputs
// normalised rates y~; the rate is y = y~ * s_out.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace sme {

constexpr int kMlpIn = 9, kMlpHid = 64, kMlpOut = 2;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHid * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpOut * kMlpHid;
constexpr int kMlpParams = kOffB3 + kMlpOut;  // 4930

// Reduced-precision inference: FP16 matrix-core operands, FP32 accumulation.
// With kappa = 2 log2(e), a layer computes u = kappa (W a + b) on the matrix
// cores (kappa folded into the FP16 weights and FP32 biases on the host) and
// tanh(u / kappa) = 1 - 2 / (1 + 2^u) in FP32 (one exp2, one add, one
// reciprocal, one FMA), rounded once to FP16 as the next layer's operand.
// The columns of w2 and w3 are stored in the order in which the matrix-core
// result of the previous layer lands in the lanes (kFoldPerm), so activations
// feed the next product without any data movement.
constexpr int kMlpInPad = 16;
struct alignas(16) ClosureFp16 {
    _Float16 w1[kMlpHid][kMlpInPad];  // kappa W1, inputs 9..15 zero
    _Float16 w2[kMlpHid][kMlpHid];    // kappa W2, permuted columns
    _Float16 w3[16][kMlpHid];         // W3, permuted columns, rows 2..15 zero
    float c1[kMlpHid];                // kappa b1
    float c2[kMlpHid];                // kappa b2
    float c3[4];                      // b3, rows 2, 3 zero
};

// Column p = 32 kc + 8 g + e of a folded matrix holds hidden unit kFoldPerm(p):
// the 16x16 result tiles 2 kc and 2 kc + 1 give lane group g the units
// 16 (2 kc) + 4 g + {0..3} and 16 (2 kc + 1) + 4 g + {0..3}.
constexpr int kFoldPerm(int p)
{
    return 32 * (p / 32) + ((p % 8) < 4 ? 4 * ((p % 32) / 8) + (p % 8) : 16 + 4 * ((p % 32) / 8) + (p % 8) - 4);
}

enum ClosurePrecision { kClosureFp32 = 0, kClosureFp16Mfma = 1 };

// Normalisation of the network's inputs and targets, passed to the training
// and forward kernels by value.
struct MlpScale {
    float mu[kMlpIn];
    float inv_sigma[kMlpIn];
    float out_scale[kMlpOut];
};

// Everything the closure rates pass needs.
struct ClosureModel {
    float params[kMlpParams];
    float mu[kMlpIn];
    float inv_sigma[kMlpIn];
    float out_scale[kMlpOut];
    double box_lo[kMlpIn];  // training range of the raw features (fallback test)
    double box_hi[kMlpIn];
    int precision;          // ClosurePrecision
    ClosureFp16 h;          // folded operands of the FP16 variant
};

// tanh(z) = sign(z) (1 - e) / (1 + e), e = exp(-2|z|) in (0, 1]: no overflow,
// absolute error about 1e-7.  Training and inference use this same function.
__device__ __forceinline__ float tanh_f(float z)
{
    const float e = __expf(-2.0f * fabsf(z));
    return copysignf(__fdividef(1.0f - e, 1.0f + e), z);
}

// copy the parameters of a model into LDS (all threads of the block call it)
__device__ __forceinline__ void mlp_stage(const float *__restrict__ g, float *s)
{
    for (int k = threadIdx.x; k < kMlpParams; k += blockDim.x) s[k] = g[k];
    __syncthreads();
}

// forward pass of one sample; P = parameters (LDS), x = normalised inputs
__device__ __forceinline__ void mlp_forward(const float *P, const float *x, float *a1, float *a2, float *y)
{
#pragma unroll
    for (int j = 0; j < kMlpHid; ++j) {
        float z = P[kOffB1 + j];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) z = fmaf(P[kOffW1 + j * kMlpIn + i], x[i], z);
        a1[j] = tanh_f(z);
    }
#pragma unroll
    for (int j = 0; j < kMlpHid; ++j) {
        float z = P[kOffB2 + j];
#pragma unroll
        for (int i = 0; i < kMlpHid; ++i) z = fmaf(P[kOffW2 + j * kMlpHid + i], a1[i], z);
        a2[j] = tanh_f(z);
    }
#pragma unroll
    for (int o = 0; o < kMlpOut; ++o) {
        float z = P[kOffB3 + o];
#pragma unroll
        for (int i = 0; i < kMlpHid; ++i) z = fmaf(P[kOffW3 + o * kMlpHid + i], a2[i], z);
        y[o] = z;
    }
}

}  // namespace sme

namespace sme {

// Inference of one sample: y~ for normalised inputs x; layer 2 and 3 are
// fused so that only the first hidden layer is held in registers.
__device__ __forceinline__ void mlp_infer(const float *P, const float *x, float *y)
{
    float a1[kMlpHid];
#pragma unroll
    for (int j = 0; j < kMlpHid; ++j) {
        float z = P[kOffB1 + j];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) z = fmaf(P[kOffW1 + j * kMlpIn + i], x[i], z);
        a1[j] = tanh_f(z);
    }
    float y0 = P[kOffB3], y1 = P[kOffB3 + 1];
    for (int j = 0; j < kMlpHid; ++j) {
        float z = P[kOffB2 + j];
#pragma unroll
        for (int i = 0; i < kMlpHid; ++i) z = fmaf(P[kOffW2 + j * kMlpHid + i], a1[i], z);
        const float a2 = tanh_f(z);
        y0 = fmaf(P[kOffW3 + j], a2, y0);
        y1 = fmaf(P[kOffW3 + kMlpHid + j], a2, y1);
    }
    y[0] = y0;
    y[1] = y1;
}

// Closure correction rates of the two normal momentum moments of one cell
// along one direction.  Features: the cell's (h, q_0, q_1), its differences to
// the neighbour ahead (p) and behind (m) along the direction.  P = parameters
// in LDS, M = the model (normalisation, output scale, training box).
// Returns false (and zero rates) if a feature lies outside the training box.
__device__ __forceinline__ bool closure_rate(const float *P, const ClosureModel *M, double h, double q0, double q1,
                                             double hp, double q0p, double q1p, double hm, double q0m, double q1m,
                                             float &r0, float &r1)
{
    const double f[kMlpIn] = {h, q0, q1, hp - h, q0p - q0, q1p - q1, h - hm, q0 - q0m, q1 - q1m};
    float x[kMlpIn];
    bool inside = true;
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) {
        inside &= (f[i] >= M->box_lo[i]) & (f[i] <= M->box_hi[i]);
        x[i] = ((float)f[i] - M->mu[i]) * M->inv_sigma[i];
    }
    float y[kMlpOut];
    mlp_infer(P, x, y);
    r0 = inside ? y[0] * M->out_scale[0] : 0.0f;
    r1 = inside ? y[1] * M->out_scale[1] : 0.0f;
    return inside;
}

}  // namespace sme

namespace sme {
// the matrix-core kernel loads 8- and 16-byte operand slices of these arrays
static_assert(offsetof(ClosureModel, h) % 16 == 0 && offsetof(ClosureFp16, w2) % 16 == 0 &&
                  offsetof(ClosureFp16, w3) % 16 == 0 && sizeof(ClosureFp16::w1[0]) % 16 == 0,
              "FP16 operand arrays must be 16-byte aligned");
}  // namespace sme
