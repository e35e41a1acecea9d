// k_closure.hip -- closure rates of every cell from the current level-1 state.
//
// Runs before each level-1 step that has a learned closure attached.  One
// lane per cell and direction: it forms the nine features (the cell's depth
// and normal momenta q_0, q_1 and their differences to the two neighbours
// along that direction, boundary ghosts as in the step), evaluates the network
// and stores the two correction rates as FP32 float2 at [dir * stride + cell].
// A direction whose features leave the training box gets zero rates and is
// counted.
//
// Two evaluations of the network:
//   FP32   one lane per sample, parameters staged in LDS, FP32 FMA chains;
//   FP16   matrix cores: a wave evaluates 64 samples as four 16-sample tiles,
//          every layer one or two v_mfma_f32_16x16x{16,32}_f16 per 16 units
//          (FP16 operands, FP32 accumulation).  Result lane layout of a
//          16x16 tile: lane l holds rows 4 (l / 16) + {0..3} of column l % 16;
//          operand lanes hold row (A) or column (B) l % 16 and the k-slice
//          [K/4 (l / 16), K/4 (l / 16 + 1)).  Hidden units are rows, samples
//          columns, so the activations of one layer are already the B operand
//          of the next (the folded weights carry the matching column order).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sme_step_common.h"

namespace sme {

using namespace detail;

namespace {

// (h, q_0, q_1) normal to the axis of the neighbour at offset (di, dj) of cell
// (i, j); blk = field index of q_0 of the momenta normal to that axis
__device__ __forceinline__ void nb_normal(const StepArgs &a, int i, int j, int di, int dj, int blk, double &h,
                                          double &q0, double &q1)
{
    bool mx = false, my = false;
    const int ii = di ? ghost_index(i + di, a.nx, a.bc[0], a.bc[1], mx) : i;
    const int jj = dj ? ghost_index(j + dj, a.ny, a.bc[2], a.bc[3], my) : j;
    const int64_t cell = (int64_t)jj * a.nx + ii;
    const double s = (mx || my) ? -1.0 : 1.0;  // a wall mirrors the normal momenta
    h = a.q[cell];
    q0 = s * a.q[(blk + 0) * a.stride + cell];
    q1 = s * a.q[(blk + 1) * a.stride + cell];
}

// grid = nblk blocks per direction; blocks [0, nblk) do x, [nblk, 2 nblk) do y
__global__ __launch_bounds__(kBlock) void k_closure_rates_valu(StepArgs a, unsigned nblk)
{
    if (!(step_dt(a) > 0.0)) return;  // a step past the end time reads no rates
    __shared__ float P[kMlpParams];
    mlp_stage(a.closure->params, P);
    const int dir = blockIdx.x >= nblk ? 1 : 0;
    const int64_t cell = (int64_t)(blockIdx.x - dir * nblk) * kBlock + threadIdx.x;
    float2 *rates = reinterpret_cast<float2 *>(const_cast<float *>(a.rates)) + dir * a.stride;
    unsigned out = 0;
    if (cell < a.ncells) {
        float2 r = make_float2(0.0f, 0.0f);
        {
            const int i = (int)(cell % a.nx), j = (int)(cell / a.nx);
            const int blk = dir ? 3 : 1;  // level 1: fields h, qx_0, qx_1, qy_0, qy_1
            const double h = a.q[cell];
            const double q0 = a.q[blk * a.stride + cell], q1 = a.q[(blk + 1) * a.stride + cell];
            double hp, q0p, q1p, hm, q0m, q1m;
            nb_normal(a, i, j, dir ? 0 : 1, dir, blk, hp, q0p, q1p);
            nb_normal(a, i, j, dir ? 0 : -1, -dir, blk, hm, q0m, q1m);
            out = closure_rate(P, a.closure, h, q0, q1, hp, q0p, q1p, hm, q0m, q1m, r.x, r.y) ? 0u : 1u;
        }
        rates[cell] = r;
    }
    publish_count(a.oor, out);
}


typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

// raw features of sample (cell, dir) and whether they lie in the training box;
// x = normalised features (FP32, same arithmetic as the FP32 variant)
__device__ __forceinline__ bool sample_features(const StepArgs &a, int i, int j, int dir, float *x)
{
    const ClosureModel *M = a.closure;
    const int64_t cell = (int64_t)j * a.nx + i;
    const int blk = dir ? 3 : 1;
    const double h = a.q[cell];
    const double q0 = a.q[blk * a.stride + cell], q1 = a.q[(blk + 1) * a.stride + cell];
    double hp, q0p, q1p, hm, q0m, q1m;
    nb_normal(a, i, j, dir ? 0 : 1, dir, blk, hp, q0p, q1p);
    nb_normal(a, i, j, dir ? 0 : -1, -dir, blk, hm, q0m, q1m);
    const double f[kMlpIn] = {h, q0, q1, hp - h, q0p - q0, q1p - q1, h - hm, q0 - q0m, q1 - q1m};
    bool inside = true;
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) {
        inside &= (f[k] >= M->box_lo[k]) & (f[k] <= M->box_hi[k]);
        x[k] = ((float)f[k] - M->mu[k]) * M->inv_sigma[k];
    }
    return inside;
}

// tanh(u / kappa) = 1 - 2 / (1 + 2^u), rounded to FP16 (exact limits +-1 for |u| -> inf)
__device__ __forceinline__ _Float16 act(float u)
{
    return (_Float16)fmaf(-2.0f, __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(u)), 1.0f);
}

// activations of the result tiles 2 kc and 2 kc + 1 as the B operand of chunk kc
__device__ __forceinline__ half8 act_pair(const float4v &lo, const float4v &hi)
{
    half8 s;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        s[e] = act(lo[e]);
        s[4 + e] = act(hi[e]);
    }
    return s;
}

constexpr int kGroup = 64;  // samples per wave and pass

// A group is 64 consecutive cells of one row and one direction: group k has
// direction k / per_dir, row r / chunks and columns 64 (r % chunks) + lane
// with r = k % per_dir and per_dir = rows x chunks, so row and first column
// are the same for the whole wave.  Waves stride over the groups.
__global__ __launch_bounds__(kBlock) void k_closure_rates_mfma(StepArgs a, int chunks, int per_dir, int ngroups)
{
    __shared__ __attribute__((aligned(16))) _Float16 X[kBlock / kWave][kGroup][kMlpInPad];
    if (!(step_dt(a) > 0.0)) return;  // a step past the end time reads no rates
    const ClosureFp16 &H = a.closure->h;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    // second-layer operand slices, staged once per block in the order the
    // lanes read them (16 contiguous bytes per lane: no bank conflicts); kept
    // out of registers, which leaves room for three waves per SIMD
    __shared__ __attribute__((aligned(16))) half8 W2s[4][2][kWave];
    for (int idx = threadIdx.x; idx < 4 * 2 * kWave; idx += kBlock) {
        const int mt = idx / (2 * kWave), kc = (idx / kWave) % 2, l = idx % kWave;
        W2s[mt][kc][l] = *reinterpret_cast<const half8 *>(&H.w2[16 * mt + (l & 15)][32 * kc + 8 * (l >> 4)]);
    }
    __syncthreads();
    half4 w1[4];
    half8 w3[2];
    float4v c1[4], c2[4], c3;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        w1[mt] = *reinterpret_cast<const half4 *>(&H.w1[16 * mt + col][4 * g]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            c1[mt][r] = H.c1[16 * mt + 4 * g + r];
            c2[mt][r] = H.c2[16 * mt + 4 * g + r];
        }
    }
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) w3[kc] = *reinterpret_cast<const half8 *>(&H.w3[col][32 * kc + 8 * g]);
#pragma unroll
    for (int r = 0; r < 4; ++r) c3[r] = g == 0 ? H.c3[r] : 0.0f;
    const float os0 = a.closure->out_scale[0], os1 = a.closure->out_scale[1];
    const int nwaves = (int)gridDim.x * (kBlock / kWave);
    unsigned out = 0;
    for (int grp = (int)blockIdx.x * (kBlock / kWave) + wv; grp < ngroups; grp += nwaves) {
        const int dir = grp >= per_dir ? 1 : 0;
        const int r = grp - dir * per_dir;
        const int j = r / chunks;
        const int i0 = (r - j * chunks) * kGroup;
        float2 *rates = reinterpret_cast<float2 *>(const_cast<float *>(a.rates)) + dir * a.stride +
                        ((int64_t)j * a.nx + i0);
        const int ncol = min(kGroup, a.nx - i0);  // columns of this group inside the grid
        // features: one sample per lane
        {
            float x[kMlpIn];
#pragma unroll
            for (int k = 0; k < kMlpIn; ++k) x[k] = 0.0f;
            bool inside = false;
            if (lane < ncol) {
                inside = sample_features(a, i0 + lane, j, dir, x);
                out += inside ? 0u : 1u;
            }
            half8 lo, hi;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                lo[k] = (_Float16)x[k];
                hi[k] = k == 0 ? (_Float16)x[8] : (_Float16)0.0f;
            }
            *reinterpret_cast<half8 *>(&X[wv][lane][0]) = lo;
            *reinterpret_cast<half8 *>(&X[wv][lane][8]) = hi;
            // keep: the in-box flag of every sample of the group
            const unsigned long long inmask = __ballot(inside);
            __builtin_amdgcn_wave_barrier();
            // two tiles at a time, interleaved layer by layer: the matrix
            // cores work on one tile while the activations of the other run
#pragma unroll 1
            for (int t = 0; t < kGroup / 16; t += 2) {
                const half4 xa = *reinterpret_cast<const half4 *>(&X[wv][16 * t + col][4 * g]);
                const half4 xb = *reinterpret_cast<const half4 *>(&X[wv][16 * t + 16 + col][4 * g]);
                float4v ua[4], ub[4], va[4], vb[4];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) ua[mt] = __builtin_amdgcn_mfma_f32_16x16x16f16(w1[mt], xa, c1[mt], 0, 0, 0);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) ub[mt] = __builtin_amdgcn_mfma_f32_16x16x16f16(w1[mt], xb, c1[mt], 0, 0, 0);
                const half8 sa0 = act_pair(ua[0], ua[1]), sa1 = act_pair(ua[2], ua[3]);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    va[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(W2s[mt][0][lane], sa0, c2[mt], 0, 0, 0);
                    va[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(W2s[mt][1][lane], sa1, va[mt], 0, 0, 0);
                }
                const half8 sb0 = act_pair(ub[0], ub[1]), sb1 = act_pair(ub[2], ub[3]);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    vb[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(W2s[mt][0][lane], sb0, c2[mt], 0, 0, 0);
                    vb[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(W2s[mt][1][lane], sb1, vb[mt], 0, 0, 0);
                }
                const half8 ta0 = act_pair(va[0], va[1]), ta1 = act_pair(va[2], va[3]);
                float4v ya = __builtin_amdgcn_mfma_f32_16x16x32_f16(w3[0], ta0, c3, 0, 0, 0);
                ya = __builtin_amdgcn_mfma_f32_16x16x32_f16(w3[1], ta1, ya, 0, 0, 0);
                const half8 tb0 = act_pair(vb[0], vb[1]), tb1 = act_pair(vb[2], vb[3]);
                float4v yb = __builtin_amdgcn_mfma_f32_16x16x32_f16(w3[0], tb0, c3, 0, 0, 0);
                yb = __builtin_amdgcn_mfma_f32_16x16x32_f16(w3[1], tb1, yb, 0, 0, 0);
                if (g == 0) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const float4v &y = h ? yb : ya;
                        const int smp = 16 * (t + h) + col;
                        if (smp < ncol) {
                            const bool ok = ((inmask >> smp) & 1ull) != 0;
                            rates[smp] = ok ? make_float2(os0 * y[0], os1 * y[1]) : make_float2(0.0f, 0.0f);
                        }
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    publish_count(a.oor, out);
}

}  // namespace

hipError_t launch_closure_rates(const StepArgs &a, int dims, int mode, int cus, hipStream_t s)
{
    if (dims < 1 || dims > 2) return hipErrorInvalidValue;
    if (mode == kClosureFp16Mfma) {
        const int64_t chunks = (a.nx + kGroup - 1) / kGroup;
        const int64_t per_dir = chunks * a.ny;
        const int64_t ngroups = per_dir * dims;
        if (ngroups > INT32_MAX) return hipErrorInvalidValue;
        // enough blocks to fill every SIMD several times; waves stride over the rest
        const int64_t want = (ngroups + kBlock / kWave - 1) / (kBlock / kWave);
        const unsigned grid = (unsigned)std::min<int64_t>(want, (int64_t)cus * 8);
        hipLaunchKernelGGL(k_closure_rates_mfma, dim3(grid), dim3(kBlock), 0, s, a, (int)chunks, (int)per_dir,
                           (int)ngroups);
        return hipGetLastError();
    }
    if (mode != kClosureFp32) return hipErrorInvalidValue;
    const unsigned nblk = blocks_for(a.ncells);
    const unsigned dirs = (unsigned)dims;
    hipLaunchKernelGGL(k_closure_rates_valu, dim3(nblk * dirs), dim3(kBlock), 0, s, a, nblk);
    return hipGetLastError();
}

}  // namespace sme
