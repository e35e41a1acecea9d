// sme_kernels.h -- launch interface between the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sme_device.h"
#include "sme_mlp.h"

namespace sme {

// Per-step bookkeeping on the device.  Three slots rotate: step n reads slot a
// (time, CFL ratio of Q^n), writes slot b (time and CFL ratio of Q^{n+1}) and
// clears slot c for step n + 1.  The ratio words hold max_i r_i (r_i = sum_f
// |e_f| lam / (2 |V_i|)) as the bit pattern of a non-negative double, so an
// unsigned atomic max is an exact, order-independent maximum.
// The max CFL ratio of a state is reduced into kRatioWords words, one per
// compute die (block b publishes into word b % kRatioWords), each on its own
// 256-byte line, so the per-block atomics of a step spread over eight
// addresses instead of queueing on one; readers take the max of the words.
constexpr int kRatioWords = 8;
struct alignas(256) RatioWord {
    unsigned long long bits;    // bit pattern of a non-negative double
};

struct Slot {
    RatioWord r[kRatioWords];   // max CFL ratio of the state this slot describes
    unsigned long long lbits;   // max lam over cells and face normals
    double t;                   // simulated time of that state
    double dt;                  // step that produced it
    long long step;             // number of steps that advanced the state
};

// max CFL ratio held by a slot (host or device)
__host__ __device__ inline double slot_ratio(const Slot &s)
{
    unsigned long long m = 0;
    for (int w = 0; w < kRatioWords; ++w) m = s.r[w].bits > m ? s.r[w].bits : m;
    double d;
    __builtin_memcpy(&d, &m, sizeof d);
    return d;
}

struct ErrWord {
    unsigned int flag;          // 1 once a non-physical value was produced
    unsigned int pad;
    unsigned long long first_step;  // smallest step index that produced one
};

enum BcKind { BC_PERIODIC = 0, BC_EXTRAP = 1, BC_WALL = 2 };

struct StepArgs {
    const double *q;     // Q^n, SoA with `stride`
    double *qn;          // Q^{n+1}
    const double *b;
    int64_t stride;
    int64_t ncells;
    // structured / 1D
    int nx, ny;
    double idx, idy;     // 1/dx, 1/dy
    int bc[4];           // W, E, S, N
    int rows;            // rows per wave strip (structured 2D)
    // triangles (internal order)
    const int32_t *nbr;  // [3][stride]
    const double *fsx, *fsy;  // [3][stride] scaled outward normals n |e| of the faces
    const double *ivol;       // [stride] 1 / |V|
    // model
    double g, c_slip, nu, cfl;
    int implicit;        // friction step: 0 forward Euler, 1 backward Euler
    Quad quad;
    // time stepping
    double dt_fixed;     // > 0: fixed step
    double t_end;        // > 0: clamp simulated time
    Slot *slots;
    int sa, sb, sc;
    ErrWord *err;
    // second-order scheme: limited slopes [axis][nv][stride] (null = first order)
    const double *slopes;
    // learned closure (level 1 only; null = plain step)
    const ClosureModel *closure;
    const float *rates;       // float2 rates of (q_0, q_1) normal to x at [cell], normal to y at [stride + cell]
    unsigned long long *oor;  // cells whose features left the training range
};

// ---------------------------------------------------------------------------
// Batched ensemble: many structured grids advanced by one persistent launch.
constexpr int kBatchMaxLevel = 4;

struct BatchInst {
    int level;
    int nx, ny, rows;
    int bc[4];
    int64_t offset;   // element offset of field 0 of this grid in the state arenas
    int64_t stride;   // field stride of this grid (elements)
    int64_t boff;     // element offset of its bathymetry
    double idx, idy;  // 1/dx, 1/dy
};

struct BatchItem {
    int inst, sx, sy, pad;  // one wave's work: strip sx, band sy of grid inst
};

// The work counters of the three time slots lie this many words apart (one
// 256-byte line each).
constexpr int kWorkStride = 64;

struct BatchArgs {
    const double *q;
    double *qn;
    const double *b;
    const BatchInst *inst;
    const BatchItem *items;
    int nitems;
    Slot *slots;       // [n_inst][3]
    int sa, sb, sc;
    unsigned *work;    // [3 * kWorkStride]: next item of the step that reads slot s at work[s * kWorkStride]
    ErrWord *err;
    double g, c_slip, nu, cfl;
    int implicit;
    Quad quad;
};

hipError_t launch_batch_step(const BatchArgs &a, int grid, hipStream_t s);
int batch_waves_per_simd();  // resident waves per SIMD of the ensemble kernel

// host-side launchers; level is 0..8
hipError_t launch_step_1d(int level, const StepArgs &a, hipStream_t s);
// nsteps steps of a 1D grid by one workgroup with the state in LDS (no closure);
// the final state goes to dst; run_1d_lds_bytes is its dynamic LDS size
size_t run_1d_lds_bytes(int level, int nx);
hipError_t launch_run_1d_lds(int level, const StepArgs &a, int nsteps, double *dst, hipStream_t s);
hipError_t launch_step_2d(int level, const StepArgs &a, hipStream_t s);
int step_2d_waves_per_simd(int level);  // resident waves per SIMD of the structured step kernel
hipError_t launch_step_tri(int level, const StepArgs &a, hipStream_t s);
// second-order step on 1D (dim 1) and structured (dim 2) grids: slopes of a.q
// into `slopes`, then stage 1 (a.qn = a.q + dt L) or stage 2 (a.qn = a.qn / 2 +
// (a.q + dt L(a.q)) / 2, friction, CFL ratio) of the two-stage Runge-Kutta step
hipError_t launch_recon2(int level, int dim, const StepArgs &a, double *slopes, hipStream_t s);
hipError_t launch_flux2(int level, int dim, int stage, const StepArgs &a, const double *slopes, hipStream_t s);
// the same stages on structured grids with the reconstruction fused in (no
// slopes array): one wave per band of a.rows rows, as launch_step_2d; levels
// 0 .. kStage2BandMaxLevel (above, the row's live set no longer fits the
// registers of one wave)
constexpr int kStage2BandMaxLevel = 6;
hipError_t launch_stage2_band(int level, int stage, const StepArgs &a, hipStream_t s);
hipError_t launch_eig(int dim, int kind, int level, const StepArgs &a, hipStream_t s);
hipError_t launch_slots_reset(Slot *slots, ErrWord *err, int sa, hipStream_t s);  // err may be null
// closure network training and samples (k_mlp.hip)
hipError_t launch_mlp_forward(const float *params, const float *x, int64_t B, const MlpScale &sc, float *y,
                              hipStream_t s);
int mlp_grad_blocks(int64_t B);
hipError_t launch_mlp_grad(const float *params, const float *x, const float *t, const int64_t *idx, int64_t B,
                           const MlpScale &sc, float *partial, float *partial_loss, float *grad, float *loss,
                           hipStream_t s);
// feature statistics: out = [sums or squared-deviation sums of 11 columns, 9 minima, 9 maxima]
int mlp_stat_width();
int mlp_stat_blocks();
hipError_t launch_mlp_stats(const float *feat, const float *targ, int64_t n, const double *mean, double *partial,
                            double *out, hipStream_t s);
hipError_t launch_mlp_adam(float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                           float c1, float c2, hipStream_t s);
hipError_t launch_closure_samples(const double *q8, int64_t s8, const double *q8n, int64_t s8n, const double *q1,
                                  int64_t s1, int64_t n, double dt, const int64_t *cells, int64_t ns, float *feat,
                                  float *targ, hipStream_t s);
// closure rates of every cell from the current state (k_closure.hip)
// dims = 1 (1D grid) or 2 (structured grid); mode = ClosurePrecision; cus = compute units
hipError_t launch_closure_rates(const StepArgs &a, int dims, int mode, int cus, hipStream_t s);
hipError_t launch_permute(const double *src, int64_t sstride, double *dst, int64_t dstride,
                          const int64_t *map, int64_t ncells, int nf, hipStream_t s);

}  // namespace sme
